// Dense products of tall panel-major blocks, for the block conjugate gradient
// of the interpolation: Gram matrices A^T B (float32 entries, float64 sums)
// and right products by a small float64 matrix (float64 sums, or float32
// sums on the float32 matrix cores under CSC_TUNE_BLOCK_PRODUCT).
//
// Both run on the float64 matrix cores (v_mfma_f64_16x16x4f64: a 16 x 16
// float64 tile += a 16 x 4 by 4 x 16 product, one element of each operand per
// lane).  Float32 entries are widened exactly, so every product is exact and
// only the float64 sums round: the orthonormalisation and the step sizes of
// the block CG keep float64 accuracy.  Operand lanes: lane l supplies row
// (l mod 16), inner index (l / 16) of the left operand and inner index
// (l / 16), column (l mod 16) of the right one; the result tile leaves lane l
// holding rows (l / 16) + 4 v, v = 0..3, of column (l mod 16).
#include <algorithm>
#include <type_traits>

#include "device.hpp"

namespace csc {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kGT = 128;  // Gram output tile per workgroup (4 waves of 64 x 64)
constexpr int kMR = 128;  // block product: rows per workgroup (2 waves of 64)
constexpr int kMC = 128;  // block product: columns per workgroup (2 waves of 64)
static_assert(kGT == kBlockTile && kMC == kBlockTile, "column tiles of the tile masks");

// Offset of column c within row 0 of a panel-major block: element (i, c) is at
// col_base(L, c) + i * pw.
__device__ inline size_t col_base(const Layout& L, int c) {
  const int pan = c / L.pw;
  return (size_t)pan * L.panel_elems() + (size_t)(c - pan * L.pw);
}

__device__ inline v4d mfma64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Columns c..c+3 (c a multiple of 4) of row i of a panel-major block, in two
// halves so that the load is issued without a branch and its wait lands where
// the value is used: cols4_load reads the four columns (or, when none of them
// is live, a stand-in at the block's start) and returns how many are live,
// cols4_mask zeroes the rest.  c < kvalid <= stored width keeps the four
// inside one panel (panel widths are multiples of 4).
__device__ inline float4 cols4_load(const Layout& L, const float* X, int i, int c, int kvalid,
                                    bool row_ok, int& live) {
  const bool ok = row_ok && c < kvalid;
  live = ok ? min(4, kvalid - c) : 0;
  return *reinterpret_cast<const float4*>(X + (ok ? col_base(L, c) + (size_t)i * L.pw : 0));
}

__device__ inline float4 cols4_mask(float4 v, int live) {
  v.x = live > 0 ? v.x : 0.f;
  v.y = live > 1 ? v.y : 0.f;
  v.z = live > 2 ? v.z : 0.f;
  v.w = live > 3 ? v.w : 0.f;
  return v;
}

constexpr int kGS = 32;         // Gram: rows per LDS stage
constexpr int kGLD = kGT + 16;  // LDS row stride (floats): the 4 rows a wave reads at once
                                // fall on disjoint banks

// part[chunk][r][c] = sum over the chunk's rows i of A[i, r] * B[i, c] for the
// 128 x 128 output tile (ti, tj); lower: only the tiles ti >= tj (a Gram whose
// upper block triangle is taken from the lower one).  The workgroup stages 32 rows of both
// column ranges in LDS (double-buffered, the next stage's global loads in
// flight during the products); wave w takes the 64 x 64 quarter
// (w / 2, w mod 2), four rows per matrix-core step.
__global__ __launch_bounds__(256) void k_gram(Layout L, const float* A, const float* B, int ka,
                                              int kb, int rows_per_chunk, int tiles_b,
                                              int rows_pad, bool lower, uint64_t amask,
                                              uint64_t bmask, double* part) {
  __shared__ float As[2][kGS][kGLD];
  __shared__ float Bs[2][kGS][kGLD];
  int ti, tj;
  if (lower) {  // the tiles on and below the diagonal only: (0,0), (1,0), (1,1), (2,0), ...
    ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= (int)blockIdx.x) ++ti;
    tj = (int)blockIdx.x - ti * (ti + 1) / 2;
  } else {
    ti = blockIdx.x / tiles_b;
    tj = blockIdx.x - ti * tiles_b;
  }
  if (!((amask >> ti) & 1) || !((bmask >> tj) & 1)) return;  // a tile nobody reads
  const int chunk = blockIdx.y;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(L.n, r0 + rows_per_chunk);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int wa = (wave >> 1) * 64, wb = (wave & 1) * 64;
  const int ca0 = ti * kGT, cb0 = tj * kGT;
  float4 ra[4], rb[4];
  int la[4], lb[4];
  auto fetch = [&](int base) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = t + 256 * u, row = f >> 5, c = (f & 31) * 4, i = base + row;
      ra[u] = cols4_load(L, A, i, ca0 + c, ka, i < r1, la[u]);
      rb[u] = cols4_load(L, B, i, cb0 + c, kb, i < r1, lb[u]);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = t + 256 * u, row = f >> 5, c = (f & 31) * 4;
      *reinterpret_cast<float4*>(&As[buf][row][c]) = cols4_mask(ra[u], la[u]);
      *reinterpret_cast<float4*>(&Bs[buf][row][c]) = cols4_mask(rb[u], lb[u]);
    }
  };
  v4d acc[4][4];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int h = 0; h < 4; ++h) acc[g][h] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nst = (r1 - r0 + kGS - 1) / kGS;
  fetch(r0);
  stash(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) fetch(r0 + (st + 1) * kGS);
#pragma unroll 2
    for (int ks = 0; ks < kGS / 4; ++ks) {
      double a[4], b[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        a[g] = (double)As[buf][4 * ks + q][wa + 16 * g + c16];
        b[g] = (double)Bs[buf][4 * ks + q][wb + 16 * g + c16];
      }
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int h = 0; h < 4; ++h) acc[g][h] = mfma64(a[g], b[h], acc[g][h]);
    }
    if (st + 1 < nst) stash(buf ^ 1);
    __syncthreads();
  }
  const int ldp = tiles_b * kGT;
  double* out = part + (size_t)chunk * rows_pad * ldp;
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[(size_t)(ca0 + wa + 16 * g + q + 4 * v) * ldp + cb0 + wb + 16 * h + c16] =
            acc[g][h][v];
}

// k_gram for ka <= 16 (a search block of at most 16 live columns): only the
// first 16 rows of each output tile hold anything, so each wave takes a
// 16 x 32 strip of the tile's columns (wave w: columns 32 w .. 32 w + 31)
// instead of a 64 x 64 quarter, an eighth of the matrix-core work.  Stages,
// steps and lanes are k_gram's: every entry takes the same products in the
// same order, so the partials (and the Gram) are k_gram's bit for bit.
constexpr int kThinA = 16;
__global__ __launch_bounds__(256) void k_gram_thin(Layout L, const float* A, const float* B,
                                                   int ka, int kb, int rows_per_chunk,
                                                   int rows_pad, uint64_t bmask, double* part) {
  __shared__ float As[2][kGS][kThinA + 4];
  __shared__ float Bs[2][kGS][kGLD];
  const int tj = blockIdx.x, chunk = blockIdx.y;
  if (!((bmask >> tj) & 1)) return;  // a tile nobody reads
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(L.n, r0 + rows_per_chunk);
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int wb = wave * 32;
  const int cb0 = tj * kGT;
  float4 ra = make_float4(0.f, 0.f, 0.f, 0.f), rb[4];
  int la = 0, lb[4];
  auto fetch = [&](int base) {
    if (t < kGS * kThinA / 4) {  // 32 rows x 16 columns of A: one float4 per thread
      const int row = t >> 2, c = (t & 3) * 4, i = base + row;
      ra = cols4_load(L, A, i, c, ka, i < r1, la);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = t + 256 * u, row = f >> 5, c = (f & 31) * 4, i = base + row;
      rb[u] = cols4_load(L, B, i, cb0 + c, kb, i < r1, lb[u]);
    }
  };
  auto stash = [&](int buf) {
    if (t < kGS * kThinA / 4)
      *reinterpret_cast<float4*>(&As[buf][t >> 2][(t & 3) * 4]) = cols4_mask(ra, la);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int f = t + 256 * u, row = f >> 5, c = (f & 31) * 4;
      *reinterpret_cast<float4*>(&Bs[buf][row][c]) = cols4_mask(rb[u], lb[u]);
    }
  };
  v4d acc[2];
#pragma unroll
  for (int h = 0; h < 2; ++h) acc[h] = v4d{0.0, 0.0, 0.0, 0.0};
  const int nst = (r1 - r0 + kGS - 1) / kGS;
  fetch(r0);
  stash(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst) fetch(r0 + (st + 1) * kGS);
#pragma unroll 2
    for (int ks = 0; ks < kGS / 4; ++ks) {
      const double a = (double)As[buf][4 * ks + q][c16];
      double b[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) b[h] = (double)Bs[buf][4 * ks + q][wb + 16 * h + c16];
#pragma unroll
      for (int h = 0; h < 2; ++h) acc[h] = mfma64(a, b[h], acc[h]);
    }
    if (st + 1 < nst) stash(buf ^ 1);
    __syncthreads();
  }
  const int ldp = gridDim.x * kGT;
  double* out = part + (size_t)chunk * rows_pad * ldp;
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      out[(size_t)(q + 4 * v) * ldp + cb0 + wb + 16 * h + c16] = acc[h][v];
}

// G[i * ldg + j] = sum over chunks of the partial tiles: 16 entries per
// workgroup, 16 threads per entry summing chunks s, s + 16, ... in order,
// then the 16 slices in order.  lower: an entry of a tile above the diagonal
// is its mirror's sum (i and j swapped), bit for bit.
__global__ __launch_bounds__(256) void k_gram_reduce(const double* part, int chunks, int rows_pad,
                                                     int cols_pad, int ka, int kb, bool lower,
                                                     double* G, int ldg) {
  __shared__ double sh[16][17];
  const int slice = threadIdx.x >> 4, el = threadIdx.x & 15;
  const int e = blockIdx.x * 16 + el;
  const bool ok = e < ka * kb;
  const int i = ok ? e / kb : 0, j = ok ? e - i * kb : 0;
  const bool mirror = lower && i / kGT < j / kGT;
  const int pi = mirror ? j : i, pj = mirror ? i : j;
  double s = 0.0;
  if (ok)
    for (int c = slice; c < chunks; c += 16) s += part[((size_t)c * rows_pad + pi) * cols_pad + pj];
  sh[slice][el] = s;
  __syncthreads();
  if (slice == 0 && ok) {
    double t = 0.0;
#pragma unroll
    for (int r = 0; r < 16; ++r) t += sh[r][el];
    G[(size_t)i * ldg + j] = t;
  }
}

// Block product stages: 16 inner columns per LDS stage keep a workgroup at
// 57 KB of LDS, so two workgroups share a CU (at 32 columns, 108 KB, one did,
// and the product ran at half the matrix-core rate).
constexpr int kBS = 16;          // inner columns per LDS stage
constexpr int kXLD = kBS + 4;    // In1 tile stride (floats): a wave's 64 reads hit 64 banks
constexpr int kSLD = kMC + 16;   // S tile stride (doubles)
constexpr int kXV = kBS / 4;     // float4 per staged In1 row
constexpr int kXU = kMR * kXV / 256;  // staged float4 of In1 per thread
constexpr int kSU = kBS * kMC / 256;  // staged doubles of S per thread
static_assert(kXU >= 1 && kSU >= 1 && kSU <= 32, "block product staging shape");

// Out[i, j] = c0 * In0[i, j] + sum_{l < kin} In1[i, l] * S[l * lds + j] for
// every stored column j of the layout (S is zero beyond its live columns, so
// padding columns stay c0 * In0).  F32 = false: float64 sums of the exact
// products of float32 entries and float64 S, on the float64 matrix cores,
// rounded once to float32; F32 = true: S rounded to float32 and float32 sums
// on the float32 matrix cores (v_mfma_f32_16x16x4f32, whose result tile leaves
// lane l holding rows 4 (l / 16) + v, v = 0..3, of column l mod 16).
// Workgroup: 128 rows x 128 columns; the inner dimension is staged 16 at a
// time in LDS (In1 rows and S rows, double-buffered); wave w takes the
// 64 x 64 quarter (w / 2, w mod 2).  Out may be In0 (each element is read and
// written by the same lane), never In1.
template <bool F32>
__global__ __launch_bounds__(256, 2) void k_block_mul(Layout L, float c0, const float* In0,
                                                   const float* In1, const double* S, int kin,
                                                   int kout, int lds, uint64_t cmask, float* Out) {
  if (!((cmask >> blockIdx.y) & 1)) return;  // columns nobody reads
  typedef typename std::conditional<F32, float, double>::type sc_t;
  typedef typename std::conditional<F32, v4f, v4d>::type acc_t;
  __shared__ float Xs[2][kMR][kXLD];
  __shared__ sc_t Ss[2][kBS][kSLD];
  const int W = L.np * L.pw;
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int q = lane >> 4, c16 = lane & 15;
  const int bi0 = blockIdx.x * kMR, bj0 = blockIdx.y * kMC;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  float4 rx[kXU];
  int lx[kXU];
  double rs[kSU];
  unsigned sok = 0;  // bit u: element u of the S stage is live
  auto fetch = [&](int l0) {
#pragma unroll
    for (int u = 0; u < kXU; ++u) {
      const int f = t + 256 * u, row = f / kXV, c = (f % kXV) * 4, i = bi0 + row;
      rx[u] = cols4_load(L, In1, i, l0 + c, kin, i < L.n, lx[u]);
    }
    sok = 0;
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const int f = t + 256 * u, r = f >> 7, c = f & 127, l = l0 + r, j = bj0 + c;
      const bool ok = l < kin && j < kout;
      sok |= (ok ? 1u : 0u) << u;
      rs[u] = S[ok ? (size_t)l * lds + j : 0];
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int u = 0; u < kXU; ++u) {
      const int f = t + 256 * u, row = f / kXV, c = (f % kXV) * 4;
      *reinterpret_cast<float4*>(&Xs[buf][row][c]) = cols4_mask(rx[u], lx[u]);
    }
#pragma unroll
    for (int u = 0; u < kSU; ++u) {
      const int f = t + 256 * u;
      Ss[buf][f >> 7][f & 127] = ((sok >> u) & 1u) ? (sc_t)rs[u] : (sc_t)0;
    }
  };
  acc_t acc[4][4];
#pragma unroll
  for (int g = 0; g < 4; ++g)
#pragma unroll
    for (int h = 0; h < 4; ++h) acc[g][h] = acc_t{0, 0, 0, 0};
  const int nst = (kin + kBS - 1) / kBS;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1, l0 = st * kBS;
    if (st + 1 < nst) fetch(l0 + kBS);
    const int ksn = min(kBS, kin - l0 + 3) / 4;  // steps holding live inner columns
    for (int ks = 0; ks < ksn; ++ks) {
      sc_t a[4], b[4];
#pragma unroll
      for (int g = 0; g < 4; ++g) a[g] = (sc_t)Xs[buf][wr + 16 * g + c16][4 * ks + q];
#pragma unroll
      for (int h = 0; h < 4; ++h) b[h] = Ss[buf][4 * ks + q][wc + 16 * h + c16];
#pragma unroll
      for (int g = 0; g < 4; ++g)
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          if constexpr (F32)
            acc[g][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[g], b[h], acc[g][h], 0, 0, 0);
          else
            acc[g][h] = mfma64(a[g], b[h], acc[g][h]);
        }
    }
    if (st + 1 < nst) stash(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    const int j = bj0 + wc + 16 * h + c16;
    if (j >= W) continue;
    const size_t cbj = col_base(L, j);
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = bi0 + wr + 16 * g + (F32 ? 4 * q + v : q + 4 * v);
        if (i >= L.n) continue;
        const size_t o = cbj + (size_t)i * L.pw;
        if constexpr (F32) {
          const float base = c0 != 0.f ? c0 * In0[o] : 0.f;
          Out[o] = base + acc[g][h][v];
        } else {
          const double base = c0 != 0.f ? (double)c0 * (double)In0[o] : 0.0;
          Out[o] = (float)(base + acc[g][h][v]);
        }
      }
  }
}

// Z = D^-1 R for the diagonal D_ii = mask_i + gamma (the Jacobi
// preconditioner of the interpolation system): every stored element, four
// columns of one row per thread (pw is a multiple of 4).
__global__ void k_jacobi(Layout L, const float* R, const float* mask, float gamma, float* Z) {
  const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t e = q * 4;
  if (e >= L.elems()) return;
  const int row = (int)((e % L.panel_elems()) / (size_t)L.pw);
  const float d = mask[row] + gamma;
  const float4 r = *reinterpret_cast<const float4*>(R + e);
  *reinterpret_cast<float4*>(Z + e) = make_float4(r.x / d, r.y / d, r.z / d, r.w / d);
}

}  // namespace

hipError_t launch_jacobi(const Layout& L, const float* R, const float* mask, float gamma, float* Z,
                         hipStream_t s) {
  const size_t q = L.elems() / 4;
  if (q == 0) return hipSuccess;
  hipLaunchKernelGGL(k_jacobi, dim3((unsigned)((q + 255) / 256)), dim3(256), 0, s, L, R, mask,
                     gamma, Z);
  return hipGetLastError();
}

GramPlan gram_plan(const Layout& L, int ka, int kb, bool lower) {
  GramPlan g;
  g.tiles_a = (ka + kGT - 1) / kGT;
  g.tiles_b = (kb + kGT - 1) / kGT;
  g.lower = lower && ka == kb;
  g.tiles = g.lower ? g.tiles_a * (g.tiles_a + 1) / 2 : g.tiles_a * g.tiles_b;
  const int tiles = g.tiles;
  // about one workgroup per CU, chunks of at least 512 rows
  int chunks = std::max(1, 256 / tiles);
  chunks = std::min(chunks, std::max(1, L.n / 512));
  int rows = (L.n + chunks - 1) / chunks;
  rows = (rows + 3) / 4 * 4;
  g.rows_per_chunk = rows;
  g.chunks = (L.n + rows - 1) / rows;
  return g;
}

size_t gram_part_elems(const Layout& L, int kmax) {
  size_t m = 0;
  for (int ka = kGT; ka < kmax + kGT; ka += kGT)
    for (int kb = kGT; kb < kmax + kGT; kb += kGT)
      for (const bool lower : {false, true}) {
        const GramPlan g = gram_plan(L, std::min(ka, kmax), std::min(kb, kmax), lower);
        m = std::max(m, (size_t)g.chunks * g.tiles_a * kGT * g.tiles_b * kGT);
      }
  return m;
}

hipError_t launch_gram(const Layout& L, const float* A, const float* B, int ka, int kb,
                       double* part, double* G, int ldg, hipStream_t s, bool lower,
                       uint64_t amask, uint64_t bmask) {
  const GramPlan g = gram_plan(L, ka, kb, lower);
  if (g.tiles_a > 64) amask = ~0ull;
  if (g.tiles_b > 64) bmask = ~0ull;
  if (ka <= kThinA)  // one tile row: a 16-row strip of each tile (tiles = tiles_b)
    hipLaunchKernelGGL(k_gram_thin, dim3((unsigned)g.tiles_b, (unsigned)g.chunks), dim3(256), 0, s,
                       L, A, B, ka, kb, g.rows_per_chunk, g.tiles_a * kGT,
                       (amask & 1) ? bmask : 0ull, part);
  else
    hipLaunchKernelGGL(k_gram, dim3((unsigned)g.tiles, (unsigned)g.chunks), dim3(256), 0, s, L, A,
                       B, ka, kb, g.rows_per_chunk, g.tiles_b, g.tiles_a * kGT, g.lower, amask,
                       bmask, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = ka * kb;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, s, part,
                     g.chunks, g.tiles_a * kGT, g.tiles_b * kGT, ka, kb, g.lower, G, ldg);
  return hipGetLastError();
}

hipError_t launch_block_mul(const Layout& L, float c0, const float* In0, const float* In1,
                            const double* S, int kin, int kout, int lds, float* Out,
                            hipStream_t s, bool f32, uint64_t cmask) {
  const int W = L.np * L.pw;
  const dim3 grid((unsigned)((L.n + kMR - 1) / kMR), (unsigned)((W + kMC - 1) / kMC));
  if (grid.y > 64) cmask = ~0ull;
  if (f32 || block_product_f32())
    hipLaunchKernelGGL(k_block_mul<true>, grid, dim3(256), 0, s, L, c0, In0, In1, S, kin, kout,
                       lds, cmask, Out);
  else
    hipLaunchKernelGGL(k_block_mul<false>, grid, dim3(256), 0, s, L, c0, In0, In1, S, kin, kout,
                       lds, cmask, Out);
  return hipGetLastError();
}

}  // namespace csc
