// Dense products of tall panel-major blocks, for the block conjugate gradient
// of the interpolation: Gram matrices A^T B (float32 entries, float64 sums)
// and right products by a small float64 matrix.
//
// Both are memory-light next to a Chebyshev pass (k x k work per node for an
// N x k block, against p gathered steps), so they use plain float64 FMAs on
// LDS tiles rather than matrix cores: float64 accumulation keeps the
// orthonormalisation and the step sizes of the block CG accurate.
#include <algorithm>

#include "device.hpp"

namespace csc {
namespace {

constexpr int kT = 64;   // output tile (64 x 64 per workgroup)
constexpr int kR = 32;   // rows (Gram) or inner columns (product) staged per round

// Offset of column c within row 0 of a panel-major block: element (i, c) is at
// col_base(L, c) + i * pw.
__device__ inline size_t col_base(const Layout& L, int c) {
  const int pan = c / L.pw;
  return (size_t)pan * L.panel_elems() + (size_t)(c - pan * L.pw);
}

// part[chunk][ti*64 + r][tj*64 + c] = sum over the chunk's rows i of
// A[i, ti*64 + r] * B[i, tj*64 + c], rows in increasing order.
__global__ __launch_bounds__(256) void k_gram(Layout L, const float* A, const float* B, int ka,
                                              int kb, int rows_per_chunk, int tiles_b,
                                              double* part) {
  __shared__ float As[kR][kT + 1];
  __shared__ float Bs[kR][kT + 1];
  const int ti = blockIdx.x / tiles_b, tj = blockIdx.x - ti * tiles_b;
  const int chunk = blockIdx.y;
  const int r0 = chunk * rows_per_chunk;
  const int r1 = min(L.n, r0 + rows_per_chunk);
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // a thread always stages the same column (256 is a multiple of 64)
  const int c = threadIdx.x & (kT - 1), r_0 = threadIdx.x >> 6;
  const int ca = ti * kT + c, cb = tj * kT + c;
  const bool va = ca < ka, vb = cb < kb;
  const float* Ac = A + (va ? col_base(L, ca) : 0);
  const float* Bc = B + (vb ? col_base(L, cb) : 0);
  for (int rb = r0; rb < r1; rb += kR) {
#pragma unroll
    for (int r = r_0; r < kR; r += 256 / kT) {
      const int gi = rb + r;
      const bool in = gi < r1;
      As[r][c] = (in && va) ? Ac[(size_t)gi * L.pw] : 0.f;
      Bs[r][c] = (in && vb) ? Bc[(size_t)gi * L.pw] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kR; ++r) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = (double)As[r][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = (double)Bs[r][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  const int ldp = tiles_b * kT;
  double* out = part + (size_t)chunk * (gridDim.x / tiles_b) * kT * ldp;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
      out[(size_t)(ti * kT + ty * 4 + i) * ldp + tj * kT + tx * 4 + j] = acc[i][j];
}

// G[i * ldg + j] = sum over chunks (in order) of the partial tiles.
__global__ void k_gram_reduce(const double* part, int chunks, int rows_pad, int cols_pad, int ka,
                              int kb, double* G, int ldg) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= ka * kb) return;
  const int i = e / kb, j = e - i * kb;
  double s = 0.0;
  for (int c = 0; c < chunks; ++c) s += part[((size_t)c * rows_pad + i) * cols_pad + j];
  G[(size_t)i * ldg + j] = s;
}

// Out[i, j] = c0 * In0[i, j] + sum_{l < kin} In1[i, l] * S[l * lds + j] for
// every stored column j of the layout (S is zero beyond its live columns, so
// padding columns stay zero); float64 sums, rounded once to float32.  Out may
// be In0, never In1.
__global__ __launch_bounds__(256) void k_block_mul(Layout L, float c0, const float* In0,
                                                   const float* In1, const double* S, int kin,
                                                   int kout, int lds, float* Out) {
  __shared__ float Xs[kT][kR + 1];
  __shared__ double Ss[kR][kT + 1];
  const int W = L.np * L.pw;
  const int i0 = blockIdx.x * kT, j0 = blockIdx.y * kT;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  // a thread always stages the same inner column of In1 and output column of S
  const int xl = threadIdx.x & (kR - 1), xr0 = threadIdx.x >> 5;
  const int sc = threadIdx.x & (kT - 1), sl0 = threadIdx.x >> 6;
  const int gj_s = j0 + sc;
  for (int lb = 0; lb < kin; lb += kR) {
    const int gl = lb + xl;
    const bool vl = gl < kin;
    const float* Xc = In1 + (vl ? col_base(L, gl) : 0);
#pragma unroll
    for (int r = xr0; r < kT; r += 256 / kR) {
      const int gi = i0 + r;
      Xs[r][xl] = (vl && gi < L.n) ? Xc[(size_t)gi * L.pw] : 0.f;
    }
#pragma unroll
    for (int l = sl0; l < kR; l += 256 / kT) {
      const int g2 = lb + l;
      Ss[l][sc] = (g2 < kin && gj_s < kout) ? S[(size_t)g2 * lds + gj_s] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int l = 0; l < kR; ++l) {
      double x[4], sv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) x[i] = (double)Xs[ty * 4 + i][l];
#pragma unroll
      for (int j = 0; j < 4; ++j) sv[j] = Ss[l][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(x[i], sv[j], acc[i][j]);
    }
    __syncthreads();
  }
  // four consecutive columns of one panel (pw is a multiple of 4): float4 access
  const int gj = j0 + tx * 4;
  if (gj >= W) return;
  const size_t cb = col_base(L, gj);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int gi = i0 + ty * 4 + i;
    if (gi >= L.n) continue;
    const size_t o = cb + (size_t)gi * L.pw;
    float4 base = make_float4(0.f, 0.f, 0.f, 0.f);
    if (c0 != 0.f) base = *reinterpret_cast<const float4*>(In0 + o);
    float4 out;
    out.x = (float)((double)c0 * (double)base.x + acc[i][0]);
    out.y = (float)((double)c0 * (double)base.y + acc[i][1]);
    out.z = (float)((double)c0 * (double)base.z + acc[i][2]);
    out.w = (float)((double)c0 * (double)base.w + acc[i][3]);
    *reinterpret_cast<float4*>(Out + o) = out;
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

GramPlan gram_plan(const Layout& L, int ka, int kb) {
  GramPlan g;
  g.tiles_a = (ka + kT - 1) / kT;
  g.tiles_b = (kb + kT - 1) / kT;
  const int tiles = g.tiles_a * g.tiles_b;
  int chunks = std::max(1, 512 / tiles);
  const int max_chunks = (L.n + kR - 1) / kR;
  chunks = std::min(chunks, max_chunks);
  int rows = (L.n + chunks - 1) / chunks;
  rows = (rows + kR - 1) / kR * kR;
  g.rows_per_chunk = rows;
  g.chunks = (L.n + rows - 1) / rows;
  return g;
}

size_t gram_part_elems(const Layout& L, int kmax) {
  size_t m = 0;
  for (int ka = kT; ka < kmax + kT; ka += kT)
    for (int kb = kT; kb < kmax + kT; kb += kT) {
      const GramPlan g = gram_plan(L, std::min(ka, kmax), std::min(kb, kmax));
      m = std::max(m, (size_t)g.chunks * g.tiles_a * kT * g.tiles_b * kT);
    }
  return m;
}

hipError_t launch_gram(const Layout& L, const float* A, const float* B, int ka, int kb,
                       double* part, double* G, int ldg, hipStream_t s) {
  const GramPlan g = gram_plan(L, ka, kb);
  hipLaunchKernelGGL(k_gram, dim3((unsigned)(g.tiles_a * g.tiles_b), (unsigned)g.chunks), dim3(256),
                     0, s, L, A, B, ka, kb, g.rows_per_chunk, g.tiles_b, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int n = ka * kb;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, part,
                     g.chunks, g.tiles_a * kT, g.tiles_b * kT, ka, kb, G, ldg);
  return hipGetLastError();
}

hipError_t launch_block_mul(const Layout& L, float c0, const float* In0, const float* In1,
                            const double* S, int kin, int kout, int lds, float* Out,
                            hipStream_t s) {
  const int W = L.np * L.pw;
  const dim3 grid((unsigned)((L.n + kT - 1) / kT), (unsigned)((W + kT - 1) / kT));
  hipLaunchKernelGGL(k_block_mul, grid, dim3(256), 0, s, L, c0, In0, In1, S, kin, kout, lds, Out);
  return hipGetLastError();
}

}  // namespace csc
