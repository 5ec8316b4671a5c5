// Device kernels of libcsc for gfx950 (CDNA4, wave64).
//
// The dominant kernel is k_cheb_step: one step of the Chebyshev three-term
// recurrence T_{m+1} = -2 A T_m - T_{m-1} (T_1 = -A T_0) on a panel-major
// float32 block, fused with the consumer of T_{m+1} (feature accumulation,
// sampled-row accumulation, float64 moments for the eigencount, or the CG
// operator).  It is a CSR SpMM: each row of A is walked by PW/4 lanes, each
// lane owning four consecutive columns of the panel, so one gathered
// neighbour row is a contiguous PW*4-byte segment read by consecutive lanes.  No MFMA: the step
// moves ~16-20 bytes per 2 flops and is bound by memory bandwidth.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "device.hpp"

namespace csc {

namespace {

using namespace dev;

template <int EPI, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void k_cheb_step(StepArgs a) {
  cheb_unit<EPI, FIRST, LAST>(a, work_unit(blockIdx.x, a.L.np * a.tiles, a.tiles, a.xcd));
}

template <int EPI, bool PREV>
__global__ __launch_bounds__(kBlock) void k_clen_scalar(StepArgs a) {
  clen_scalar_unit<EPI, PREV>(a, blockIdx.x);
}

hipError_t launch_step(const StepArgs& a, int epi, bool first, bool last, hipStream_t s) {
  const dim3 grid((unsigned)(a.L.np * a.tiles)), block(kBlock);
#define CSC_STEP(E, F, L) hipLaunchKernelGGL((k_cheb_step<E, F, L>), grid, block, 0, s, a)
  switch (epi) {
    case EPI_Y:
      if (first) { if (last) CSC_STEP(EPI_Y, true, true); else CSC_STEP(EPI_Y, true, false); }
      else { if (last) CSC_STEP(EPI_Y, false, true); else CSC_STEP(EPI_Y, false, false); }
      break;
    case EPI_MOM:
      if (first) { if (last) CSC_STEP(EPI_MOM, true, true); else CSC_STEP(EPI_MOM, true, false); }
      else { if (last) CSC_STEP(EPI_MOM, false, true); else CSC_STEP(EPI_MOM, false, false); }
      break;
    case EPI_MOMG:
      if (a.mgroup < 2 || a.mgroup > kMaxCountGroup || a.mnc4 < 4 || (a.mnc4 & 3))
        return hipErrorInvalidValue;
      if (first) { if (last) CSC_STEP(EPI_MOMG, true, true); else CSC_STEP(EPI_MOMG, true, false); }
      else { if (last) CSC_STEP(EPI_MOMG, false, true); else CSC_STEP(EPI_MOMG, false, false); }
      break;
    case EPI_YS:
      if (first) { if (last) CSC_STEP(EPI_YS, true, true); else CSC_STEP(EPI_YS, true, false); }
      else { if (last) CSC_STEP(EPI_YS, false, true); else CSC_STEP(EPI_YS, false, false); }
      break;
    case EPI_CG:
      if (first) CSC_STEP(EPI_CG, true, true); else CSC_STEP(EPI_CG, false, true);
      break;
    case EPI_CLEN:
      if (first) CSC_STEP(EPI_CLEN, true, false); else CSC_STEP(EPI_CLEN, false, false);
      break;
    case EPI_CLEN_Y:
      if (first) CSC_STEP(EPI_CLEN_Y, true, false); else CSC_STEP(EPI_CLEN_Y, false, false);
      break;
    case EPI_CLEN_CG:
      if (first) CSC_STEP(EPI_CLEN_CG, true, false); else CSC_STEP(EPI_CLEN_CG, false, false);
      break;
    case EPI_SPMM:
      CSC_STEP(EPI_SPMM, true, false);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef CSC_STEP
  return hipGetLastError();
}

// ------------------------------------------------------------ Laplacian ---
__global__ void k_degree_scale(int n, const int* row_ptr, const int* col, const float* w,
                               float* dinv_sqrt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k)
    if (col[k] != i) d += w ? (double)w[k] : 1.0;
  dinv_sqrt[i] = d > 0.0 ? (float)(1.0 / sqrt(d)) : 0.f;
}

__global__ void k_adjacency_values(int n, const int* row_ptr, const int* col, const float* w,
                                   const float* s, float* val) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double si = s[i];
  for (int k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
    const int j = col[k];
    const double wij = w ? (double)w[k] : 1.0;
    val[k] = (j == i) ? 0.f : (float)(si * wij * (double)s[j]);
  }
}

__global__ void k_check_csr(int n, int nnz, const int* row_ptr, const int* col, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (i == 0 && row_ptr[0] != 0) atomicOr(flag, 1);
  if (i == n) {
    if (row_ptr[n] != nnz) atomicOr(flag, 2);
    return;
  }
  const int b = row_ptr[i], e = row_ptr[i + 1];
  if (e < b || b < 0 || e > nnz) {
    atomicOr(flag, 4);
    return;
  }
  for (int k = b; k < e; ++k)
    if (col[k] < 0 || col[k] >= n) {
      atomicOr(flag, 8);
      return;
    }
}

// Stricter checks on a CSR that passed k_check_csr: no stored diagonal entry
// (16), columns strictly increasing within each row (32), and W symmetric,
// entry (j, i) present with the same weight for every stored (i, j) (64),
// found by binary search in row j.
__global__ void k_check_graph_strict(int n, const int* row_ptr, const int* col, const float* w,
                                     int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = row_ptr[i], e = row_ptr[i + 1];
  int bits = 0;
  for (int k = b; k < e; ++k) {
    const int j = col[k];
    if (j == i) bits |= 16;
    if (k > b && col[k - 1] >= j) bits |= 32;
    int lo = row_ptr[j], hi = row_ptr[j + 1] - 1, at = -1;
    while (lo <= hi) {
      const int m = lo + ((hi - lo) >> 1);
      const int cm = col[m];
      if (cm == i) {
        at = m;
        break;
      }
      if (cm < i)
        lo = m + 1;
      else
        hi = m - 1;
    }
    if (at < 0 || (w && w[at] != w[k])) bits |= 64;
  }
  if (bits) atomicOr(flag, bits);
}

// -------------------------------------------------------------- random ---
__global__ void k_gaussian_panels(Layout L, uint64_t seed, uint32_t t, uint32_t sid, float* out) {
  const size_t total = L.elems();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x)
    gaussian_elem(L, seed, t, sid, out, idx);
}

__global__ void k_gaussian_group(Layout L, uint64_t seed, uint32_t t, uint32_t sid, int nc,
                                 int nc4, float* out) {
  const size_t total = L.elems();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x)
    gaussian_group_elem(L, seed, t, sid, nc, nc4, out, idx);
}

__global__ void k_gaussian_rows(int n_rows, int w, uint64_t seed, uint32_t t, uint32_t sid,
                                float* R, int ld) {
  const size_t total = (size_t)n_rows * w;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const size_t i = e / w, j = e - i * w;
    R[i * ld + j] = gauss_entry(e, t, sid, seed, w);
  }
}

// -------------------------------------------------------------- layout ---
// Columns [0, wc) of a block between a wide layout Lw and a compact layout
// Lc (one thread per element of Lc; Lc's columns from wc on are zero).
__global__ void k_to_compact(Layout Lc, float* dst, Layout Lw, const float* src, int wc) {
  const size_t total = Lc.elems(), pe = Lc.panel_elems(), pw_pe = Lw.panel_elems();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t q = idx / pe, rem = idx - q * pe;
    const size_t i = rem / Lc.pw;
    const int cg = (int)q * Lc.pw + (int)(rem - i * Lc.pw);
    dst[idx] = cg < wc ? src[(size_t)(cg / Lw.pw) * pw_pe + i * Lw.pw + cg % Lw.pw] : 0.f;
  }
}

__global__ void k_from_compact(Layout Lc, const float* src, Layout Lw, float* dst, int wc) {
  const size_t total = Lc.elems(), pe = Lc.panel_elems(), pw_pe = Lw.panel_elems();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t q = idx / pe, rem = idx - q * pe;
    const size_t i = rem / Lc.pw;
    const int cg = (int)q * Lc.pw + (int)(rem - i * Lc.pw);
    if (cg < wc) dst[(size_t)(cg / Lw.pw) * pw_pe + i * Lw.pw + cg % Lw.pw] = src[idx];
  }
}

__global__ void k_pack(Layout L, const float* X, int ld, float* out) {
  const size_t total = L.elems(), pe = L.panel_elems();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t q = idx / pe, rem = idx - q * pe;
    const size_t i = rem / L.pw;
    const int cg = (int)q * L.pw + (int)(rem - i * L.pw);
    out[idx] = cg < L.w ? X[i * ld + cg] : 0.f;
  }
}

// Rows of an n_rows x w block written row-major to Y (leading dimension ld),
// from the panel-major layout L (PANEL) or from Y itself, optionally
// normalised to unit length (sq: the squared norms, or NULL).  A workgroup
// takes kTileRows rows and moves them with consecutive threads on
// consecutive elements (a thread per row would touch a cache line per row
// and per load); the norms go through LDS in chunks of kTileCols columns,
// where thread r adds up row r's float64 squares in column order.  When the
// row fits one chunk the staged tile also feeds the writes.
constexpr int kTileRows = 64, kTileCols = 128;

template <bool PANEL>
__global__ __launch_bounds__(256) void k_rows_out(Layout L, const float* in, int n_rows, int w,
                                                  float* Y, int ld, int normalize, double* sq) {
  __shared__ float tile[kTileRows][kTileCols + 1];
  __shared__ double inv[kTileRows];
  const int i0 = blockIdx.x * kTileRows;
  auto src = [&](int i, int c) -> float {
    if (PANEL) return in[(size_t)(c / L.pw) * L.panel_elems() + (size_t)i * L.pw + c % L.pw];
    return in[(size_t)i * ld + c];
  };
  const bool staged = normalize && w <= kTileCols;
  if (normalize) {
    double s = 0.0;
    for (int c0 = 0; c0 < w; c0 += kTileCols) {
      const int cw = min(kTileCols, w - c0);
      __syncthreads();
      for (int e = threadIdx.x; e < kTileRows * cw; e += blockDim.x) {
        const int r = e / cw, c = e - r * cw, i = i0 + r;
        tile[r][c] = i < n_rows ? src(i, c0 + c) : 0.f;
      }
      __syncthreads();
      if (threadIdx.x < kTileRows)
        for (int c = 0; c < cw; ++c) {
          const double v = tile[threadIdx.x][c];
          s += v * v;
        }
    }
    if (threadIdx.x < kTileRows) {
      const int i = i0 + threadIdx.x;
      if (sq && i < n_rows) sq[i] = s;
      inv[threadIdx.x] = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    }
    __syncthreads();
  }
  for (int c0 = 0; c0 < w; c0 += kTileCols) {
    const int cw = min(kTileCols, w - c0);
    for (int e = threadIdx.x; e < kTileRows * cw; e += blockDim.x) {
      const int r = e / cw, c = e - r * cw, i = i0 + r;
      if (i >= n_rows) continue;
      const float v = staged ? tile[r][c] : src(i, c0 + c);
      Y[(size_t)i * ld + c0 + c] = normalize ? (float)((double)v * inv[r]) : v;
    }
  }
}

template <class T>
__global__ void k_fill(T* p, size_t n, T v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_slot_map(int n_rows, const int* rows, int n, int* slot, int* bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_rows) return;
  const int r = rows[s];
  if (r < 0 || r >= n) {
    atomicOr(bad, 1);
    return;
  }
  slot[r] = s;
}

// ---------------------------------------------------------- reductions ---
__global__ __launch_bounds__(kBlock) void k_reduce(const double* part, int len, double* out) {
  reduce_vec(part + (size_t)blockIdx.x * len, len, out + blockIdx.x);
}

__global__ __launch_bounds__(kBlock) void k_col_dot(Layout L, int chunks, int rows,
                                                    const float* A, const float* B, double* part) {
  col_dot_unit(L, chunks, rows, A, B, part, blockIdx.x);
}

// ------------------------------------------------------------ sampling ---
constexpr int kChunk = kBlock * 4;

__device__ inline uint64_t sample_key(int i, uint64_t seed) {
  return philox4x64_10((uint64_t)i, 0ull, (uint64_t)CSC_STREAM_SAMPLE, 0ull, seed, 0ull).x0;
}

__global__ __launch_bounds__(kBlock) void k_sample_count(int N, uint64_t seed, uint64_t thresh,
                                                         int* counts) {
  __shared__ int sh[4];
  int c = 0;
  const int base = blockIdx.x * kChunk + threadIdx.x * 4;
  for (int e = 0; e < 4; ++e)
    if (base + e < N && sample_key(base + e, seed) <= thresh) ++c;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) c += __shfl_xor(c, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) counts[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void k_scan_counts(const int* counts, int nchunks, int* offsets, int* total) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int run = 0;
  for (int c = 0; c < nchunks; ++c) {
    offsets[c] = run;
    run += counts[c];
  }
  *total = run;
}

__global__ __launch_bounds__(kBlock) void k_sample_write(int N, uint64_t seed, uint64_t thresh,
                                                         const int* offsets, uint64_t* keys,
                                                         int* idx) {
  __shared__ int pre[kBlock];
  const int base = blockIdx.x * kChunk + threadIdx.x * 4;
  uint64_t kk[4];
  bool f[4];
  int c = 0;
  for (int e = 0; e < 4; ++e) {
    f[e] = false;
    if (base + e < N) {
      kk[e] = sample_key(base + e, seed);
      f[e] = kk[e] <= thresh;
    }
    c += f[e] ? 1 : 0;
  }
  pre[threadIdx.x] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int t = 0; t < kBlock; ++t) {
      const int v = pre[t];
      pre[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int pos = offsets[blockIdx.x] + pre[threadIdx.x];
  for (int e = 0; e < 4; ++e)
    if (f[e]) {
      keys[pos] = kk[e];
      idx[pos] = base + e;
      ++pos;
    }
}

// ------------------------------------------------------------------ CG ---
__global__ void k_cg_scatter(Layout L, int n, const int* idx, const int* lab, const float* wts,
                             float* R, float* P, float* mask, int* bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = idx[s], j = lab[s];
  if (i < 0 || i >= L.n || j < 0 || j >= L.w) {
    atomicOr(bad, 1);
    return;
  }
  const float w = wts ? wts[s] : 1.f;  // fidelity weight of sampled node s
  const size_t o = (size_t)(j / L.pw) * L.panel_elems() + (size_t)i * L.pw + j % L.pw;
  R[o] = w;
  P[o] = w;
  mask[i] = w;
}

__global__ void k_cg_alpha(int k, const double* rr, const double* pAp, int* active, double* alpha,
                           int* breakdown) {
  cg_alpha_block(k, rr, pAp, active, alpha, breakdown);
}

__global__ __launch_bounds__(kBlock) void k_cg_update1(Layout L, int tiles, const float* AP,
                                                       const float* P, float* X, float* R,
                                                       const double* alpha, double* part) {
  cg_update1_unit(L, tiles, AP, P, X, R, alpha, part, blockIdx.x);
}

__global__ void k_cg_scalar(int k, const double* rrn, double* rr, const double* bnorm2,
                            double* beta, int* active, int* iters, double* relres, int it,
                            double tol, int* nactive) {
  cg_scalar_block(k, rrn, rr, bnorm2, beta, active, iters, relres, it, tol, nactive);
}

__global__ __launch_bounds__(kBlock) void k_cg_update2(Layout L, const float* R, float* P,
                                                       const double* beta, const int* active) {
  const size_t total4 = L.elems() / 4;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total4;
       t += (size_t)gridDim.x * blockDim.x)
    cg_update2_elem(L, R, P, beta, active, t);
}

// Hard labels with one wave per row (rows grid-strided over the waves): lane
// l takes columns l, l + 64, ... under labels_row's rule (the first column of
// the largest x_c / sqrt(n2_c) among columns with n2_c > 0), and the lanes'
// picks merge to the larger value, the lower column on equal values: for
// finite values the column labels_row picks.  The row's reads and the copy
// out of X are coalesced over the lanes.
__global__ __launch_bounds__(kBlock) void k_labels(Layout L, const float* X,
                                                   const double* colnorm2, int* labels,
                                                   float* Xout, int ldx, const int* out_map) {
  const int lane = threadIdx.x & 63;
  const int nw = (int)((gridDim.x * blockDim.x) >> 6);
  const size_t pe = L.panel_elems();
  for (int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6); i < L.n; i += nw) {
    const int o = out_map ? out_map[i] : i;
    double best = 0.0;
    int arg = -1;  // no column with n2 > 0 yet
    for (int c = lane; c < L.w; c += 64) {
      const float x = X[(size_t)(c / L.pw) * pe + (size_t)i * L.pw + c % L.pw];
      if (Xout) Xout[(size_t)o * ldx + c] = x;
      const double n2 = colnorm2[c];
      if (n2 > 0.0) {
        const double v = (double)x / sqrt(n2);
        if (arg < 0 || v > best) {
          best = v;
          arg = c;
        }
      }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off);
      const int oa = __shfl_xor(arg, off);
      if (oa >= 0 && (arg < 0 || ob > best || (ob == best && oa < arg))) {
        best = ob;
        arg = oa;
      }
    }
    if (lane == 0) labels[o] = arg < 0 ? 0 : arg;
  }
}

inline unsigned grid_for(size_t n, size_t per = kBlock, size_t cap = 65536) {
  size_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ============================================================ launchers ===
// rows of a workgroup: PW/4 lanes per row, or one row per thread for the
// single-column layout (PW = 1)
int rows_per_tile(int pw) { return pw < 4 ? kBlock : 4 * (64 / (pw / 4)); }
int tiles_for(const Layout& L) { return (L.n + rows_per_tile(L.pw) - 1) / rows_per_tile(L.pw); }

hipError_t launch_cheb_step(const StepArgs& a, int epi, bool first, bool last, hipStream_t s) {
  if (a.L.pw == 1 && a.L.w == 1 && a.L.np == 1) {  // a single column as an n-vector
    const dim3 grid((unsigned)tiles_for(a.L)), block(kBlock);
    if (epi == EPI_CLEN) {
      if (first) hipLaunchKernelGGL((k_clen_scalar<EPI_CLEN, false>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_clen_scalar<EPI_CLEN, true>), grid, block, 0, s, a);
    } else if (epi == EPI_CLEN_CG) {
      if (first) hipLaunchKernelGGL((k_clen_scalar<EPI_CLEN_CG, false>), grid, block, 0, s, a);
      else hipLaunchKernelGGL((k_clen_scalar<EPI_CLEN_CG, true>), grid, block, 0, s, a);
    } else {
      return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if (a.L.pw < 4 || a.L.pw > 256 || (a.L.pw & 3)) return hipErrorInvalidValue;
  return launch_step(a, epi, first, last, s);
}

hipError_t launch_degree_scale(int n, const int* row_ptr, const int* col, const float* w,
                               float* dinv_sqrt, hipStream_t s) {
  hipLaunchKernelGGL(k_degree_scale, dim3(grid_for(n, kBlock, 1u << 30)), dim3(kBlock), 0, s, n,
                     row_ptr, col, w, dinv_sqrt);
  return hipGetLastError();
}

hipError_t launch_adjacency_values(int n, const int* row_ptr, const int* col, const float* w,
                                   const float* dinv_sqrt, float* val, hipStream_t s) {
  hipLaunchKernelGGL(k_adjacency_values, dim3(grid_for(n, kBlock, 1u << 30)), dim3(kBlock), 0, s,
                     n, row_ptr, col, w, dinv_sqrt, val);
  return hipGetLastError();
}

hipError_t launch_check_graph_strict(int n, const int* row_ptr, const int* col, const float* w,
                                     int* flag, hipStream_t s) {
  hipLaunchKernelGGL(k_check_graph_strict, dim3(grid_for((size_t)n, kBlock, 1u << 30)), dim3(kBlock),
                     0, s, n, row_ptr, col, w, flag);
  return hipGetLastError();
}

hipError_t launch_check_csr(int n, int nnz, const int* row_ptr, const int* col, int* flag,
                            hipStream_t s) {
  hipLaunchKernelGGL(k_check_csr, dim3(grid_for((size_t)n + 1, kBlock, 1u << 30)), dim3(kBlock),
                     0, s, n, nnz, row_ptr, col, flag);
  return hipGetLastError();
}

hipError_t launch_gaussian_panels(const Layout& L, uint64_t seed, uint32_t t, uint32_t sid,
                                  float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gaussian_panels, dim3(grid_for(L.elems())), dim3(kBlock), 0, s, L, seed, t,
                     sid, out);
  return hipGetLastError();
}

hipError_t launch_gaussian_group(const Layout& L, uint64_t seed, uint32_t t, uint32_t sid, int nc,
                                 int nc4, float* out, hipStream_t s) {
  if (nc < 1 || nc4 < nc || (nc4 & 3)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gaussian_group, dim3(grid_for(L.elems())), dim3(kBlock), 0, s, L, seed, t,
                     sid, nc, nc4, out);
  return hipGetLastError();
}

hipError_t launch_gaussian_rows(int n_rows, int w, uint64_t seed, uint32_t t, uint32_t sid,
                                float* R, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_gaussian_rows, dim3(grid_for((size_t)n_rows * w)), dim3(kBlock), 0, s,
                     n_rows, w, seed, t, sid, R, ld);
  return hipGetLastError();
}

hipError_t launch_pack(const Layout& L, const float* X, int ld, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(L.elems())), dim3(kBlock), 0, s, L, X, ld, out);
  return hipGetLastError();
}

hipError_t launch_to_compact(const Layout& Lc, float* dst, const Layout& Lw, const float* src,
                             int wc, hipStream_t s) {
  if (wc > Lc.w || wc > Lw.w || Lc.n != Lw.n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_to_compact, dim3(grid_for(Lc.elems())), dim3(kBlock), 0, s, Lc, dst, Lw, src,
                     wc);
  return hipGetLastError();
}

hipError_t launch_from_compact(const Layout& Lc, const float* src, const Layout& Lw, float* dst,
                               int wc, hipStream_t s) {
  if (wc > Lc.w || wc > Lw.w || Lc.n != Lw.n) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_from_compact, dim3(grid_for(Lc.elems())), dim3(kBlock), 0, s, Lc, src, Lw,
                     dst, wc);
  return hipGetLastError();
}

hipError_t launch_unpack(const Layout& L, const float* in, float* Y, int ld, int normalize,
                         hipStream_t s) {
  if (L.n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_out<true>, dim3((unsigned)((L.n + kTileRows - 1) / kTileRows)),
                     dim3(256), 0, s, L, in, L.n, L.w, Y, ld, normalize, (double*)nullptr);
  return hipGetLastError();
}

hipError_t launch_normalize_rows(int n_rows, int w, float* Y, int ld, hipStream_t s,
                                double* sq) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_rows_out<false>, dim3((unsigned)((n_rows + kTileRows - 1) / kTileRows)),
                     dim3(256), 0, s, Layout{}, (const float*)Y, n_rows, w, Y, ld, 1, sq);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<float>, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, size_t n, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<int>, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_slot_map(int n_rows, const int* rows, int n, int* slot, int* bad,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_slot_map, dim3(grid_for(n_rows, kBlock, 1u << 30)), dim3(kBlock), 0, s,
                     n_rows, rows, n, slot, bad);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* part, int len, int nvec, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce, dim3(nvec), dim3(kBlock), 0, s, part, len, out);
  return hipGetLastError();
}

int col_dot_chunks(const Layout& L) { return std::max(1, std::min(tiles_for(L), 2048 / L.np)); }
int col_dot_rows(const Layout& L) {
  const int c = col_dot_chunks(L);
  return (L.n + c - 1) / c;
}

hipError_t launch_col_dot(const Layout& L, const float* A, const float* B, double* part,
                          hipStream_t s) {
  const int chunks = col_dot_chunks(L);
  hipLaunchKernelGGL(k_col_dot, dim3((unsigned)(L.np * chunks)), dim3(kBlock), 0, s, L, chunks,
                     col_dot_rows(L), A, B, part);
  return hipGetLastError();
}

int sample_chunks(int N) { return (N + kChunk - 1) / kChunk; }

hipError_t launch_sample_count(int N, uint64_t seed, uint64_t thresh, int* counts, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_count, dim3(sample_chunks(N)), dim3(kBlock), 0, s, N, seed, thresh,
                     counts);
  return hipGetLastError();
}

hipError_t launch_scan_counts(const int* counts, int nchunks, int* offsets, int* total,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(64), 0, s, counts, nchunks, offsets, total);
  return hipGetLastError();
}

hipError_t launch_sample_write(int N, uint64_t seed, uint64_t thresh, const int* offsets,
                               uint64_t* keys, int* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_sample_write, dim3(sample_chunks(N)), dim3(kBlock), 0, s, N, seed, thresh,
                     offsets, keys, idx);
  return hipGetLastError();
}

size_t sort_pairs_temp_bytes(int count) {
  size_t bytes = 0;
  hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                     (const int*)nullptr, (int*)nullptr, count, 0, 64, nullptr);
  return bytes;
}

hipError_t sort_pairs(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout,
                      const int* vin, int* vout, int count, hipStream_t s) {
  return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, kin, kout, vin, vout, count, 0, 64,
                                            s);
}

hipError_t launch_cg_scatter(const Layout& L, int n, const int* idx, const int* lab,
                             const float* wts, float* R, float* P, float* mask, int* bad,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_cg_scatter, dim3(grid_for(n, kBlock, 1u << 30)), dim3(kBlock), 0, s, L, n,
                     idx, lab, wts, R, P, mask, bad);
  return hipGetLastError();
}

hipError_t launch_cg_alpha(int k, const double* rr, const double* pAp, int* active,
                           double* alpha, int* breakdown, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(kBlock), 0, s, k, rr, pAp, active, alpha,
                     breakdown);
  return hipGetLastError();
}

hipError_t launch_cg_update1(const Layout& L, const float* AP, const float* P, float* X, float* R,
                             const double* alpha, double* part, hipStream_t s) {
  const int tiles = tiles_for(L);
  hipLaunchKernelGGL(k_cg_update1, dim3((unsigned)(L.np * tiles)), dim3(kBlock), 0, s, L, tiles,
                     AP, P, X, R, alpha, part);
  return hipGetLastError();
}

hipError_t launch_cg_scalar(int k, const double* rrn, double* rr, const double* bnorm2,
                            double* beta, int* active, int* iters, double* relres, int it,
                            double tol, int* nactive, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_scalar, dim3(1), dim3(kBlock), 0, s, k, rrn, rr, bnorm2, beta, active,
                     iters, relres, it, tol, nactive);
  return hipGetLastError();
}

hipError_t launch_cg_update2(const Layout& L, const float* R, float* P, const double* beta,
                             const int* active, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_update2, dim3(grid_for(L.elems() / 4)), dim3(kBlock), 0, s, L, R, P,
                     beta, active);
  return hipGetLastError();
}

hipError_t launch_labels(const Layout& L, const float* X, const double* colnorm2, int* labels,
                         float* Xout, int ldx, const int* out_map, hipStream_t s) {
  // a wave per row: 4 rows per workgroup, at most 16384 workgroups (rows grid-strided)
  hipLaunchKernelGGL(k_labels, dim3(grid_for((size_t)L.n, kBlock / 64, 16384)), dim3(kBlock), 0, s,
                     L, X, colnorm2, labels, Xout, ldx, out_map);
  return hipGetLastError();
}

}  // namespace csc
