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
#include <hipcub/hipcub.hpp>

#include "kernels.hpp"

namespace csc {

namespace {

constexpr int kBlock = 256;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum over the 256 threads of a block in a fixed order; result on thread 0.
__device__ inline double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  return r;
}

__device__ inline float gauss_entry(uint64_t e, uint32_t t, uint32_t sid, uint64_t seed, int w) {
  const Words4 x = philox4x64_10(e, (uint64_t)t, (uint64_t)sid, 0ull, seed, 0ull);
  const double u1 = (double)((x.x0 >> 11) + 1ull) * 0x1p-53;
  const double u2 = (double)(x.x1 >> 11) * 0x1p-53;
  const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
  return (float)(z / sqrt((double)w));
}

// ------------------------------------------------------- Chebyshev step ---
typedef float v4f __attribute__((ext_vector_type(4)));

__device__ inline v4f fma4(float a, v4f x, v4f acc) {
  return __builtin_elementwise_fma((v4f)a, x, acc);
}

__device__ inline v4f ld4(const float* base, size_t o4, int nt) {
  const v4f* p = reinterpret_cast<const v4f*>(base) + o4;
  return nt ? __builtin_nontemporal_load(p) : *p;
}

__device__ inline void st4(float* base, size_t o4, v4f v, int nt) {
  v4f* p = reinterpret_cast<v4f*>(base) + o4;
  if (nt)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

__device__ inline double dot4v(v4f a, v4f b) {
  return (double)a.x * (double)b.x + (double)a.y * (double)b.y + (double)a.z * (double)b.z +
         (double)a.w * (double)b.w;
}

// Workgroups are handed to the 8 XCDs round-robin (workgroup b runs on XCD
// b mod 8).  With xcd mapping on, XCD x processes a contiguous range of the
// panel-major work units, so each XCD's L2 sees the gathered rows of one
// panel at a time instead of all panels at once.
__device__ inline int work_unit(int b, int U, int xcd) {
  if (!xcd) return b;
  const int x = b & 7, j = b >> 3, q = U >> 3, r = U & 7;
  return x * q + (x < r ? x : r) + j;
}

// Lanes of a wave walk rows of a panel: a row takes lpr = PW/4 lanes (one
// float4 each), a wave holds rpw = floor(64 / lpr) rows, spare lanes idle.
struct RowMap {
  int lpr, rpw, rpb, r, q;
  bool lane_ok;
};

__device__ inline RowMap row_map(int pw) {
  RowMap m;
  m.lpr = pw >> 2;
  m.rpw = 64 / m.lpr;
  m.rpb = 4 * m.rpw;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane / m.lpr;
  m.q = lane - lr * m.lpr;
  m.lane_ok = lr < m.rpw;
  m.r = wave * m.rpw + lr;
  return m;
}

// Row i of A times the gathered panel: sum_k val[k] T_m[col[k]], k in CSR order.
__device__ inline v4f spmm_row(const StepArgs& a, const v4f* __restrict__ Tm4, int i, int q,
                               int lpr, bool valid) {
  v4f acc = (v4f)0.f;
  if (valid) {
    int k = a.row_ptr[i];
    const int end = a.row_ptr[i + 1];
    for (; k + 4 <= end; k += 4) {
      const int j0 = a.col[k], j1 = a.col[k + 1], j2 = a.col[k + 2], j3 = a.col[k + 3];
      const float v0 = a.val[k], v1 = a.val[k + 1], v2 = a.val[k + 2], v3 = a.val[k + 3];
      const v4f t0 = Tm4[(unsigned)j0 * lpr + q];
      const v4f t1 = Tm4[(unsigned)j1 * lpr + q];
      const v4f t2 = Tm4[(unsigned)j2 * lpr + q];
      const v4f t3 = Tm4[(unsigned)j3 * lpr + q];
      acc = fma4(v0, t0, acc);
      acc = fma4(v1, t1, acc);
      acc = fma4(v2, t2, acc);
      acc = fma4(v3, t3, acc);
    }
    for (; k < end; ++k) acc = fma4(a.val[k], Tm4[(unsigned)a.col[k] * lpr + q], acc);
  }
  return acc;
}

// Per-column sums over the rows of a workgroup in a fixed order, written to
// out[c * stride] for the pw columns c of the panel.  sh holds 4*64*4 doubles.
__device__ inline void column_partials(const double cs[4], const RowMap& m, int pw, double* sh,
                                       double* out, size_t stride) {
  if (m.lane_ok) {
#pragma unroll
    for (int e = 0; e < 4; ++e) sh[m.r * pw + m.q * 4 + e] = cs[e];
  }
  __syncthreads();
  if ((int)threadIdx.x < pw) {
    double t = 0.0;
    for (int rr = 0; rr < m.rpb; ++rr) t += sh[rr * pw + threadIdx.x];
    out[(size_t)threadIdx.x * stride] = t;
  }
}

template <int EPI, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void k_cheb_step(StepArgs a) {
  const RowMap m = row_map(a.L.pw);
  const int u = work_unit(blockIdx.x, a.L.np * a.tiles, a.xcd);
  const int panel = u / a.tiles;
  const int tile = u - panel * a.tiles;
  const int n = a.L.n;
  const int i = tile * m.rpb + m.r;
  const bool valid = m.lane_ok && i < n;
  const int nt = a.nt;
  const size_t pbase4 = (size_t)panel * a.L.panel_elems() / 4;
  const size_t o4 = pbase4 + (size_t)i * m.lpr + m.q;
  const v4f* __restrict__ Tm4 = reinterpret_cast<const v4f*>(a.Tm) + pbase4;

  const v4f acc = spmm_row(a, Tm4, i, m.q, m.lpr, valid);

  v4f tn = (v4f)0.f;
  v4f x0 = (v4f)0.f;  // T_0 row (first step, moments, CG)
  if (valid) {
    if (FIRST) {
      x0 = ld4(a.Tprev, o4, nt);
      tn = -acc;
    } else {
      const v4f tp = ld4(a.Tprev, o4, nt);
      tn = __builtin_elementwise_fma((v4f)-2.f, acc, -tp);
    }
    if (!LAST && EPI != EPI_CG) st4(a.Tnext, o4, tn, nt);
  }

  if constexpr (EPI == EPI_Y) {
    if (valid) {
      v4f y;
      if (FIRST)
        y = __builtin_elementwise_fma((v4f)a.c1, tn, (v4f)a.c0 * x0);
      else
        y = fma4(a.c1, tn, ld4(a.Y, o4, nt));
      st4(a.Y, o4, y, nt);
    }
  } else if constexpr (EPI == EPI_YS) {
    if (valid) {
      const int s = a.slot[i];
      if (s >= 0) {
        const float t[4] = {tn.x, tn.y, tn.z, tn.w};
        const float z[4] = {x0.x, x0.y, x0.z, x0.w};
        const int c0 = panel * a.L.pw + m.q * 4;
        float* out = a.Ys + (size_t)s * a.lds;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          if (c0 + e < a.L.w) {
            if (FIRST)
              out[c0 + e] = fmaf(a.c1, t[e], a.c0 * z[e]);
            else
              out[c0 + e] = fmaf(a.c1, t[e], out[c0 + e]);
          }
        }
      }
    }
  } else if constexpr (EPI == EPI_MOM) {
    __shared__ double sh[8];
    double s1 = 0.0, s0 = 0.0;
    if (valid) {
      const v4f r0 = FIRST ? x0 : ld4(a.T0, o4, nt);
      s1 = dot4v(r0, tn);
      if (FIRST) s0 = dot4v(r0, r0);
    }
    const double b1 = block_sum(s1, sh);
    if (threadIdx.x == 0) a.part[blockIdx.x] = b1;
    if (FIRST) {
      __syncthreads();
      const double b0 = block_sum(s0, sh);
      if (threadIdx.x == 0) a.part2[blockIdx.x] = b0;
    }
  } else if constexpr (EPI == EPI_CG) {
    __shared__ double sh[4 * 64 * 4];
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      const v4f p0 = FIRST ? x0 : ld4(a.T0, o4, nt);
      v4f yf;
      if (FIRST)
        yf = __builtin_elementwise_fma((v4f)a.c1, tn, (v4f)a.c0 * p0);
      else
        yf = fma4(a.c1, tn, ld4(a.Y, o4, nt));
      const float mk = a.mask[i];
      const v4f ap = __builtin_elementwise_fma((v4f)mk, p0, (v4f)a.gamma * (p0 - yf));
      st4(a.Y, o4, ap, nt);
      cs[0] = (double)p0.x * (double)ap.x;
      cs[1] = (double)p0.y * (double)ap.y;
      cs[2] = (double)p0.z * (double)ap.z;
      cs[3] = (double)p0.w * (double)ap.w;
    }
    column_partials(cs, m, a.L.pw, sh, a.part + (size_t)panel * a.L.pw * a.tiles + tile,
                    (size_t)a.tiles);
  }
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
    case EPI_YS:
      if (first) { if (last) CSC_STEP(EPI_YS, true, true); else CSC_STEP(EPI_YS, true, false); }
      else { if (last) CSC_STEP(EPI_YS, false, true); else CSC_STEP(EPI_YS, false, false); }
      break;
    case EPI_CG:
      if (first) CSC_STEP(EPI_CG, true, true); else CSC_STEP(EPI_CG, false, true);
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

// -------------------------------------------------------------- random ---
__global__ void k_gaussian_panels(Layout L, uint64_t seed, uint32_t t, uint32_t sid, float* out) {
  const size_t total = L.elems(), pe = L.panel_elems();
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (size_t)gridDim.x * blockDim.x) {
    const size_t q = idx / pe, rem = idx - q * pe;
    const int i = (int)(rem / L.pw), c = (int)(rem - (size_t)i * L.pw);
    const int cg = (int)q * L.pw + c;
    out[idx] = cg < L.w ? gauss_entry((uint64_t)i * L.w + cg, t, sid, seed, L.w) : 0.f;
  }
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

__global__ void k_unpack(Layout L, const float* in, float* Y, int ld, int normalize) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const size_t pe = L.panel_elems();
  double inv = 1.0;
  if (normalize) {
    double s = 0.0;
    for (int c = 0; c < L.w; ++c) {
      const double v = in[(size_t)(c / L.pw) * pe + (size_t)i * L.pw + c % L.pw];
      s += v * v;
    }
    inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  }
  for (int c = 0; c < L.w; ++c) {
    const float v = in[(size_t)(c / L.pw) * pe + (size_t)i * L.pw + c % L.pw];
    Y[(size_t)i * ld + c] = normalize ? (float)((double)v * inv) : v;
  }
}

__global__ void k_normalize_rows(int n_rows, int w, float* Y, int ld) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_rows) return;
  float* y = Y + (size_t)i * ld;
  double s = 0.0;
  for (int c = 0; c < w; ++c) s += (double)y[c] * (double)y[c];
  const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int c = 0; c < w; ++c) y[c] = (float)((double)y[c] * inv);
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
  __shared__ double sh[8];
  const size_t base = (size_t)blockIdx.x * len;
  double s = 0.0;
  for (int t = threadIdx.x; t < len; t += kBlock) s += part[base + t];
  const double b = block_sum(s, sh);
  if (threadIdx.x == 0) out[blockIdx.x] = b;
}

__global__ __launch_bounds__(kBlock) void k_col_dot(Layout L, int tiles, const float* A,
                                                    const float* B, double* part) {
  __shared__ double sh[4 * 64 * 4];
  const RowMap m = row_map(L.pw);
  const int panel = blockIdx.x / tiles, tile = blockIdx.x - panel * tiles;
  const int i = tile * m.rpb + m.r;
  double cs[4] = {0.0, 0.0, 0.0, 0.0};
  if (m.lane_ok && i < L.n) {
    const size_t o4 = (size_t)panel * L.panel_elems() / 4 + (size_t)i * m.lpr + m.q;
    const v4f x = reinterpret_cast<const v4f*>(A)[o4];
    const v4f y = reinterpret_cast<const v4f*>(B)[o4];
    cs[0] = (double)x.x * y.x;
    cs[1] = (double)x.y * y.y;
    cs[2] = (double)x.z * y.z;
    cs[3] = (double)x.w * y.w;
  }
  column_partials(cs, m, L.pw, sh, part + (size_t)panel * L.pw * tiles + tile, (size_t)tiles);
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
__global__ void k_cg_scatter(Layout L, int n, const int* idx, const int* lab, float* R, float* P,
                             float* mask, int* bad) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const int i = idx[s], j = lab[s];
  if (i < 0 || i >= L.n || j < 0 || j >= L.w) {
    atomicOr(bad, 1);
    return;
  }
  const size_t o = (size_t)(j / L.pw) * L.panel_elems() + (size_t)i * L.pw + j % L.pw;
  R[o] = 1.f;
  P[o] = 1.f;
  mask[i] = 1.f;
}

__global__ void k_cg_alpha(int k, const double* rr, const double* pAp, int* active, double* alpha,
                           int* breakdown) {
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double al = 0.0;
    if (active[j]) {
      if (pAp[j] > 0.0) {
        al = rr[j] / pAp[j];
      } else {
        active[j] = 0;
        atomicOr(breakdown, 1);
      }
    }
    alpha[j] = al;
  }
}

// x += alpha p and r -= alpha A p per column (float64 scalars), then the
// per-column partial sums of r^T r.
__global__ __launch_bounds__(kBlock) void k_cg_update1(Layout L, int tiles, const float* AP,
                                                       const float* P, float* X, float* R,
                                                       const double* alpha, double* part) {
  __shared__ double sh[4 * 64 * 4];
  const RowMap m = row_map(L.pw);
  const int panel = blockIdx.x / tiles, tile = blockIdx.x - panel * tiles;
  const int i = tile * m.rpb + m.r;
  const int c0 = panel * L.pw + m.q * 4;
  double cs[4] = {0.0, 0.0, 0.0, 0.0};
  if (m.lane_ok && i < L.n) {
    const size_t o4 = (size_t)panel * L.panel_elems() / 4 + (size_t)i * m.lpr + m.q;
    const v4f ap = reinterpret_cast<const v4f*>(AP)[o4];
    const v4f p = reinterpret_cast<const v4f*>(P)[o4];
    v4f x = reinterpret_cast<v4f*>(X)[o4];
    v4f rr = reinterpret_cast<v4f*>(R)[o4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      const double al = c < L.w ? alpha[c] : 0.0;
      x[e] = (float)((double)x[e] + al * (double)p[e]);
      rr[e] = (float)((double)rr[e] - al * (double)ap[e]);
      cs[e] = (double)rr[e] * (double)rr[e];
    }
    reinterpret_cast<v4f*>(X)[o4] = x;
    reinterpret_cast<v4f*>(R)[o4] = rr;
  }
  column_partials(cs, m, L.pw, sh, part + (size_t)panel * L.pw * tiles + tile, (size_t)tiles);
}

__global__ void k_cg_scalar(int k, const double* rrn, double* rr, const double* bnorm2,
                            double* beta, int* active, int* iters, double* relres, int it,
                            double tol, int* nactive) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  int mine = 0;
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    double b = 0.0;
    if (active[j]) {
      const double rel = sqrt(rrn[j]) / sqrt(bnorm2[j]);
      relres[j] = rel;
      iters[j] = it;
      b = rrn[j] / rr[j];
      rr[j] = rrn[j];
      if (rel <= tol)
        active[j] = 0;
      else
        ++mine;
    }
    beta[j] = b;
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) *nactive = cnt;
}

// p = r + beta p for the columns still iterating.
__global__ __launch_bounds__(kBlock) void k_cg_update2(Layout L, const float* R, float* P,
                                                       const double* beta, const int* active) {
  const int lpr = L.pw >> 2;
  const size_t total4 = L.elems() / 4, pe4 = L.panel_elems() / 4;
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total4;
       t += (size_t)gridDim.x * blockDim.x) {
    const int panel = (int)(t / pe4);
    const int q = (int)((t - (size_t)panel * pe4) % lpr);
    const int c0 = panel * L.pw + q * 4;
    const v4f rv = reinterpret_cast<const v4f*>(R)[t];
    v4f pv = reinterpret_cast<v4f*>(P)[t];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int c = c0 + e;
      if (c < L.w && active[c]) pv[e] = (float)((double)rv[e] + beta[c] * (double)pv[e]);
    }
    reinterpret_cast<v4f*>(P)[t] = pv;
  }
}

__global__ void k_labels(Layout L, const float* X, const double* colnorm2, int* labels,
                         float* Xout, int ldx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L.n) return;
  const size_t pe = L.panel_elems();
  double best = 0.0;
  int arg = 0;
  bool found = false;
  for (int c = 0; c < L.w; ++c) {
    const float x = X[(size_t)(c / L.pw) * pe + (size_t)i * L.pw + c % L.pw];
    if (Xout) Xout[(size_t)i * ldx + c] = x;
    const double n2 = colnorm2[c];
    if (n2 > 0.0) {
      const double v = (double)x / sqrt(n2);
      if (!found || v > best) {
        best = v;
        arg = c;
        found = true;
      }
    }
  }
  labels[i] = arg;
}

inline unsigned grid_for(size_t n, size_t per = kBlock, size_t cap = 65536) {
  size_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

// ============================================================ launchers ===
int rows_per_tile(int pw) { return 4 * (64 / (pw / 4)); }
int tiles_for(const Layout& L) { return (L.n + rows_per_tile(L.pw) - 1) / rows_per_tile(L.pw); }

hipError_t launch_cheb_step(const StepArgs& a, int epi, bool first, bool last, hipStream_t s) {
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

hipError_t launch_unpack(const Layout& L, const float* in, float* Y, int ld, int normalize,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_unpack, dim3(grid_for(L.n, kBlock, 1u << 30)), dim3(kBlock), 0, s, L, in, Y,
                     ld, normalize);
  return hipGetLastError();
}

hipError_t launch_normalize_rows(int n_rows, int w, float* Y, int ld, hipStream_t s) {
  hipLaunchKernelGGL(k_normalize_rows, dim3(grid_for(n_rows, kBlock, 1u << 30)), dim3(kBlock), 0,
                     s, n_rows, w, Y, ld);
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

hipError_t launch_col_dot(const Layout& L, const float* A, const float* B, double* part,
                          hipStream_t s) {
  const int tiles = tiles_for(L);
  hipLaunchKernelGGL(k_col_dot, dim3((unsigned)(L.np * tiles)), dim3(kBlock), 0, s, L, tiles, A,
                     B, part);
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

hipError_t launch_cg_scatter(const Layout& L, int n, const int* idx, const int* lab, float* R,
                             float* P, float* mask, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_scatter, dim3(grid_for(n, kBlock, 1u << 30)), dim3(kBlock), 0, s, L, n,
                     idx, lab, R, P, mask, bad);
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
                         float* Xout, int ldx, hipStream_t s) {
  hipLaunchKernelGGL(k_labels, dim3(grid_for(L.n, kBlock, 1u << 30)), dim3(kBlock), 0, s, L, X,
                     colnorm2, labels, Xout, ldx);
  return hipGetLastError();
}

}  // namespace csc
