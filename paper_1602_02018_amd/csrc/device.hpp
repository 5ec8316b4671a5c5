// Device-side building blocks shared by the single-graph and the batched
// kernels: each body processes one work unit, so both launch styles run the
// same arithmetic.
#pragma once

#include "kernels.hpp"

namespace csc {
namespace dev {

constexpr int kBlock = 256;
static_assert(kMomSlots * 64 == kBlock, "one moment partial per wave of a step workgroup");

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

__host__ __device__ inline v4f fma4(float a, v4f x, v4f acc) {
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
// b mod 8).  Orders of the U = P * T panel-major work units (P panels of T
// row tiles):
//   0  unit b: consecutive workgroups on different XCDs;
//   1  XCD x takes the x-th contiguous eighth of the units, so with several
//      panels each XCD's L2 sees the gathered rows of one panel;
//   2  the units are re-listed slab-major (row slab s = the s-th eighth of
//      the tiles, then panel, then tile) before the split of order 1: every
//      XCD keeps one row slab and all XCDs walk the panels in step, so only
//      one panel's gathered rows are live at a time.
// Each order is a bijection of [0, U).
__host__ __device__ inline int work_unit(int b, int U, int T, int xcd) {
  if (!xcd) return b;
  const int x = b & 7, j = b >> 3, q = U >> 3, r = U & 7;
  const int v = x * q + (x < r ? x : r) + j;
  if (xcd == 1) return v;
  const int P = U / T, tq = T >> 3, tr = T & 7;
  const int big = P * (tq + 1);  // units of a slab with tq + 1 tiles
  int s, start, ts;
  if (v < big * tr) {
    s = v / big;
    start = s * big;
    ts = tq + 1;
  } else {  // tq >= 1 here: slabs with tq + 1 tiles hold every unit when tq == 0
    s = tr + (v - big * tr) / (P * tq);
    start = big * tr + (s - tr) * P * tq;
    ts = tq;
  }
  const int off = v - start, panel = off / ts;
  return panel * T + s * tq + (s < tr ? s : tr) + (off - panel * ts);
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

// Row handled at walk position r of a step: r itself, or sched[r] when the
// step follows a row schedule; -1 past the last row (or for a schedule entry
// outside [0, n), which a valid schedule never holds).
__host__ __device__ inline int step_row(const StepArgs& a, int r) {
  if (r >= a.L.n) return -1;
  if (!a.sched) return r;
  const int i = a.sched[r];
  return (unsigned)i < (unsigned)a.L.n ? i : -1;
}

// Row i of A times the gathered panel: sum_k val[k] T_m[col[k]], k in CSR order.
// A row of 64 or more neighbours gathers 8 rows per round trip while the next
// 8 column indices load, so a high-degree row's lane waits one round trip per
// 8 neighbours instead of two per 4: on power-law graphs those lanes' chains
// (~1000 round trips for a degree-2000 hub) otherwise set the step time at
// narrow widths.  Shorter rows keep the 4-wide loop (measured no slower; the
// threshold 16, 24, 32 or 64 changes little, 64 was best by 1-3%).  The sums
// stay in CSR order either way.
// T is v4f (lane q of the lpr lanes of a row, four columns) or float (a
// single column, lpr = 1, q = 0).  Host-callable too, so that a CPU build
// can check the loop's accesses and sums (tests/step_host.cpp).
__host__ __device__ inline v4f fma_elt(float a, v4f x, v4f acc) { return fma4(a, x, acc); }
__host__ __device__ inline float fma_elt(float a, float x, float acc) {
  return __builtin_fmaf(a, x, acc);
}

template <class T>
__host__ __device__ inline T spmm_row_t(const StepArgs& a, const T* __restrict__ Tm4, int i, int q,
                                        int lpr, bool valid) {
  T acc = (T)0.f;
  if (valid) {
    int k = a.row_ptr[i];
    const int end = a.row_ptr[i + 1];
    if (end - k >= 64) {
      int j[8], jn[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) j[e] = a.col[k + e];
      for (;;) {  // entries k .. k + 7 exist here
        T t[8];
        float v[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = Tm4[(unsigned)j[e] * lpr + q];
#pragma unroll
        for (int e = 0; e < 8; ++e) v[e] = a.val[k + e];
        const bool more = k + 16 <= end;
        if (more) {
#pragma unroll
          for (int e = 0; e < 8; ++e) jn[e] = a.col[k + 8 + e];
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) acc = fma_elt(v[e], t[e], acc);
        k += 8;
        if (!more) break;  // fewer than 8 entries left
#pragma unroll
        for (int e = 0; e < 8; ++e) j[e] = jn[e];
      }
    }
    for (; k + 4 <= end; k += 4) {
      const int j0 = a.col[k], j1 = a.col[k + 1], j2 = a.col[k + 2], j3 = a.col[k + 3];
      const float v0 = a.val[k], v1 = a.val[k + 1], v2 = a.val[k + 2], v3 = a.val[k + 3];
      const T t0 = Tm4[(unsigned)j0 * lpr + q];
      const T t1 = Tm4[(unsigned)j1 * lpr + q];
      const T t2 = Tm4[(unsigned)j2 * lpr + q];
      const T t3 = Tm4[(unsigned)j3 * lpr + q];
      acc = fma_elt(v0, t0, acc);
      acc = fma_elt(v1, t1, acc);
      acc = fma_elt(v2, t2, acc);
      acc = fma_elt(v3, t3, acc);
    }
    for (; k < end; ++k) acc = fma_elt(a.val[k], Tm4[(unsigned)a.col[k] * lpr + q], acc);
  }
  return acc;
}

__device__ inline v4f spmm_row(const StepArgs& a, const v4f* __restrict__ Tm4, int i, int q,
                               int lpr, bool valid) {
  return spmm_row_t<v4f>(a, Tm4, i, q, lpr, valid);
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

// One work unit (panel, row tile) of one Chebyshev step.
// One step of Clenshaw's recurrence for sum_m a_m T_m(L - I) R:
// out = c0 R + c1 (A Tm) - Tprev (Tprev only when PREV).  Each element reads
// R, Tprev and the gathered rows of Tm and writes one block: four block
// accesses where the forward recurrence with a running sum needs five.
template <int EPI, bool PREV>
__device__ inline void clen_unit(const StepArgs& a, int u) {
  const RowMap m = row_map(a.L.pw);
  const int panel = u / a.tiles;
  const int tile = u - panel * a.tiles;
  const int i = step_row(a, tile * m.rpb + m.r);
  const bool valid = m.lane_ok && i >= 0;
  const int nt = a.nt;
  const size_t pbase4 = (size_t)panel * a.L.panel_elems() / 4;
  const size_t o4 = pbase4 + (size_t)i * m.lpr + m.q;
  const v4f* __restrict__ Tm4 = reinterpret_cast<const v4f*>(a.Tm) + pbase4;

  const v4f acc = spmm_row(a, Tm4, i, m.q, m.lpr, valid);
  if constexpr (EPI == EPI_SPMM) {
    if (valid) st4(a.Tnext, o4, acc, nt);
    return;
  }
  v4f r = (v4f)0.f, out = (v4f)0.f;
  if (valid) {
    r = ld4(a.T0, o4, nt);
    out = __builtin_elementwise_fma((v4f)a.c1, acc, (v4f)a.c0 * r);
    if (PREV) out = out - ld4(a.Tprev, o4, nt);
    if constexpr (EPI == EPI_CLEN) st4(a.Tnext, o4, out, nt);
    if constexpr (EPI == EPI_CLEN_Y) st4(a.Y, o4, out, nt);
  }
  if constexpr (EPI == EPI_CLEN_CG) {
    __shared__ double sh[4 * 64 * 4];
    double cs[4] = {0.0, 0.0, 0.0, 0.0};
    if (valid) {
      const float mk = a.mask[i];
      const v4f ap = __builtin_elementwise_fma((v4f)mk, r, (v4f)a.gamma * (r - out));
      st4(a.Y, o4, ap, nt);
      cs[0] = (double)r.x * (double)ap.x;
      cs[1] = (double)r.y * (double)ap.y;
      cs[2] = (double)r.z * (double)ap.z;
      cs[3] = (double)r.w * (double)ap.w;
    }
    if (a.part) {  // the per-column <p, Ap> partials (NULL: not wanted, no barrier)
      column_partials(cs, m, a.L.pw, sh, a.part + (size_t)panel * a.L.pw * a.tiles + tile,
                      (size_t)a.tiles);
      __syncthreads();
    }
  }
}

// One Clenshaw step (EPI_CLEN or EPI_CLEN_CG) on a single column stored as
// an n-vector (layout width and panel width 1): one row per thread, rows
// u*256 .. u*256+255 of unit u in natural order.  Every element takes the
// operations of clen_unit's lane for that column, so the results are the
// same bit for bit; the gathered vector is a quarter of a 4-column panel's
// bytes (4 MB at 1e6 nodes, about an XCD's L2).  EPI_CLEN_CG writes the
// unit's partial of <r, ap> to part[u] (column 0 of the column partials)
// unless part is NULL.
template <int EPI, bool PREV>
__device__ inline void clen_scalar_unit(const StepArgs& a, int u) {
  static_assert(EPI == EPI_CLEN || EPI == EPI_CLEN_CG, "single-column Clenshaw steps");
  const int i = u * kBlock + (int)threadIdx.x;
  const bool valid = i < a.L.n;
  const float acc = spmm_row_t<float>(a, a.Tm, i, 0, 1, valid);
  float r = 0.f, out = 0.f;
  if (valid) {
    r = a.T0[i];
    out = __builtin_fmaf(a.c1, acc, a.c0 * r);
    if (PREV) out = out - a.Tprev[i];
    if constexpr (EPI == EPI_CLEN) a.Tnext[i] = out;
  }
  if constexpr (EPI == EPI_CLEN_CG) {
    __shared__ double sh[8];
    double cs = 0.0;
    if (valid) {
      const float ap = __builtin_fmaf(a.mask[i], r, a.gamma * (r - out));
      a.Y[i] = ap;
      cs = (double)r * (double)ap;
    }
    if (a.part) {
      const double b = block_sum(cs, sh);
      if (threadIdx.x == 0) a.part[u] = b;
    }
  }
}

template <int EPI, bool FIRST, bool LAST>
__device__ inline void cheb_unit(const StepArgs& a, int u) {
  if constexpr ((EPI >= EPI_CLEN && EPI <= EPI_CLEN_CG) || EPI == EPI_SPMM) {
    clen_unit<EPI, !FIRST>(a, u);
    return;
  }
  const RowMap m = row_map(a.L.pw);
  const int panel = u / a.tiles;
  const int tile = u - panel * a.tiles;
  const int i = step_row(a, tile * m.rpb + m.r);
  const bool valid = m.lane_ok && i >= 0;
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
    // products for the Chebyshev doubling identities T_{2m} = 2 T_m^2 - 1 and
    // T_{2m+1} = 2 T_m T_{m+1} - T_1: <T_m, T_{m+1}> and <T_{m+1}, T_{m+1}>
    // (and <T_0, T_0> on the first step), so that p moments take p/2 steps
    // each wave writes its own sums (slot u kMomSlots + wave): no barrier
    double sx = 0.0, sq = 0.0, s0 = 0.0;
    if (valid) {
      const v4f tm = FIRST ? x0 : ld4(a.Tm, o4, nt);
      sx = dot4v(tm, tn);
      sq = dot4v(tn, tn);
      if (FIRST) s0 = dot4v(tm, tm);
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t slot = (size_t)u * kMomSlots + wave;
    const double wx = wave_sum(sx), wq = wave_sum(sq);
    const double w0 = FIRST ? wave_sum(s0) : 0.0;
    if (lane == 0) {
      a.part[slot] = wx;
      a.part2[slot] = wq;
      if (FIRST) a.part0[slot] = w0;
    }
  } else if constexpr (EPI == EPI_MOMG) {
    // the same products for a group of eigencount tests side by side, one set
    // of sums per test: this lane's four columns lie in test
    // (panel pw + 4 q) / mnc4 (lanes past the group's columns hold zeros);
    // wave sums per test, each wave writing its own slot as above
    double sx = 0.0, sq = 0.0, s0 = 0.0;
    if (valid) {
      const v4f tm = FIRST ? x0 : ld4(a.Tm, o4, nt);
      sx = dot4v(tm, tn);
      sq = dot4v(tn, tn);
      if (FIRST) s0 = dot4v(tm, tm);
    }
    const int jl = (panel * a.L.pw + m.q * 4) / a.mnc4;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const size_t slot = (size_t)u * kMomSlots + wave;
    for (int j = 0; j < a.mgroup; ++j) {
      const bool mine = jl == j;
      const double wx = wave_sum(mine ? sx : 0.0);
      const double wq = wave_sum(mine ? sq : 0.0);
      const double w0 = FIRST ? wave_sum(mine ? s0 : 0.0) : 0.0;
      if (lane == 0) {
        const size_t o = (size_t)j * a.mstride + slot;
        a.part[o] = wx;
        a.part2[o] = wq;
        if (FIRST) a.part0[o] = w0;
      }
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
    if (a.part) {  // as in clen_unit
      column_partials(cs, m, a.L.pw, sh, a.part + (size_t)panel * a.L.pw * a.tiles + tile,
                      (size_t)a.tiles);
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------ random -----
__device__ inline void gaussian_elem(const Layout& L, uint64_t seed, uint32_t t, uint32_t sid,
                                     float* out, size_t idx) {
  const size_t pe = L.panel_elems();
  const size_t q = idx / pe, rem = idx - q * pe;
  const int i = (int)(rem / L.pw), c = (int)(rem - (size_t)i * L.pw);
  const int cg = (int)q * L.pw + c;
  out[idx] = cg < L.w ? gauss_entry((uint64_t)i * L.w + cg, t, sid, seed, L.w) : 0.f;
}

// Element idx of the signals of tests t, t + 1, ... side by side (test j in
// columns [j nc4, j nc4 + nc), each drawn as the n x nc block of sub-stream
// t + j), the other columns zero.
__device__ inline void gaussian_group_elem(const Layout& L, uint64_t seed, uint32_t t, uint32_t sid,
                                           int nc, int nc4, float* out, size_t idx) {
  const size_t pe = L.panel_elems();
  const size_t q = idx / pe, rem = idx - q * pe;
  const int i = (int)(rem / L.pw), c = (int)(rem - (size_t)i * L.pw);
  const int cg = (int)q * L.pw + c, j = cg / nc4, cc = cg - j * nc4;
  out[idx] = (cg < L.w && cc < nc) ? gauss_entry((uint64_t)i * nc + cc, t + (uint32_t)j, sid, seed, nc)
                                   : 0.f;
}

// ---------------------------------------------------------- reductions ---
// out[0] = sum_t part[t], t < len, by one workgroup in a fixed order: thread
// x keeps four running sums (of the elements x + 256 (4 r + c), c = 0..3),
// so that four loads are in flight instead of one dependent chain, then the
// four in order and the threads by block_sum.
__device__ inline void reduce_vec(const double* part, int len, double* out) {
  __shared__ double sh[8];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int t = threadIdx.x;
  for (; t + 3 * kBlock < len; t += 4 * kBlock) {
    s0 += part[t];
    s1 += part[t + kBlock];
    s2 += part[t + 2 * kBlock];
    s3 += part[t + 3 * kBlock];
  }
  for (; t < len; t += kBlock) s0 += part[t];
  const double b = block_sum((s0 + s1) + (s2 + s3), sh);
  if (threadIdx.x == 0) *out = b;
  __syncthreads();
}

// Work unit u = (panel, chunk) of np * chunks: per-column sums of A(i, c) B(i, c)
// over rows [chunk * rows, (chunk + 1) * rows), to part[c * chunks + chunk].
// Each lane sums its four columns over its rows of the chunk in order (the
// products of float32 entries are exact in float64), then the workgroup's
// row slots are added in a fixed order.  One partial per column and chunk
// (a few thousand chunks in all), so the writes and the reduction after them
// stay small; units past np * chunks (a work list sized for more) do nothing.
__device__ inline void col_dot_unit(const Layout& L, int chunks, int rows, const float* A,
                                    const float* B, double* part, int u) {
  if (u >= L.np * chunks) return;  // uniform over the workgroup
  __shared__ double sh[4 * 64 * 4];
  const RowMap m = row_map(L.pw);
  const int panel = u / chunks, chunk = u - panel * chunks;
  const long long c0 = (long long)chunk * rows;  // chunks * rows < n + chunks
  const int r0 = (int)min((long long)L.n, c0), r1 = (int)min((long long)L.n, c0 + rows);
  double cs[4] = {0.0, 0.0, 0.0, 0.0};
  if (m.lane_ok) {
    const size_t pb4 = (size_t)panel * L.panel_elems() / 4;
    for (int i = r0 + m.r; i < r1; i += m.rpb) {
      const size_t o4 = pb4 + (size_t)i * m.lpr + m.q;
      const v4f x = reinterpret_cast<const v4f*>(A)[o4];
      const v4f y = reinterpret_cast<const v4f*>(B)[o4];
      cs[0] += (double)x.x * (double)y.x;
      cs[1] += (double)x.y * (double)y.y;
      cs[2] += (double)x.z * (double)y.z;
      cs[3] += (double)x.w * (double)y.w;
    }
  }
  column_partials(cs, m, L.pw, sh, part + (size_t)panel * L.pw * chunks + chunk, (size_t)chunks);
  __syncthreads();
}

// ------------------------------------------------------------------ CG ---
__device__ inline void cg_alpha_block(int k, const double* rr, const double* pAp, int* active,
                                      double* alpha, int* breakdown) {
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
// per-column partial sums of r^T r for work unit u = (panel, tile).
__device__ inline void cg_update1_unit(const Layout& L, int tiles, const float* AP,
                                       const float* P, float* X, float* R, const double* alpha,
                                       double* part, int u) {
  __shared__ double sh[4 * 64 * 4];
  const RowMap m = row_map(L.pw);
  const int panel = u / tiles, tile = u - panel * tiles;
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
  __syncthreads();
}

__device__ inline void cg_scalar_block(int k, const double* rrn, double* rr, const double* bnorm2,
                                       double* beta, int* active, int* iters, double* relres,
                                       int it, double tol, int* nactive) {
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
  __syncthreads();
}

// p = r + beta p for the columns still iterating; t indexes float4 elements.
__device__ inline void cg_update2_elem(const Layout& L, const float* R, float* P,
                                       const double* beta, const int* active, size_t t) {
  const int lpr = L.pw >> 2;
  const size_t pe4 = L.panel_elems() / 4;
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

// labels[i] = argmax_c X(i, c) / ||X_c|| (ties and zero columns -> lowest c);
// also copies row i to the node-major output when Xout is given.
// Row i of the layout is node out_map[i] of the caller (out_map NULL: node i).
__device__ inline void labels_row(const Layout& L, const float* X, const double* colnorm2,
                                  int* labels, float* Xout, int ldx, const int* out_map, int i) {
  const size_t pe = L.panel_elems();
  const int o = out_map ? out_map[i] : i;
  double best = 0.0;
  int arg = 0;
  bool found = false;
  for (int c = 0; c < L.w; ++c) {
    const float x = X[(size_t)(c / L.pw) * pe + (size_t)i * L.pw + c % L.pw];
    if (Xout) Xout[(size_t)o * ldx + c] = x;
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
  labels[o] = arg;
}

}  // namespace dev
}  // namespace csc
