// k-means on the sampled features (Alg. 2 step 6) on the GPU, float64, with
// the same arithmetic as the host form in kmeans.hip: k-means++ seeding from
// Philox draws, Lloyd iterations, empty clusters re-seeded with the farthest
// point, the lowest inertia over replicates kept.  Every sum keeps the host's
// order (squared distances over coordinates in order, the k-means++ running
// sum over points in blocks of kSeedBlock, centroids over members in index order, inertia
// over points in order), every tie goes to the lowest index, and this file is
// compiled without floating-point contraction, so labels and inertia are
// bit-identical to the host's.
//
// The seeding runs one workgroup per replicate (its rounds are sequential;
// each thread keeps one point's coordinates in registers when n <= 1024 and
// d <= 48);
// each Lloyd step is an assignment spread over the GPU (a workgroup per
// replicate and stripe of 8 centroids) and an update with one workgroup per
// replicate.  The parallel parts are the distance evaluations (independent
// per point and centroid), the centroid sums (independent per centroid and
// coordinate) and order-free reductions (argmin / argmax with index ties,
// integer counts).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"
#include "kmeans.hpp"

namespace csc {
namespace {

constexpr int kKmBlock = 1024;
// Seeding: the D^2 weights and their running sums (2 n doubles) stay in LDS
// up to n = 9216 (144 KB of the CU's 160 KB)
constexpr int kLdsDoubles = 18432;
constexpr int kCcLds = 256;  // the newest seed centroid in LDS when d <= 256
constexpr int kStripe = 8;       // centroids per assignment workgroup
constexpr int kStripeMaxD = 512;  // stripe centroids staged in LDS up to this d
constexpr int kChecks = 4;       // Lloyd iterations launched between convergence checks
constexpr int kUpdLds = 8192;    // update step: labels and members in LDS up to this n
constexpr int kUpdK = 1024;      // update step: cluster sizes and offsets in LDS up to this k
constexpr int kHistRows = 64;     // update step: points per block of the member-list counts
constexpr int kHistInts = 12288;  // update step: those (blocks x k) counts in LDS up to this size

struct KmItem {
  // the float32 points (k-means takes float32 features; every sum widens a
  // coordinate to float64 exactly where it is used, so storing them as float
  // changes no value and halves the bytes each pass reads)
  const float* X;   // n x d, row-major
  const float* Xt;  // d x n (coordinate j of point i at Xt[j * n + i])
  int n, d, k, r, max_iter;
  uint64_t seed;
  double* C;        // k x d
  double* mind;     // n (used when the weights do not fit in LDS)
  double* cum;      // n (likewise)
  double* blk;      // ceil(n / kSeedBlock): block offsets (when the weights are not in LDS)
  int* lab;         // n
  int* fresh;       // n
  int* counts;      // k
  int* mstart;      // k + 1
  int* members;     // n
  int* out_labels;  // n
  double* out_inertia;
  double* pbest;    // ceil(k / kStripe) x n: nearest centroid distance per stripe
  int* parg;        // ceil(k / kStripe) x n: its index
  int* flags;       // 4: Lloyd state between launches
  int* picks;       // k seeding picks, or NULL
};

// the same sum with the point read from the transposed block (coalesced
// across the threads of a wave, one point per thread); the coordinate loads
// of eight terms are issued before their additions, which stay in order
__device__ inline double sqd_t(const float* Xt, int n, int i, const double* c, int d) {
  double acc = 0.0;
  int j = 0;
  for (; j + 8 <= d; j += 8) {
    double xv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) xv[q] = Xt[(size_t)(j + q) * n + i];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const double diff = xv[q] - c[j + q];
      acc = acc + diff * diff;
    }
  }
  for (; j < d; ++j) {
    const double diff = Xt[(size_t)j * n + i] - c[j];
    acc = acc + diff * diff;
  }
  return acc;
}

// sqd_t for the points i, i + s and i + 2 s (those below n) at once: each sum
// runs over the coordinates in order exactly as sqd_t's, the three points'
// loads in flight together (a point past n reads point i's coordinates as a
// stand-in and its result is not used).
__device__ inline void sqd_t3(const float* Xt, int n, int i, int s, const double* c, int d,
                              double out[3]) {
  const int i1 = i + s < n ? i + s : i, i2 = i + 2 * s < n ? i + 2 * s : i;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  int j = 0;
  for (; j + 4 <= d; j += 4) {  // 12 loads in flight (the kernel keeps within 128 VGPRs)
    float x0[4], x1[4], x2[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      x0[q] = Xt[(size_t)(j + q) * n + i];
      x1[q] = Xt[(size_t)(j + q) * n + i1];
      x2[q] = Xt[(size_t)(j + q) * n + i2];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double cq = c[j + q];
      const double e0 = (double)x0[q] - cq, e1 = (double)x1[q] - cq, e2 = (double)x2[q] - cq;
      a0 = a0 + e0 * e0;
      a1 = a1 + e1 * e1;
      a2 = a2 + e2 * e2;
    }
  }
  for (; j < d; ++j) {
    const double cq = c[j];
    const double e0 = (double)Xt[(size_t)j * n + i] - cq, e1 = (double)Xt[(size_t)j * n + i1] - cq,
                 e2 = (double)Xt[(size_t)j * n + i2] - cq;
    a0 = a0 + e0 * e0;
    a1 = a1 + e1 * e1;
    a2 = a2 + e2 * e2;
  }
  out[0] = a0;
  out[1] = a1;
  out[2] = a2;
}

// The same sum with the point's coordinates held in registers (d <= kSeedRegD).
// The blocks k-means runs on are float32 features widened exactly to float64,
// so a float copy of a coordinate is exact.  Coordinates d..kSeedRegD-1 are
// zero in x and in c, so their terms add exact zeros and the sum is unchanged.
constexpr int kSeedRegD = 48;

__device__ inline double sqd_reg(const float (&x)[kSeedRegD], const double* c) {
  double acc = 0.0;
#pragma unroll
  for (int j = 0; j < kSeedRegD; ++j) {
    float xj = x[j];
    asm volatile("" : "+v"(xj));  // widen at the use: a hoisted float64 copy would not fit
    const double diff = (double)xj - c[j];
    acc = acc + diff * diff;
  }
  return acc;
}

__device__ inline double draw_uniform(uint64_t seed, uint64_t j, uint64_t r) {
  const Words4 x = philox4x64_10(j, r, (uint64_t)CSC_STREAM_KMEANS, 0ull, seed, 0ull);
  return (double)(x.x0 >> 11) * 0x1p-53;
}

// Block-wide reductions over (value, index) with index ties to the lowest.
struct VI {
  double v;
  int i;
};

__device__ inline VI better_min(VI a, VI b) { return (b.v < a.v || (b.v == a.v && b.i < a.i)) ? b : a; }
__device__ inline VI better_max(VI a, VI b) { return (b.v > a.v || (b.v == a.v && b.i < a.i)) ? b : a; }

template <bool MAX>
__device__ VI block_reduce(VI x, VI* sh) {
  for (int o = 32; o > 0; o >>= 1) {
    VI y;
    y.v = __shfl_down(x.v, o, 64);
    y.i = __shfl_down(x.i, o, 64);
    x = MAX ? better_max(x, y) : better_min(x, y);
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    VI b = sh[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) b = MAX ? better_max(b, sh[w]) : better_min(b, sh[w]);
    sh[0] = b;
  }
  __syncthreads();
  const VI out = sh[0];
  __syncthreads();
  return out;
}

// Smallest v over the workgroup (sh: one int per wave): the seeding's pick
// needs only an index, and this takes two barriers where the (value, index)
// reduction takes four.
__device__ inline int block_min(int v, int* sh) {
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  int m = sh[0];
  for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = min(m, sh[w]);
  __syncthreads();
  return m;
}

__device__ inline int block_or(int v, int* sh) {
  __syncthreads();
  if (threadIdx.x == 0) *sh = 0;
  __syncthreads();
  if (v) atomicOr(sh, 1);
  __syncthreads();
  const int out = *sh;
  __syncthreads();
  return out;
}

// Lloyd state of one replicate between launches (flags[]): whether the last
// assignment changed a label, whether the replicate has finished, whether the
// last update re-seeded an empty cluster, and whether labels exist yet.
enum { KM_CHANGED = 0, KM_DONE = 1, KM_RESEEDED = 2, KM_HAVE = 3 };

// k-means++ seeding of one replicate per workgroup (SEED_LDS: the D^2
// weights and their running sums in LDS); leaves the k seeds in t.C, every
// label at -1 and the Lloyd state cleared.
template <bool SEED_LDS>
__global__ __launch_bounds__(kKmBlock) void k_km_seed(const KmItem* items) {
  const KmItem t = items[blockIdx.x];
  const int n = t.n, d = t.d, k = t.k;
  __shared__ VI sh_vi[kKmBlock / 64];
  __shared__ int sh_min[kKmBlock / 64];
  __shared__ double sh_cc[kCcLds];

  // ---- k-means++ seeding.  The D^2 weights and their running sums live in
  // LDS when they fit.  The running sums take the host's two-level order: one
  // thread per block of kSeedBlock points forms the in-block running sums,
  // one thread the block offsets, and every point adds its block's offset;
  // the first point whose running sum passes u * total is found by an index
  // reduction.
  __shared__ double smem[SEED_LDS ? kLdsDoubles : 1];
  __shared__ double sh_blk[SEED_LDS ? kLdsDoubles / (2 * kSeedBlock) : 1];
  double* mind = SEED_LDS ? smem : t.mind;
  double* cum = SEED_LDS ? smem + n : t.cum;
  double* blk = SEED_LDS ? sh_blk : t.blk;
  const int nb = (n + kSeedBlock - 1) / kSeedBlock;
  // one point per thread with its coordinates in registers when they fit
  const bool reg = n <= (int)blockDim.x && d <= kSeedRegD;
  float xr[kSeedRegD];
  if (reg && (int)threadIdx.x < n) {
#pragma unroll
    for (int j = 0; j < kSeedRegD; ++j)
      xr[j] = j < d ? (float)t.Xt[(size_t)j * n + threadIdx.x] : 0.f;
  }
  {
    const double u = draw_uniform(t.seed, 0, (uint64_t)t.r);
    const int first = min((int)floor(u * n), n - 1);
    if (t.picks && threadIdx.x == 0) t.picks[0] = first;
    for (int j = threadIdx.x; j < d; j += blockDim.x) t.C[j] = t.X[(size_t)first * d + j];
    if (reg && (int)threadIdx.x < kSeedRegD)  // the centroid zero-padded to kSeedRegD
      sh_cc[threadIdx.x] = (int)threadIdx.x < d ? t.X[(size_t)first * d + threadIdx.x] : 0.0;
    __syncthreads();
    if (reg) {
      if ((int)threadIdx.x < n) mind[threadIdx.x] = sqd_reg(xr, sh_cc);
    } else {
      for (int i = threadIdx.x; i < n; i += blockDim.x) mind[i] = sqd_t(t.Xt, n, i, t.C, d);
    }
    __syncthreads();
  }
  for (int c = 1; c < k; ++c) {
    const double u = draw_uniform(t.seed, (uint64_t)c, (uint64_t)t.r);
    for (int q = threadIdx.x; q < nb; q += blockDim.x) {
      const int i0 = q * kSeedBlock, i1 = min(n, i0 + kSeedBlock);
      double in = 0.0;
      for (int i = i0; i < i1; ++i) {
        in = in + mind[i];
        cum[i] = in;
      }
      blk[q] = in;
    }
    __syncthreads();
    if (threadIdx.x == 0) {  // block totals -> block offsets, in block order
      double off = 0.0;
      for (int q = 0; q < nb; ++q) {
        const double tq = blk[q];
        blk[q] = off;
        off = off + tq;
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) cum[i] = blk[i / kSeedBlock] + cum[i];
    __syncthreads();
    const double total = cum[n - 1];
    int pick;
    if (total == 0.0) {
      pick = min((int)floor(u * n), n - 1);
    } else {
      const double target = u * total;
      int first = n;
      for (int i = threadIdx.x; i < n; i += blockDim.x)
        if (cum[i] > target && i < first) first = i;
      pick = block_min(first, sh_min);
      if (pick >= n) {  // rounding left the target at the total: last point with mass
        VI z{0.0, n};   // n - 1 - i of the largest such i, under the lowest-index rule
        for (int i = threadIdx.x; i < n; i += blockDim.x)
          if (mind[i] > 0.0 && n - 1 - i < z.i) z.i = n - 1 - i;
        const int m = block_reduce<false>(z, sh_vi).i;
        pick = m < n ? n - 1 - m : n - 1;  // none only with non-finite weights
      }
    }
    if (t.picks && threadIdx.x == 0) t.picks[c] = pick;
    double* cc = t.C + (size_t)c * d;
    const double* ccr = d <= kCcLds ? sh_cc : cc;  // the new centroid, read by every thread
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
      const double v = t.X[(size_t)pick * d + j];
      cc[j] = v;
      if (d <= kCcLds) sh_cc[j] = v;
    }
    __syncthreads();
    if (reg) {
      const int i = threadIdx.x;
      if (i < n) {
        const double v = sqd_reg(xr, sh_cc);
        mind[i] = v < mind[i] ? v : mind[i];
      }
    } else {  // three points per thread at a time
      const int bs = blockDim.x;
      for (int i = threadIdx.x; i < n; i += 3 * bs) {
        double v[3];
        sqd_t3(t.Xt, n, i, bs, ccr, d, v);
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const int ir = i + r * bs;
          if (ir < n) mind[ir] = v[r] < mind[ir] ? v[r] : mind[ir];
        }
      }
    }
    __syncthreads();
  }

  for (int i = threadIdx.x; i < n; i += blockDim.x) t.lab[i] = -1;
  if (threadIdx.x < 4) t.flags[threadIdx.x] = 0;
}

// Squared distances of one point (coordinate j at x[j n]) to the nc <= kStripe
// centroids of a stripe (centroid u's coordinates at cb[u d ..]), each summed
// over the coordinates in order.  FULL (nc == kStripe) drops the per-centroid
// guards, which kept the compiler from scheduling the full stripe's products
// freely (measured: the assignment 180 -> 112 us per launch).
template <bool FULL>
__device__ inline void stripe_sqd(const float* x, int n, const double* cb, int d, int nc,
                                  double (&a)[kStripe]) {
#pragma unroll
  for (int u = 0; u < kStripe; ++u) a[u] = 0.0;
  int j = 0;
  for (; j + 4 <= d; j += 4) {
    double xv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) xv[q] = x[(size_t)(j + q) * n];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int u = 0; u < kStripe; ++u)
        if (FULL || u < nc) {
          const double e = xv[q] - cb[(size_t)u * d + j + q];
          a[u] = a[u] + e * e;
        }
  }
  for (; j < d; ++j) {
    const double xj = x[(size_t)j * n];
#pragma unroll
    for (int u = 0; u < kStripe; ++u)
      if (FULL || u < nc) {
        const double e = xj - cb[(size_t)u * d + j];
        a[u] = a[u] + e * e;
      }
  }
}

// Assignment step, spread over the GPU: workgroup (s, r) finds, for every
// point of replicate r, the nearest of the centroids s*8 .. s*8+7 (squared
// distances summed over coordinates in order, ties to the lowest index) and
// leaves (distance, index) for the update to merge stripe by stripe.
__global__ __launch_bounds__(256) void k_km_assign(const KmItem* items, int count) {
  if ((int)blockIdx.y >= count) return;
  const KmItem t = items[blockIdx.y];
  if (t.flags[KM_DONE]) return;
  const int s = blockIdx.x, c0 = s * kStripe;
  if (c0 >= t.k) return;
  const int n = t.n, d = t.d, nc = min(kStripe, t.k - c0);
  __shared__ double cs[kStripe * kStripeMaxD];
  const double* cb = t.C + (size_t)c0 * d;
  if (d <= kStripeMaxD) {
    for (int e = threadIdx.x; e < nc * d; e += blockDim.x) cs[e] = cb[e];
    __syncthreads();
    cb = cs;
  }
  // one point per thread, the points spread over the z blocks
  for (int i = blockIdx.z * blockDim.x + threadIdx.x; i < n; i += blockDim.x * gridDim.z) {
    double a[kStripe];
    if (nc == kStripe)  // uniform over the workgroup: every stripe but the last
      stripe_sqd<true>(t.Xt + i, n, cb, d, nc, a);
    else
      stripe_sqd<false>(t.Xt + i, n, cb, d, nc, a);
    double best = a[0];
    int arg = c0;
#pragma unroll
    for (int u = 1; u < kStripe; ++u)
      if (u < nc && a[u] < best) {
        best = a[u];
        arg = c0 + u;
      }
    t.pbest[(size_t)s * n + i] = best;
    t.parg[(size_t)s * n + i] = arg;
  }
}

// Update step of one replicate per workgroup: merge the stripes (in centroid
// order, so ties keep the lowest index), stop when nothing changed after a
// step without re-seeding, else move the labels, recompute the centroids
// (members summed in index order) and re-seed empty clusters with the
// farthest point.
__global__ __launch_bounds__(kKmBlock) void k_km_update(const KmItem* items) {
  const KmItem t = items[blockIdx.x];
  if (t.flags[KM_DONE]) return;
  const int n = t.n, d = t.d, k = t.k, ns = (k + kStripe - 1) / kStripe;
  __shared__ VI sh_vi[kKmBlock / 64];
  __shared__ int sh_i;
  __shared__ __align__(16) int s_lab[kUpdLds];
  __shared__ int s_mem[kUpdLds];
  __shared__ int s_cnt[kUpdK], s_start[kUpdK + 1];
  __shared__ int s_hist[kHistInts];
  const bool in_lds = n <= kUpdLds;  // labels and member lists in LDS for the scans
  const bool k_lds = k <= kUpdK;     // cluster sizes and list offsets likewise
  double* C = t.C;
  int* lab = in_lds ? s_lab : t.lab;
  int* members = in_lds ? s_mem : t.members;
  int* counts = k_lds ? s_cnt : t.counts;
  int* mstart = k_lds ? s_start : t.mstart;
  int diff = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double best = t.pbest[i];
    int arg = t.parg[i];
    for (int s0 = 1; s0 < ns; s0 += 8) {  // eight stripes' loads in flight, merged in order
      double v[8];
      int a[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const bool ok = s0 + q < ns;
        v[q] = ok ? t.pbest[(size_t)(s0 + q) * n + i] : 0.0;
        a[q] = ok ? t.parg[(size_t)(s0 + q) * n + i] : 0;
      }
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (s0 + q < ns && v[q] < best) {
          best = v[q];
          arg = a[q];
        }
    }
    t.fresh[i] = arg;
    diff |= arg != t.lab[i];
  }
  const int changed = block_or(diff, &sh_i);
  const bool have = t.flags[KM_HAVE] != 0, was_reseeded = t.flags[KM_RESEEDED] != 0;
  __syncthreads();
  if (have && !was_reseeded && !changed) {
    if (threadIdx.x == 0) t.flags[KM_DONE] = 1;
    return;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) lab[i] = t.fresh[i];
  __syncthreads();
  // cluster sizes, then the members of every cluster in index order.  With
  // the labels in LDS and (blocks of kHistRows points) x k counts fitting
  // there too: per block and cluster the count, per cluster the running
  // offsets over the blocks (so the sizes), and each block's points placed in
  // order by one thread; else the sizes by integer atomics and each cluster's
  // members by a scan of all labels.  Both give the same lists.
  const int nbk = (n + kHistRows - 1) / kHistRows;
  const bool hist = in_lds && (size_t)nbk * k <= (size_t)kHistInts;
  if (hist) {
    for (int e = threadIdx.x; e < nbk * k; e += blockDim.x) s_hist[e] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x)
      atomicAdd(&s_hist[(i / kHistRows) * k + lab[i]], 1);
    __syncthreads();
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
      int run = 0;
      for (int b = 0; b < nbk; ++b) {
        const int h = s_hist[b * k + c];
        s_hist[b * k + c] = run;
        run += h;
      }
      counts[c] = run;
    }
  } else {
    for (int c = threadIdx.x; c < k; c += blockDim.x) counts[c] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) atomicAdd(&counts[lab[i]], 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int sum = 0;
    for (int c = 0; c < k; ++c) {
      mstart[c] = sum;
      sum += counts[c];
    }
    mstart[k] = sum;
  }
  __syncthreads();
  if (hist) {
    for (int b = threadIdx.x; b < nbk; b += blockDim.x) {
      int* off = s_hist + b * k;
      const int i1 = min(n, (b + 1) * kHistRows);
      for (int i = b * kHistRows; i < i1; ++i) {
        const int c = lab[i];
        members[mstart[c] + off[c]++] = i;
      }
    }
  } else {
    for (int c = threadIdx.x; c < k; c += blockDim.x) {
      int w = mstart[c];
      int i = 0;
      if (in_lds) {  // four labels per LDS read
        const int4* l4 = reinterpret_cast<const int4*>(lab);
        for (; i + 4 <= n; i += 4) {
          const int4 q = l4[i >> 2];
          if (q.x == c) members[w++] = i;
          if (q.y == c) members[w++] = i + 1;
          if (q.z == c) members[w++] = i + 2;
          if (q.w == c) members[w++] = i + 3;
        }
      }
      for (; i < n; ++i)
        if (lab[i] == c) members[w++] = i;
    }
  }
  __syncthreads();
  // centroid sums over members in index order; the d threads of one cluster
  // read one member row of X together, four members' loads in flight
  for (int e = threadIdx.x; e < k * d; e += blockDim.x) {
    const int c = e / d, j = e - c * d;
    const int cnt = counts[c];
    if (cnt == 0) continue;
    double acc = 0.0;
    const float* xj = t.X + j;
    int m = mstart[c];
    const int m1 = mstart[c + 1];
    for (; m + 8 <= m1; m += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = xj[(size_t)members[m + q] * d];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc = acc + v[q];
    }
    for (; m < m1; ++m) acc = acc + xj[(size_t)members[m] * d];
    C[(size_t)c * d + j] = acc / (double)cnt;
  }
  __syncthreads();
  int empty = 0;
  for (int c = threadIdx.x; c < k; c += blockDim.x) empty |= counts[c] == 0;
  const bool reseeded = block_or(empty, &sh_i) != 0;
  if (reseeded) {
    for (int c = 0; c < k; ++c) {
      if (counts[c] != 0) continue;  // uniform: every thread reads the same value
      VI x{-1.0, n};
      for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const double v = sqd_t(t.Xt, n, i, C + (size_t)lab[i] * d, d);
        x = better_max(x, VI{v, i});
      }
      const int far = block_reduce<true>(x, sh_vi).i;
      for (int j = threadIdx.x; j < d; j += blockDim.x) C[(size_t)c * d + j] = t.X[(size_t)far * d + j];
      __syncthreads();
      if (threadIdx.x == 0) {
        --counts[lab[far]];
        lab[far] = c;
        counts[c] = 1;
      }
      __syncthreads();
    }
  }
  if (in_lds) {
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += blockDim.x) t.lab[i] = lab[i];
  }
  if (threadIdx.x == 0) {
    t.flags[KM_HAVE] = 1;
    t.flags[KM_RESEEDED] = reseeded ? 1 : 0;
  }
}

// Inertia (points in order) and labels of one replicate per workgroup.
__global__ __launch_bounds__(kKmBlock) void k_km_finish(const KmItem* items) {
  const KmItem t = items[blockIdx.x];
  const int n = t.n, d = t.d;
  for (int i = threadIdx.x; i < n; i += blockDim.x)
    t.mind[i] = sqd_t(t.Xt, n, i, t.C + (size_t)t.lab[i] * d, d);
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = acc + t.mind[i];
    *t.out_inertia = acc;
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) t.out_labels[i] = t.lab[i];
}

__global__ void k_stage_points(int n, int d, const float* F, int ld, float* X, float* Xt) {
  const size_t total = (size_t)n * d;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int i = (int)(e / d), j = (int)(e - (size_t)i * d);
    const float v = F[(size_t)i * ld + j];
    X[e] = v;
    Xt[(size_t)j * n + i] = v;
  }
}

// Launches the seeding of `count` replicates (SEED_LDS when the D^2 weights fit).
hipError_t launch_seed(bool seed_lds, const KmItem* items, int count, hipStream_t s) {
  if (seed_lds)
    hipLaunchKernelGGL(k_km_seed<true>, dim3((unsigned)count), dim3(kKmBlock), 0, s, items);
  else
    hipLaunchKernelGGL(k_km_seed<false>, dim3((unsigned)count), dim3(kKmBlock), 0, s, items);
  return hipGetLastError();
}

bool seed_in_lds(int n) { return 2 * (size_t)n <= (size_t)kLdsDoubles; }

int stripes(int k) { return (k + kStripe - 1) / kStripe; }

// Lloyd iterations of `count` seeded replicates (items on the device, flags
// of replicate r at flags + 4 r): kChecks iterations of assign + update per
// round, then a look at the done flags; at most max_iter iterations.
csc_status run_lloyd(const KmItem* items, int count, int max_stripes, int max_n, int max_iter,
                     int* flags, hipStream_t s) {
  std::vector<int> h((size_t)count * 4);
  const unsigned chunks = (unsigned)std::min(64, std::max(1, (max_n + 255) / 256));
  for (int it = 0; it < max_iter;) {
    const int round = std::min(kChecks, max_iter - it);
    for (int q = 0; q < round; ++q) {
      hipLaunchKernelGGL(k_km_assign, dim3((unsigned)max_stripes, (unsigned)count, chunks), dim3(256),
                         0, s, items, count);
      CSC_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_km_update, dim3((unsigned)count), dim3(kKmBlock), 0, s, items);
      CSC_HIP(hipGetLastError());
    }
    it += round;
    if (it >= max_iter) break;
    CSC_HIP(hipMemcpyAsync(h.data(), flags, h.size() * sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    bool all = true;
    for (int r = 0; r < count && all; ++r) all = h[(size_t)r * 4 + KM_DONE] != 0;
    if (all) break;
  }
  hipLaunchKernelGGL(k_km_finish, dim3((unsigned)count), dim3(kKmBlock), 0, s, items);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// workspace of one input: X and its transpose (n x d floats) + per replicate C, mind, cum,
// lab, fresh, counts, mstart, members, labels, stripe results, seeding block
// offsets, Lloyd flags;
// plus inertias
size_t km_bytes(int n, int d, int k, int reps) {
  size_t b = 2 * align_up((size_t)n * d * sizeof(float));
  const size_t ns = (size_t)stripes(k);
  const size_t per = align_up((size_t)k * d * sizeof(double)) + 2 * align_up((size_t)n * sizeof(double)) +
                     4 * align_up((size_t)n * sizeof(int)) + 2 * align_up(((size_t)k + 1) * sizeof(int)) +
                     align_up(ns * n * sizeof(double)) + align_up(ns * n * sizeof(int)) +
                     align_up((size_t)((n + kSeedBlock - 1) / kSeedBlock) * sizeof(double));
  b += per * reps + align_up((size_t)reps * sizeof(double)) + align_up((size_t)reps * 4 * sizeof(int));
  b += align_up((size_t)reps * k * sizeof(int));  // seeding picks (csc_kmeans_seeds_device)
  return b;
}

struct KmPlan {
  float* X;
  float* Xt;
  std::vector<KmItem> items;
  double* inertia;
  int* labels0;  // replicate r's labels at labels0 + r * n
};

csc_status plan_km(Arena& ar, const float* F, int n, int d, int ld, int k, int reps, int max_iter,
                   uint64_t seed, KmPlan& P, hipStream_t s) {
  P.X = ar.take<float>((size_t)n * d);
  P.Xt = ar.take<float>((size_t)n * d);
  P.inertia = ar.take<double>(reps);
  P.items.resize(reps);
  P.labels0 = nullptr;
  for (int r = 0; r < reps; ++r) {
    KmItem& t = P.items[r];
    t.X = P.X;
    t.Xt = P.Xt;
    t.n = n;
    t.d = d;
    t.k = k;
    t.r = r;
    t.max_iter = max_iter;
    t.seed = seed;
    t.C = ar.take<double>((size_t)k * d);
    t.mind = ar.take<double>(n);
    t.cum = ar.take<double>(n);
    t.blk = ar.take<double>((n + kSeedBlock - 1) / kSeedBlock);
    t.lab = ar.take<int>(n);
    t.fresh = ar.take<int>(n);
    t.members = ar.take<int>(n);
    t.counts = ar.take<int>((size_t)k + 1);
    t.mstart = ar.take<int>((size_t)k + 1);
    t.out_labels = ar.take<int>(n);
    t.out_inertia = P.inertia + r;
    t.pbest = ar.take<double>((size_t)stripes(k) * n);
    t.parg = ar.take<int>((size_t)stripes(k) * n);
    t.picks = nullptr;
  }
  if (!ar.ok()) {
    set_error("internal: k-means workspace overflow");
    return CSC_E_INVALID_ARG;
  }
  hipLaunchKernelGGL(k_stage_points, dim3((unsigned)std::min<size_t>(((size_t)n * d + 255) / 256, 4096)),
                     dim3(256), 0, s, n, d, F, ld, P.X, P.Xt);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// best replicate in replicate order (first minimum), as the host form
csc_status finish_km(const KmPlan& P, int n, int reps, int32_t* labels, double* inertia_out,
                     hipStream_t s) {
  std::vector<double> in(reps);
  CSC_HIP(hipMemcpyAsync(in.data(), P.inertia, reps * sizeof(double), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  int best = 0;
  for (int r = 1; r < reps; ++r)
    if (in[r] < in[best]) best = r;
  CSC_HIP(hipMemcpyAsync(labels, P.items[best].out_labels, (size_t)n * sizeof(int),
                         hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  if (inertia_out) *inertia_out = in[best];
  return CSC_OK;
}

csc_status check_args(const float* F, int n, int d, int ld, int k, int reps, int max_iter,
                      const int32_t* labels) {
  CSC_REQUIRE(F && labels, "F and labels must be non-NULL");
  CSC_REQUIRE(n >= 1 && d >= 1 && ld >= d, "need n >= 1, d >= 1, ld >= d");
  CSC_REQUIRE(k >= 1 && k <= n, "k must lie in [1, n]");
  CSC_REQUIRE(reps >= 1 && max_iter >= 1, "need replicates >= 1 and max_iter >= 1");
  return CSC_OK;
}

}  // namespace
}  // namespace csc

using namespace csc;

extern "C" size_t csc_kmeans_device_workspace_bytes(int32_t n, int32_t d, int32_t k,
                                                    int32_t replicates) {
  if (n < 1 || d < 1 || k < 1 || replicates < 1) return 0;
  return km_bytes(n, d, k, replicates) + 256 * (14 * (size_t)replicates + 6);
}

extern "C" csc_status csc_kmeans_reduced_device(const float* F, int32_t n, int32_t d, int32_t ld,
                                                int32_t k, int32_t replicates, int32_t max_iter,
                                                uint64_t seed, int32_t* labels,
                                                double* inertia_out, void* ws, size_t ws_bytes,
                                                void* stream) {
  clear_error();
  CSC_TRY(check_args(F, n, d, ld, k, replicates, max_iter, labels));
  CSC_TRY(check_ws(ws, ws_bytes, csc_kmeans_device_workspace_bytes(n, d, k, replicates)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  KmPlan P;
  CSC_TRY(plan_km(ar, F, n, d, ld, k, replicates, max_iter, seed, P, s));
  KmItem* d_items = ar.take<KmItem>(replicates);
  int* flags = ar.take<int>((size_t)replicates * 4);
  if (!ar.ok()) {
    set_error("internal: k-means workspace overflow");
    return CSC_E_INVALID_ARG;
  }
  for (int r = 0; r < replicates; ++r) P.items[r].flags = flags + 4 * r;
  CSC_HIP(hipMemcpyAsync(d_items, P.items.data(), replicates * sizeof(KmItem),
                         hipMemcpyHostToDevice, s));
  CSC_HIP(launch_seed(seed_in_lds(n), d_items, replicates, s));
  CSC_TRY(run_lloyd(d_items, replicates, stripes(k), n, max_iter, flags, s));
  return finish_km(P, n, replicates, labels, inertia_out, s);
}

extern "C" csc_status csc_kmeans_seeds_device(const float* F, int32_t n, int32_t d, int32_t ld,
                                              int32_t k, int32_t replicates, uint64_t seed,
                                              int32_t* picks, void* ws, size_t ws_bytes,
                                              void* stream) {
  clear_error();
  CSC_TRY(check_args(F, n, d, ld, k, replicates, 1, picks));
  CSC_TRY(check_ws(ws, ws_bytes, csc_kmeans_device_workspace_bytes(n, d, k, replicates)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  KmPlan P;
  CSC_TRY(plan_km(ar, F, n, d, ld, k, replicates, 1, seed, P, s));
  KmItem* d_items = ar.take<KmItem>(replicates);
  int* flags = ar.take<int>((size_t)replicates * 4);
  int* d_picks = ar.take<int>((size_t)replicates * k);
  if (!ar.ok()) {
    set_error("internal: k-means workspace overflow");
    return CSC_E_INVALID_ARG;
  }
  for (int r = 0; r < replicates; ++r) {
    P.items[r].flags = flags + 4 * r;
    P.items[r].picks = d_picks + (size_t)r * k;
  }
  CSC_HIP(hipMemcpyAsync(d_items, P.items.data(), replicates * sizeof(KmItem),
                         hipMemcpyHostToDevice, s));
  CSC_HIP(launch_seed(seed_in_lds(n), d_items, replicates, s));
  CSC_HIP(hipMemcpyAsync(picks, d_picks, (size_t)replicates * k * sizeof(int), hipMemcpyDeviceToHost,
                         s));
  CSC_HIP(hipStreamSynchronize(s));
  return CSC_OK;
}

extern "C" size_t csc_kmeans_device_workspace_bytes_batched(int32_t G, const int32_t* n,
                                                            const int32_t* d, const int32_t* k,
                                                            int32_t replicates) {
  if (G < 1 || !n || !d || !k || replicates < 1) return 0;
  size_t b = 256 * 4 + align_up((size_t)G * replicates * sizeof(KmItem));
  for (int g = 0; g < G; ++g) b += csc_kmeans_device_workspace_bytes(n[g], d[g], k[g], replicates);
  return b;
}

extern "C" csc_status csc_kmeans_reduced_device_batched(int32_t G, const float* const* F,
                                                        const int32_t* n, const int32_t* d,
                                                        const int32_t* k, int32_t replicates,
                                                        int32_t max_iter, const uint64_t* seeds,
                                                        int32_t* const* labels,
                                                        double* inertia_out, void* ws,
                                                        size_t ws_bytes, void* stream) {
  clear_error();
  CSC_REQUIRE(G >= 1 && F && n && d && k && seeds && labels, "bad batched k-means arguments");
  for (int g = 0; g < G; ++g)
    CSC_TRY(check_args(F[g], n[g], d[g], d[g], k[g], replicates, max_iter, labels[g]));
  CSC_TRY(check_ws(ws, ws_bytes, csc_kmeans_device_workspace_bytes_batched(G, n, d, k, replicates)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  std::vector<KmPlan> P(G);
  std::vector<KmItem> all;
  std::vector<int> order;  // inputs whose seeding fits in LDS first, one seed launch per group
  for (int pass = 0; pass < 2; ++pass)
    for (int g = 0; g < G; ++g)
      if (seed_in_lds(n[g]) == (pass == 0)) order.push_back(g);
  int n_lds = 0, max_stripes = 1, max_n = 1;
  for (int g : order) {
    CSC_TRY(plan_km(ar, F[g], n[g], d[g], d[g], k[g], replicates, max_iter, seeds[g], P[g], s));
    all.insert(all.end(), P[g].items.begin(), P[g].items.end());
    if (seed_in_lds(n[g])) n_lds += replicates;
    max_stripes = std::max(max_stripes, stripes(k[g]));
    max_n = std::max(max_n, n[g]);
  }
  const int total = (int)all.size();
  KmItem* d_items = ar.take<KmItem>(all.size());
  int* flags = ar.take<int>((size_t)total * 4);
  if (!ar.ok()) {
    set_error("internal: k-means workspace overflow");
    return CSC_E_INVALID_ARG;
  }
  for (int r = 0; r < total; ++r) all[r].flags = flags + 4 * r;
  CSC_HIP(hipMemcpyAsync(d_items, all.data(), all.size() * sizeof(KmItem), hipMemcpyHostToDevice,
                         s));
  if (n_lds > 0) CSC_HIP(launch_seed(true, d_items, n_lds, s));
  if (total > n_lds) CSC_HIP(launch_seed(false, d_items + n_lds, total - n_lds, s));
  CSC_TRY(run_lloyd(d_items, total, max_stripes, max_n, max_iter, flags, s));
  for (int g = 0; g < G; ++g)
    CSC_TRY(finish_km(P[g], n[g], replicates, labels[g], inertia_out ? inertia_out + g : nullptr,
                      s));
  return CSC_OK;
}
