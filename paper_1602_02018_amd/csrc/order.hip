// Node orders for locality of the gathered rows.
//
// A Chebyshev step gathers, for every node, the rows of its neighbours.  On a
// graph with communities listed in random order those rows are scattered over
// the whole block, and most gathers miss the L2 of the XCD that runs them.
// Listing the nodes community by community puts most neighbours of a node
// (all of them on a disconnected graph, Sec. 3.2.1) within the row range the
// same XCD is walking, so the gathers hit its L2.  The paper fixes no node
// order; this is a memory-layout choice and changes no result beyond the
// rounding order of float64 sums over rows.
//
// csc_community_order labels every node with the nearest centroid of the
// sampled, clustered features (the centroids of Alg. 2 step 6) and lists the
// nodes by that label, ties in index order.  csc_interpolate can run its CG on
// the graph permuted to such an order and writes its outputs back in the
// caller's order.
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "host.hpp"

namespace csc {
namespace {

constexpr int kBlk = 256;
constexpr int kLdsFloats = 12288;  // 48 KB of centroids per chunk
constexpr int kUseMax = 2048;      // centroids per chunk at most (their usable flags)

inline unsigned blocks_for(size_t n, size_t per) {
  size_t g = (n + per - 1) / per;
  return (unsigned)std::min<size_t>(std::max<size_t>(g, 1), 1u << 20);
}

__global__ void k_perm_inverse(int N, const int* order, int* inv, int* bad) {
  for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < (size_t)N;
       r += (size_t)gridDim.x * blockDim.x) {
    const int o = order[r];
    if (o < 0 || o >= N)
      atomicOr(bad, 1);
    else
      inv[o] = (int)r;
  }
}

__global__ void k_perm_check(int N, const int* inv, int* bad) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)N;
       i += (size_t)gridDim.x * blockDim.x)
    if (inv[i] < 0) atomicOr(bad, 1);
}

__global__ void k_perm_degrees(int N, const int* order, const int* row_ptr, int* deg,
                               int* row_ptr_out) {
  for (size_t r = blockIdx.x * (size_t)blockDim.x + threadIdx.x; r < (size_t)N;
       r += (size_t)gridDim.x * blockDim.x) {
    const int o = order[r];
    deg[r] = row_ptr[o + 1] - row_ptr[o];
    if (r == 0) row_ptr_out[0] = 0;
  }
}

// One wave per permuted row: the neighbours keep their CSR order, relabelled.
__global__ __launch_bounds__(kBlk) void k_perm_rows(int N, const int* order, const int* inv,
                                                    const int* row_ptr, const int* col,
                                                    const float* val, const int* row_ptr_out,
                                                    int* col_out, float* val_out) {
  const int lane = threadIdx.x & 63;
  const size_t waves = (size_t)gridDim.x * (kBlk / 64);
  for (size_t r = blockIdx.x * (size_t)(kBlk / 64) + (threadIdx.x >> 6); r < (size_t)N;
       r += waves) {
    const int o = order[r];
    const int src = row_ptr[o], len = row_ptr[o + 1] - src, dst = row_ptr_out[r];
    for (int e = lane; e < len; e += 64) {
      col_out[dst + e] = inv[col[src + e]];
      val_out[dst + e] = val[src + e];
    }
  }
}

// An index outside [0, N) maps to -1, which the consumer's own range check
// reports.
__global__ void k_map_indices(int n, int N, const int* inv, const int* idx, int* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) {
    const int i = idx[s];
    out[s] = (i >= 0 && i < N) ? inv[i] : -1;
  }
}

__global__ void k_gather_rows(int n, int d, const float* F, size_t ldf, const int* rows, int N,
                              float* out, int ldo, int* bad) {
  const size_t total = (size_t)n * d;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int s = (int)(e / d), j = (int)(e - (size_t)s * d);
    const int i = rows[s];
    if (i < 0 || i >= N) {
      if (j == 0) atomicOr(bad, 1);
      continue;
    }
    out[(size_t)s * ldo + j] = F[(size_t)i * ldf + j];
  }
}

__global__ void k_iota(int N, int* out) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)N;
       i += (size_t)gridDim.x * blockDim.x)
    out[i] = (int)i;
}

// Nearest usable centroid of every row of F (squared Euclidean distance,
// coordinates summed in order, ties to the lowest index).  A thread keeps its
// row in registers; centroids are staged through LDS in chunks, each row
// padded with zeros to DMAX coordinates like the thread's own, so that the
// distance loop runs the same DMAX steps for every d (a padded step adds
// (0 - 0)^2 = 0 to a sum of squares, which leaves it unchanged) and its LDS
// reads need no guard and can all be in flight at once.
template <int DMAX>
__global__ __launch_bounds__(kBlk) void k_nearest_centroid(int N, int d, const float* F,
                                                           size_t ldf, const float* C,
                                                           const int* usable, int k,
                                                           int* labels) {
  static_assert(DMAX % 4 == 0 && DMAX <= kLdsFloats, "padded centroid rows");
  __shared__ __align__(16) float cs[kLdsFloats];
  __shared__ int use[kUseMax];
  const int i = blockIdx.x * kBlk + threadIdx.x;
  const bool row = i < N;
  float f[DMAX];
#pragma unroll
  for (int j = 0; j < DMAX; ++j) f[j] = (row && j < d) ? F[(size_t)i * ldf + j] : 0.f;
  constexpr int kc = kUseMax < kLdsFloats / DMAX ? kUseMax : kLdsFloats / DMAX;
  float best = 0.f;
  int arg = 0;
  bool found = false;
  for (int c0 = 0; c0 < k; c0 += kc) {
    const int nc = min(kc, k - c0);
    __syncthreads();
    for (int e = threadIdx.x; e < nc * DMAX; e += kBlk) {
      const int c = e / DMAX, j = e - c * DMAX;
      cs[e] = j < d ? C[(size_t)(c0 + c) * d + j] : 0.f;
    }
    for (int e = threadIdx.x; e < nc; e += kBlk) use[e] = usable[c0 + e];
    __syncthreads();
    if (row) {
      for (int c = 0; c < nc; c += 2) {
        const bool two = c + 1 < nc;
        const float* ca = cs + c * DMAX;
        const float* cb = cs + (two ? c + 1 : c) * DMAX;
        float da = 0.f, db = 0.f;
#pragma unroll
        for (int j = 0; j < DMAX; ++j) {
          const float ta = f[j] - ca[j], tb = f[j] - cb[j];
          da = fmaf(ta, ta, da);
          db = fmaf(tb, tb, db);
        }
        if (use[c] && (!found || da < best)) {
          best = da;
          arg = c0 + c;
          found = true;
        }
        if (two && use[c + 1] && (!found || db < best)) {
          best = db;
          arg = c0 + c + 1;
          found = true;
        }
      }
    }
  }
  if (row) labels[i] = arg;
}

// Number of stored edges whose two ends carry the same label (integer atomics:
// the count does not depend on the order of the additions).
__global__ void k_same_label_edges(int N, const int* row_ptr, const int* col, const int* lab,
                                   unsigned long long* count) {
  unsigned long long c = 0;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)N;
       i += (size_t)gridDim.x * blockDim.x) {
    const int li = lab[i];
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) c += lab[col[e]] == li;
  }
  if (c) atomicAdd(count, c);
}

// Exponential-race keys of variable-density sampling: E_i / w_i with
// E_i = -ln(u_i), u_i = ((x0 >> 11) + 1) 2^-53 from Philox at counter
// (i, 1, SAMPLE, 0); +inf when w_i is not positive.  A positive double's bits
// order like the double, so the keys sort as unsigned integers.
__global__ void k_density_keys(int N, const double* w, uint64_t seed, uint64_t* keys, int* vals) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < (size_t)N;
       i += (size_t)gridDim.x * blockDim.x) {
    const Words4 x = philox4x64_10((uint64_t)i, 1ull, (uint64_t)CSC_STREAM_SAMPLE, 0ull, seed, 0ull);
    const double u = (double)((x.x0 >> 11) + 1ull) * 0x1p-53;
    const double wi = w[i];
    const double key = (wi > 0.0 && wi <= 1.7976931348623157e308) ? -log(u) / wi : __builtin_inf();
    keys[i] = (uint64_t)__double_as_longlong(key);
    vals[i] = (int)i;
  }
}

// Per-block float64 partial sums over contiguous ranges (fixed order).
__global__ __launch_bounds__(kBlk) void k_sum_parts(const double* x, int N, int per, double* part) {
  __shared__ double sh[kBlk / 64];
  const int b = blockIdx.x;
  const size_t lo = (size_t)b * per, hi = min((size_t)N, lo + per);
  double acc = 0.0;
  for (size_t i = lo + threadIdx.x; i < hi; i += kBlk) acc += x[i];
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlk / 64; ++w) t += sh[w];
    part[b] = t;
  }
}

__global__ void k_sum_final(const double* part, int nparts, double* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double t = 0.0;
    for (int b = 0; b < nparts; ++b) t += part[b];
    *out = t;
  }
}

// decoder weight 1 / (N p_i) = (sum(w) / N) / w_i of every sampled node
__global__ void k_decoder_weights(int n, const int* idx, const double* w, const double* sum, int N,
                                  float* out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double wi = w[idx[s]];
  out[s] = wi > 0.0 ? (float)((*sum / (double)N) / wi) : 0.f;
}

// Degree skew of the natural row order: acc[0] += max degree of each group of
// 8 consecutive rows, acc[1] += degrees (integer sums, so order-free).
__global__ __launch_bounds__(256) void k_wave_skew(int n, const int* row_ptr,
                                                   unsigned long long* acc) {
  __shared__ unsigned long long sh[2][256];
  const int grp = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long mx = 0, sum = 0;
  for (int r = grp * 8; r < min(n, grp * 8 + 8); ++r) {
    const unsigned long long dg = (unsigned)(row_ptr[r + 1] - row_ptr[r]);
    mx = dg > mx ? dg : mx;
    sum += dg;
  }
  sh[0][threadIdx.x] = mx;
  sh[1][threadIdx.x] = sum;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicAdd(acc, sh[0][0]);
    atomicAdd(acc + 1, sh[1][0]);
  }
}

// Row schedule: block b sorts the rows of chunk b by (decreasing degree,
// index) with a bitonic network on 64-bit keys in LDS (padding keys sort
// last) and writes them back in that order.
__global__ __launch_bounds__(256) void k_row_schedule(int n, const int* row_ptr, int* sched) {
  __shared__ unsigned long long key[kSchedChunk];
  const int base = blockIdx.x * kSchedChunk;
  const int cnt = min(kSchedChunk, n - base);
  for (int e = threadIdx.x; e < kSchedChunk; e += blockDim.x) {
    unsigned long long v = ~0ull;
    if (e < cnt) {
      const unsigned deg = (unsigned)(row_ptr[base + e + 1] - row_ptr[base + e]);
      v = ((unsigned long long)(0xFFFFFFFFu - deg) << 32) | (unsigned)e;
    }
    key[e] = v;
  }
  __syncthreads();
  for (int size = 2; size <= kSchedChunk; size <<= 1)
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int e = threadIdx.x; e < kSchedChunk / 2; e += blockDim.x) {
        const int lo = 2 * e - (e & (stride - 1)), hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long x = key[lo], y = key[hi];
        if ((x > y) == up) {
          key[lo] = y;
          key[hi] = x;
        }
      }
      __syncthreads();
    }
  for (int e = threadIdx.x; e < cnt; e += blockDim.x)
    sched[base + e] = base + (int)(key[e] & 0xFFFFFFFFull);
}

}  // namespace

hipError_t launch_density_keys(int N, const double* w, uint64_t seed, uint64_t* keys, int* vals,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_density_keys, dim3(blocks_for(N, kBlk)), dim3(kBlk), 0, s, N, w, seed, keys,
                     vals);
  return hipGetLastError();
}

hipError_t launch_sum_f64(const double* x, int N, double* part, int nparts, double* out,
                          hipStream_t s) {
  const int per = (N + nparts - 1) / nparts;
  hipLaunchKernelGGL(k_sum_parts, dim3((unsigned)nparts), dim3(kBlk), 0, s, x, N, per, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(64), 0, s, part, nparts, out);
  return hipGetLastError();
}

hipError_t launch_decoder_weights(int n, const int* idx, const double* w, const double* sum, int N,
                                  float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_decoder_weights, dim3((n + kBlk - 1) / kBlk), dim3(kBlk), 0, s, n, idx, w,
                     sum, N, out);
  return hipGetLastError();
}

hipError_t launch_perm_inverse(int N, const int* order, int* inv, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_inverse, dim3(blocks_for(N, kBlk)), dim3(kBlk), 0, s, N, order, inv,
                     bad);
  return hipGetLastError();
}

hipError_t launch_perm_check(int N, const int* inv, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_check, dim3(blocks_for(N, kBlk)), dim3(kBlk), 0, s, N, inv, bad);
  return hipGetLastError();
}

size_t perm_graph_temp_bytes(int N) {
  size_t bytes = 0;  // a failed query leaves 0, and the scan then reports the error
  (void)hipcub::DeviceScan::InclusiveSum(nullptr, bytes, (const int*)nullptr, (int*)nullptr, N);
  return bytes;
}

hipError_t perm_graph(int N, const int* order, const int* inv, const int* row_ptr, const int* col,
                      const float* val, int* row_ptr_out, int* col_out, float* val_out, int* deg,
                      void* temp, size_t temp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(k_perm_degrees, dim3(blocks_for(N, kBlk)), dim3(kBlk), 0, s, N, order,
                     row_ptr, deg, row_ptr_out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = hipcub::DeviceScan::InclusiveSum(temp, temp_bytes, deg, row_ptr_out + 1, N, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_perm_rows, dim3(blocks_for(N, kBlk / 64)), dim3(kBlk), 0, s, N, order, inv,
                     row_ptr, col, val, row_ptr_out, col_out, val_out);
  return hipGetLastError();
}

hipError_t launch_map_indices(int n, int N, const int* inv, const int* idx, int* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_map_indices, dim3((n + kBlk - 1) / kBlk), dim3(kBlk), 0, s, n, N, inv, idx,
                     out);
  return hipGetLastError();
}

hipError_t launch_gather_rows(int n, int d, const float* F, size_t ldf, const int* rows, int N,
                              float* out, int ldo, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks_for((size_t)n * d, kBlk)), dim3(kBlk), 0, s, n, d,
                     F, ldf, rows, N, out, ldo, bad);
  return hipGetLastError();
}

hipError_t launch_nearest_centroid(int N, int d, const float* F, size_t ldf, const float* C,
                                   const int* usable, int k, int* labels, hipStream_t s) {
  const dim3 grid((unsigned)((N + kBlk - 1) / kBlk)), block(kBlk);
  // the padded width: the smallest instance that holds d (the padding is work)
  if (d <= 32)
    hipLaunchKernelGGL(k_nearest_centroid<32>, grid, block, 0, s, N, d, F, ldf, C, usable, k,
                       labels);
  else if (d <= 48)
    hipLaunchKernelGGL(k_nearest_centroid<48>, grid, block, 0, s, N, d, F, ldf, C, usable, k,
                       labels);
  else if (d <= 56)
    hipLaunchKernelGGL(k_nearest_centroid<56>, grid, block, 0, s, N, d, F, ldf, C, usable, k,
                       labels);
  else if (d <= 64)
    hipLaunchKernelGGL(k_nearest_centroid<64>, grid, block, 0, s, N, d, F, ldf, C, usable, k,
                       labels);
  else if (d <= 96)
    hipLaunchKernelGGL(k_nearest_centroid<96>, grid, block, 0, s, N, d, F, ldf, C, usable, k,
                       labels);
  else
    hipLaunchKernelGGL(k_nearest_centroid<128>, grid, block, 0, s, N, d, F, ldf, C, usable, k,
                       labels);
  return hipGetLastError();
}

size_t sort_labels_temp_bytes(int N) {
  size_t bytes = 0;  // a failed query leaves 0, and the sort then reports the error
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, (const unsigned*)nullptr,
                                           (unsigned*)nullptr, (const int*)nullptr, (int*)nullptr,
                                           N);
  return bytes;
}

hipError_t sort_labels(void* temp, size_t temp_bytes, const int* kin, int* kout, const int* vin,
                       int* vout, int N, int key_bits, hipStream_t s) {
  // LSD radix sort: stable, so equal labels keep their index order
  return hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, (const unsigned*)kin,
                                            (unsigned*)kout, vin, vout, N, 0, key_bits, s);
}

hipError_t launch_iota(int N, int* out, hipStream_t s) {
  hipLaunchKernelGGL(k_iota, dim3(blocks_for(N, kBlk)), dim3(kBlk), 0, s, N, out);
  return hipGetLastError();
}

hipError_t launch_row_schedule(int n, const int* row_ptr, int* sched, hipStream_t s) {
  if (n < 1) return hipSuccess;
  hipLaunchKernelGGL(k_row_schedule, dim3((unsigned)((n + kSchedChunk - 1) / kSchedChunk)),
                     dim3(256), 0, s, n, row_ptr, sched);
  return hipGetLastError();
}

}  // namespace csc

using namespace csc;

extern "C" csc_status csc_row_schedule(int32_t n, const int32_t* row_ptr, int32_t* sched,
                                       double* skew_out, void* ws, size_t ws_bytes,
                                       void* stream) {
  clear_error();
  CSC_REQUIRE(n >= 1, "n must be >= 1");
  CSC_REQUIRE(row_ptr && sched, "row_ptr and sched must be non-NULL");
  if (skew_out) CSC_TRY(check_ws(ws, ws_bytes, 2 * sizeof(unsigned long long)));
  hipStream_t s = as_stream(stream);
  CSC_HIP(launch_row_schedule(n, row_ptr, sched, s));
  if (skew_out) {
    unsigned long long* acc = static_cast<unsigned long long*>(ws);
    CSC_HIP(launch_fill_i32(reinterpret_cast<int*>(acc), 4, 0, s));
    const int groups = (n + 7) / 8;
    hipLaunchKernelGGL(k_wave_skew, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, n,
                       row_ptr, acc);
    CSC_HIP(hipGetLastError());
    unsigned long long h[2] = {0, 0};
    CSC_HIP(hipMemcpyAsync(h, acc, sizeof(h), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    *skew_out = h[1] ? 8.0 * (double)h[0] / (double)h[1] : 1.0;
  }
  return CSC_OK;
}

extern "C" csc_status csc_gather_rows(const float* F, int64_t ldf, int32_t N, int32_t d,
                                      const int32_t* rows, int32_t n, float* out, int32_t ldo,
                                      void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  CSC_REQUIRE(N >= 1 && d >= 1 && ldf >= d && n >= 0 && ldo >= d,
              "need N >= 1, d >= 1, ldf >= d, n >= 0 and ldo >= d");
  CSC_REQUIRE(F && (rows || n == 0) && (out || n == 0), "F, rows and out must be non-NULL");
  CSC_TRY(check_ws(ws, ws_bytes, 256));
  if (n == 0) return CSC_OK;
  hipStream_t s = as_stream(stream);
  int* bad = static_cast<int*>(ws);
  CSC_HIP(launch_fill_i32(bad, 1, 0, s));
  CSC_HIP(launch_gather_rows(n, d, F, (size_t)ldf, rows, N, out, ldo, bad, s));
  int hbad = 0;
  CSC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  CSC_REQUIRE(!hbad, "rows holds an index outside [0, N)");
  return CSC_OK;
}

namespace {
size_t order_bytes(int N, int d, int k, int n) {
  size_t b = align_up((size_t)n * d * sizeof(float));         // sampled rows
  b += align_up((size_t)k * d * sizeof(float));               // centroids
  b += align_up((size_t)k * sizeof(int));                     // usable
  b += 4 * align_up((size_t)N * sizeof(int));                 // labels, sorted labels, iota, out
  b += align_up(sort_labels_temp_bytes(N)) + align_up(4 * sizeof(int));
  return b + 256;
}
}  // namespace

extern "C" size_t csc_community_order_workspace_bytes(int32_t N, int32_t d, int32_t k,
                                                      int32_t n) {
  if (N < 1 || d < 1 || k < 1 || n < 1) return 0;
  return order_bytes(N, d, k, n);
}

extern "C" csc_status csc_community_order(const csc_graph* g, const float* F, int64_t ldf,
                                          int32_t d, const int32_t* idx,
                                          const int32_t* labels_r, int32_t n, int32_t k,
                                          int32_t* order, int32_t* node_labels,
                                          double* same_label_frac, void* ws, size_t ws_bytes,
                                          void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  const int32_t N = g->n;
  CSC_REQUIRE(d >= 1 && d <= 128 && ldf >= d, "need 1 <= d <= 128 and ldf >= d");
  CSC_REQUIRE(k >= 1 && n >= 1 && n <= N, "need k >= 1 and 1 <= n <= N");
  CSC_REQUIRE(F && idx && labels_r && order, "F, idx, labels_r and order must be non-NULL");
  for (int s = 0; s < n; ++s)
    CSC_REQUIRE(labels_r[s] >= 0 && labels_r[s] < k, "labels_r holds a value outside [0, k)");
  CSC_TRY(check_ws(ws, ws_bytes, order_bytes(N, d, k, n)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  float* Fs = ar.take<float>((size_t)n * d);
  float* C = ar.take<float>((size_t)k * d);
  int* usable = ar.take<int>(k);
  int* lab = ar.take<int>(N);
  int* lab_sorted = ar.take<int>(N);
  int* iota = ar.take<int>(N);
  int* out = ar.take<int>(N);
  const size_t temp_bytes = sort_labels_temp_bytes(N);
  void* temp = ar.take<char>(temp_bytes);
  int* bad = ar.take<int>(4);

  // centroids of the clustered sampled rows, summed in sample order in float64
  CSC_HIP(launch_fill_i32(bad, 1, 0, s));
  CSC_HIP(launch_gather_rows(n, d, F, (size_t)ldf, idx, N, Fs, d, bad, s));
  std::vector<float> hF((size_t)n * d);
  int hbad = 0;
  CSC_HIP(hipMemcpyAsync(hF.data(), Fs, hF.size() * sizeof(float), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  CSC_REQUIRE(!hbad, "idx holds an index outside [0, N)");
  std::vector<double> sum((size_t)k * d, 0.0);
  std::vector<int> cnt(k, 0);
  for (int r = 0; r < n; ++r) {
    const int c = labels_r[r];
    ++cnt[c];
    for (int j = 0; j < d; ++j) sum[(size_t)c * d + j] += (double)hF[(size_t)r * d + j];
  }
  std::vector<float> hC((size_t)k * d, 0.f);
  for (int c = 0; c < k; ++c)
    if (cnt[c] > 0)
      for (int j = 0; j < d; ++j) hC[(size_t)c * d + j] = (float)(sum[(size_t)c * d + j] / cnt[c]);
  std::vector<int> hu(k);
  for (int c = 0; c < k; ++c) hu[c] = cnt[c] > 0 ? 1 : 0;
  CSC_HIP(hipMemcpyAsync(C, hC.data(), hC.size() * sizeof(float), hipMemcpyHostToDevice, s));
  CSC_HIP(hipMemcpyAsync(usable, hu.data(), k * sizeof(int), hipMemcpyHostToDevice, s));

  CSC_HIP(launch_nearest_centroid(N, d, F, (size_t)ldf, C, usable, k, lab, s));
  CSC_HIP(launch_iota(N, iota, s));
  int bits = 1;
  while (bits < 31 && (1 << bits) < k) ++bits;
  CSC_HIP(sort_labels(temp, temp_bytes, lab, lab_sorted, iota, out, N, bits, s));
  CSC_HIP(hipMemcpyAsync(order, out, (size_t)N * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (node_labels)
    CSC_HIP(hipMemcpyAsync(node_labels, lab, (size_t)N * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (same_label_frac) {
    unsigned long long* cnt = reinterpret_cast<unsigned long long*>(bad);
    CSC_HIP(launch_fill_i32(bad, 2, 0, s));  // the 64-bit counter
    if (g->nnz > 0) {
      hipLaunchKernelGGL(k_same_label_edges, dim3(blocks_for(N, kBlk)), dim3(kBlk), 0, s, N,
                         g->row_ptr, g->col, lab, cnt);
      CSC_HIP(hipGetLastError());
    }
    unsigned long long h = 0;
    CSC_HIP(hipMemcpyAsync(&h, cnt, sizeof(h), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    *same_label_frac = g->nnz > 0 ? (double)h / (double)g->nnz : 0.0;
  }
  CSC_HIP(hipStreamSynchronize(s));
  return CSC_OK;
}

namespace {
constexpr int kSumParts = 256;
size_t density_bytes(int N) {
  size_t b = 2 * align_up((size_t)N * sizeof(uint64_t)) + 2 * align_up((size_t)N * sizeof(int));
  b += align_up(sort_pairs_temp_bytes(N)) + align_up(kSumParts * sizeof(double));
  return b + align_up(4 * sizeof(double)) + 256;
}
}  // namespace

extern "C" size_t csc_sample_density_workspace_bytes(int32_t N) {
  if (N < 1) return 0;
  return density_bytes(N);
}

extern "C" csc_status csc_sample_density(int32_t N, int32_t n, uint64_t seed, const double* w,
                                         int32_t* idx, float* dec_weights, void* ws,
                                         size_t ws_bytes, void* stream) {
  clear_error();
  CSC_REQUIRE(N >= 1 && n >= 1 && n <= N, "need 1 <= n <= N");
  CSC_REQUIRE(w && idx, "w and idx must be non-NULL");
  CSC_TRY(check_ws(ws, ws_bytes, density_bytes(N)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  uint64_t* kin = ar.take<uint64_t>(N);
  uint64_t* kout = ar.take<uint64_t>(N);
  int* vin = ar.take<int>(N);
  int* vout = ar.take<int>(N);
  const size_t temp_bytes = sort_pairs_temp_bytes(N);
  void* temp = ar.take<char>(temp_bytes);
  double* part = ar.take<double>(kSumParts);
  double* sum = ar.take<double>(4);
  CSC_HIP(launch_density_keys(N, w, seed, kin, vin, s));
  CSC_HIP(sort_pairs(temp, temp_bytes, kin, kout, vin, vout, N, s));
  CSC_HIP(hipMemcpyAsync(idx, vout, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
  if (dec_weights) {
    CSC_HIP(launch_sum_f64(w, N, part, std::min(kSumParts, N), sum, s));
    CSC_HIP(launch_decoder_weights(n, vout, w, sum, N, dec_weights, s));
  }
  CSC_HIP(hipStreamSynchronize(s));
  return CSC_OK;
}

extern "C" csc_status csc_normalize_rows(float* Y, int64_t ld, int32_t n_rows, int32_t d,
                                         double* sqnorm, void* stream) {
  clear_error();
  CSC_REQUIRE(n_rows >= 0 && d >= 1 && ld >= d, "need n_rows >= 0, d >= 1, ld >= d");
  CSC_REQUIRE(Y || n_rows == 0, "Y is NULL");
  if (n_rows == 0) return CSC_OK;
  CSC_HIP(launch_normalize_rows(n_rows, d, Y, (int)ld, as_stream(stream), sqnorm));
  return CSC_OK;
}
