// Batched kernels: one launch advances the same step for G graphs of uneven
// size and width.  Workgroup b reads entry b of a work list (graph, first
// work unit, unit count), loads that graph's descriptor once and runs its
// units with the same bodies as the single-graph kernels, so results are
// bit-identical to processing the graphs one at a time.  A graph whose
// liveness flag is 0 is skipped, which lets one captured HIP graph serve
// every pass while graphs finish.
#include <algorithm>

#include "device.hpp"

namespace csc {
namespace {

using namespace dev;

template <int EPI, bool FIRST, bool LAST>
__global__ __launch_bounds__(kBlock) void kb_cheb_step(const StepArgs* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const StepArgs a = items[w.item];
  if (a.live && *a.live == 0) return;
  for (int u = w.u0; u < w.u0 + w.cnt; ++u) cheb_unit<EPI, FIRST, LAST>(a, u);
}

__global__ __launch_bounds__(kBlock) void kb_gaussian(const GaussItem* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const GaussItem it = items[w.item];
  if (it.live && *it.live == 0) return;
  const size_t total = it.L.elems();
  for (int u = w.u0; u < w.u0 + w.cnt; ++u) {
    const size_t base = (size_t)u * kElemsPerUnit;
    for (int e = threadIdx.x; e < kElemsPerUnit; e += kBlock)
      if (base + e < total) {
        if (it.nc4 > 0)
          gaussian_group_elem(it.L, it.seed, it.t, it.sid, it.nc, it.nc4, it.out, base + e);
        else
          gaussian_elem(it.L, it.seed, it.t, it.sid, it.out, base + e);
      }
  }
}

__global__ __launch_bounds__(kBlock) void kb_reduce(const ReduceItem* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const ReduceItem it = items[w.item];
  if (it.live && *it.live == 0) return;
  for (int v = w.u0; v < w.u0 + w.cnt; ++v)
    reduce_vec(it.part + (size_t)v * it.len, it.len, it.out + v);
}

__global__ __launch_bounds__(kBlock) void kb_col_dot(const ColDotItem* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const ColDotItem it = items[w.item];
  if (it.live && *it.live == 0) return;
  for (int u = w.u0; u < w.u0 + w.cnt; ++u)
    col_dot_unit(it.L, it.chunks, it.rows, it.A, it.B, it.part, u);
}

__global__ __launch_bounds__(kBlock) void kb_cg_alpha(const CgItem* items) {
  const CgItem it = items[blockIdx.x];
  if (*it.live == 0) return;
  cg_alpha_block(it.k, it.rr, it.pAp, it.active, it.alpha, it.breakdown);
}

__global__ __launch_bounds__(kBlock) void kb_cg_update1(const CgItem* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const CgItem it = items[w.item];
  if (*it.live == 0) return;
  for (int u = w.u0; u < w.u0 + w.cnt; ++u)
    cg_update1_unit(it.L, it.tiles, it.AP, it.P, it.X, it.R, it.alpha, it.part, u);
}

__global__ __launch_bounds__(kBlock) void kb_cg_scalar(const CgItem* items) {
  const CgItem it = items[blockIdx.x];
  __shared__ int was_live;
  if (threadIdx.x == 0) was_live = *it.live;
  __syncthreads();
  if (!was_live) return;
  const int itv = *it.it + 1;
  cg_scalar_block(it.k, it.rrn, it.rr, it.bnorm2, it.beta, it.active, it.iters, it.relres, itv,
                  it.tol, it.nactive);
  if (threadIdx.x == 0) {
    *it.it = itv;
    if (*it.nactive == 0 || itv >= it.max_iter) *it.live = 0;
  }
}

__global__ __launch_bounds__(kBlock) void kb_cg_update2(const CgItem* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const CgItem it = items[w.item];
  if (*it.live == 0) return;
  const size_t total4 = it.L.elems() / 4;
  for (int u = w.u0; u < w.u0 + w.cnt; ++u) {
    const size_t base = (size_t)u * kElemsPerUnit;
    for (int e = threadIdx.x; e < kElemsPerUnit; e += kBlock)
      if (base + e < total4) cg_update2_elem(it.L, it.R, it.P, it.beta, it.active, base + e);
  }
}

__global__ __launch_bounds__(kBlock) void kb_labels(const LabelItem* items, const Work* work) {
  const Work w = work[blockIdx.x];
  const LabelItem it = items[w.item];
  for (int u = w.u0; u < w.u0 + w.cnt; ++u) {
    const int i = u * kBlock + threadIdx.x;
    if (i < it.L.n) labels_row(it.L, it.X, it.colnorm2, it.labels, it.Xout, it.ldx, it.out_map, i);
  }
}

}  // namespace

void build_work(const int* units, int G, int chunk, bool xcd, std::vector<Work>& out) {
  out.clear();
  for (int g = 0; g < G; ++g) {
    const int U = units[g];
    if (!xcd) {
      for (int u = 0; u < U; u += chunk) out.push_back(Work{g, u, std::min(chunk, U - u), 0});
      continue;
    }
    // The single-graph kernels' contiguous-eighths order: XCD x walks the
    // x-th eighth of the graph's units.  Entry j of the graph's block goes to
    // XCD (j mod 8), so the block starts on a multiple of 8 and slab x's
    // chunks sit at positions x, x + 8, ...; slabs shorter than the longest
    // are padded with empty entries.
    while (out.size() % 8) out.push_back(Work{g, 0, 0, 0});
    const int q = U >> 3, r = U & 7;
    const int rounds = (q + (r ? 1 : 0) + chunk - 1) / chunk;
    for (int j = 0; j < rounds; ++j)
      for (int x = 0; x < 8; ++x) {
        const int start = x * q + (x < r ? x : r), len = q + (x < r ? 1 : 0);
        const int u0 = j * chunk;
        const int cnt = std::max(0, std::min(chunk, len - u0));
        out.push_back(Work{g, cnt ? start + u0 : 0, cnt, 0});
      }
  }
}

hipError_t launch_cheb_step_batched(const StepArgs* items, BTable t, int epi, bool first,
                                    bool last, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  const dim3 grid((unsigned)t.n), block(kBlock);
#define CSC_BSTEP(E, F, L) \
  hipLaunchKernelGGL((kb_cheb_step<E, F, L>), grid, block, 0, s, items, t.work)
  switch (epi) {
    case EPI_Y:
      if (first) { if (last) CSC_BSTEP(EPI_Y, true, true); else CSC_BSTEP(EPI_Y, true, false); }
      else { if (last) CSC_BSTEP(EPI_Y, false, true); else CSC_BSTEP(EPI_Y, false, false); }
      break;
    case EPI_MOM:
      if (first) { if (last) CSC_BSTEP(EPI_MOM, true, true); else CSC_BSTEP(EPI_MOM, true, false); }
      else { if (last) CSC_BSTEP(EPI_MOM, false, true); else CSC_BSTEP(EPI_MOM, false, false); }
      break;
    case EPI_MOMG:
      if (first) { if (last) CSC_BSTEP(EPI_MOMG, true, true); else CSC_BSTEP(EPI_MOMG, true, false); }
      else { if (last) CSC_BSTEP(EPI_MOMG, false, true); else CSC_BSTEP(EPI_MOMG, false, false); }
      break;
    case EPI_YS:
      if (first) { if (last) CSC_BSTEP(EPI_YS, true, true); else CSC_BSTEP(EPI_YS, true, false); }
      else { if (last) CSC_BSTEP(EPI_YS, false, true); else CSC_BSTEP(EPI_YS, false, false); }
      break;
    case EPI_CG:
      if (first) CSC_BSTEP(EPI_CG, true, true); else CSC_BSTEP(EPI_CG, false, true);
      break;
    case EPI_CLEN:
      if (first) CSC_BSTEP(EPI_CLEN, true, false); else CSC_BSTEP(EPI_CLEN, false, false);
      break;
    case EPI_CLEN_Y:
      if (first) CSC_BSTEP(EPI_CLEN_Y, true, false); else CSC_BSTEP(EPI_CLEN_Y, false, false);
      break;
    case EPI_CLEN_CG:
      if (first) CSC_BSTEP(EPI_CLEN_CG, true, false); else CSC_BSTEP(EPI_CLEN_CG, false, false);
      break;
    default:
      return hipErrorInvalidValue;
  }
#undef CSC_BSTEP
  return hipGetLastError();
}

hipError_t launch_gaussian_batched(const GaussItem* items, BTable t, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  hipLaunchKernelGGL(kb_gaussian, dim3((unsigned)t.n), dim3(kBlock), 0, s, items, t.work);
  return hipGetLastError();
}

hipError_t launch_reduce_batched(const ReduceItem* items, BTable t, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  hipLaunchKernelGGL(kb_reduce, dim3((unsigned)t.n), dim3(kBlock), 0, s, items, t.work);
  return hipGetLastError();
}

hipError_t launch_col_dot_batched(const ColDotItem* items, BTable t, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  hipLaunchKernelGGL(kb_col_dot, dim3((unsigned)t.n), dim3(kBlock), 0, s, items, t.work);
  return hipGetLastError();
}

hipError_t launch_cg_alpha_batched(const CgItem* items, int G, hipStream_t s) {
  hipLaunchKernelGGL(kb_cg_alpha, dim3(G), dim3(kBlock), 0, s, items);
  return hipGetLastError();
}

hipError_t launch_cg_update1_batched(const CgItem* items, BTable t, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  hipLaunchKernelGGL(kb_cg_update1, dim3((unsigned)t.n), dim3(kBlock), 0, s, items, t.work);
  return hipGetLastError();
}

hipError_t launch_cg_scalar_batched(const CgItem* items, int G, hipStream_t s) {
  hipLaunchKernelGGL(kb_cg_scalar, dim3(G), dim3(kBlock), 0, s, items);
  return hipGetLastError();
}

hipError_t launch_cg_update2_batched(const CgItem* items, BTable t, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  hipLaunchKernelGGL(kb_cg_update2, dim3((unsigned)t.n), dim3(kBlock), 0, s, items, t.work);
  return hipGetLastError();
}

hipError_t launch_labels_batched(const LabelItem* items, BTable t, hipStream_t s) {
  if (t.n < 1) return hipSuccess;
  hipLaunchKernelGGL(kb_labels, dim3((unsigned)t.n), dim3(kBlock), 0, s, items, t.work);
  return hipGetLastError();
}

}  // namespace csc
