// Launch wrappers of the libcsc device kernels (kernels.hip).
#pragma once

#include <vector>

#include "common.hpp"

namespace csc {

enum Epi : int {
  EPI_Y = 0,    // Y (panel-major) accumulates coefficient * T_{m+1}
  EPI_MOM = 1,  // float64 partials of <T_m, T_{m+1}> and <T_{m+1}, T_{m+1}> per workgroup
  EPI_YS = 2,   // only sampled rows accumulate, straight into a node-major output
  EPI_CG = 3,   // last step of the CG operator: AP = mask*P + gamma*(P - h~(L)P)
  // Clenshaw's backward recurrence (b_m = c0 R + c1 A b_{m+1} - b_{m+2}, with
  // T0 = R, Tm = b_{m+1}, Tprev = b_{m+2}, Tnext = b_m); FIRST = no b_{m+2}
  EPI_CLEN = 4,     // intermediate b_m
  EPI_CLEN_Y = 5,   // final step: Y = h~(L) R
  EPI_CLEN_CG = 6,  // final step of the CG operator, as EPI_CG
  EPI_MOMG = 7,     // EPI_MOM for a group of eigencount tests side by side (mgroup > 1)
  EPI_SPMM = 8,     // measurement only: Tnext = A Tm (the gathers, one block written)
};

// Eigencount tests whose passes one EPI_MOMG launch may carry side by side.
constexpr int kMaxCountGroup = 4;

// Moment partial sums per work unit (EPI_MOM, EPI_MOMG): one per wave of the
// 256-thread workgroup, so that no wave waits for the others of its
// workgroup (on skewed degrees their rows end at very different times).  The
// partial of wave v of unit u sits at index u * kMomSlots + v.
constexpr int kMomSlots = 4;

struct StepArgs {
  Layout L;
  int tiles = 0;  // row tiles per panel
  const int* row_ptr = nullptr;
  const int* col = nullptr;
  const float* val = nullptr;
  const int* sched = nullptr;    // row walk (a permutation of [0, n)) or NULL
  const float* Tm = nullptr;     // T_m, gathered through A
  const float* Tprev = nullptr;  // T_{m-1}; on the first step T_0
  float* Tnext = nullptr;        // T_{m+1} (may alias Tprev)
  const float* T0 = nullptr;     // T_0 (moments, CG)
  float* Y = nullptr;            // accumulator (EPI_Y, EPI_CG)
  float c0 = 0.f, c1 = 0.f;      // first step: Y = c0 T_0 + c1 T_1; later: Y += c1 T_{m+1}
  double* part = nullptr;        // partial sums (EPI_MOM: of <T_m, T_{m+1}>, kMomSlots per unit)
  double* part2 = nullptr;       // EPI_MOM: partial of <T_{m+1}, T_{m+1}>
  double* part0 = nullptr;       // EPI_MOM, first step: partial of <T_0, T_0>
  const int* slot = nullptr;     // EPI_YS: output row of node i or -1
  float* Ys = nullptr;
  int lds = 0;
  const float* mask = nullptr;   // EPI_CG
  float gamma = 0.f;
  int xcd = 0;                   // XCD-aware work-unit order
  int nt = 0;                    // non-temporal loads/stores for streamed blocks
  const int* live = nullptr;     // batched launches: skip the graph when *live == 0
  // EPI_MOMG: mgroup eigencount passes side by side (pass j in columns
  // [j mnc4, (j + 1) mnc4), mnc4 a multiple of 4); pass j's partial sums go
  // to part / part2 / part0 + j mstride
  int mgroup = 1;
  int mnc4 = 0;
  size_t mstride = 0;
};

// ------------------------------------------------------- batched launches --
// A batched launch covers G items (graphs).  Its work list has one entry per
// workgroup: (item, first local work unit, number of units), so a workgroup
// reads one entry and one descriptor and then runs up to kChunk consecutive
// units of that item with the same bodies as the single-graph kernels.
struct Work {
  int item, u0, cnt, pad;
};

struct BTable {
  const Work* work = nullptr;
  int n = 0;  // entries (= workgroups)
};

struct GaussItem {
  Layout L;
  uint64_t seed = 0;
  uint32_t t = 0, sid = 0;
  float* out = nullptr;
  const int* live = nullptr;
  int nc = 0, nc4 = 0;  // nc4 > 0: tests t, t + 1, ... side by side, nc4 columns each
};

// one item per graph; its units are its nvec vectors
struct ReduceItem {
  const double* part = nullptr;
  int len = 0;
  double* out = nullptr;
  const int* live = nullptr;
};

struct ColDotItem {
  Layout L;
  int chunks = 0;  // col_dot_chunks(L)
  int rows = 0;    // col_dot_rows(L)
  const float* A = nullptr;
  const float* B = nullptr;
  double* part = nullptr;
  const int* live = nullptr;
};

struct CgItem {
  Layout L;
  int tiles = 0;
  int k = 0;
  const float* AP = nullptr;
  float* P = nullptr;
  float* X = nullptr;
  float* R = nullptr;
  double* rr = nullptr;
  double* rrn = nullptr;
  double* pAp = nullptr;
  double* alpha = nullptr;
  double* beta = nullptr;
  const double* bnorm2 = nullptr;
  int* active = nullptr;
  int* iters = nullptr;
  double* relres = nullptr;
  double* part = nullptr;        // per-column partials (columns x tiles)
  int* nactive = nullptr;
  int* breakdown = nullptr;
  int* it = nullptr;             // iterations done by this graph
  double tol = 0.0;
  int max_iter = 0;
  int* live = nullptr;           // cleared once no column iterates
};

struct LabelItem {
  Layout L;
  const float* X = nullptr;
  const double* colnorm2 = nullptr;
  int* labels = nullptr;
  float* Xout = nullptr;
  int ldx = 0;
  const int* out_map = nullptr;  // layout row i is node out_map[i] (NULL: i)
};

hipError_t launch_cheb_step_batched(const StepArgs* items, BTable t, int epi, bool first,
                                    bool last, hipStream_t s);
hipError_t launch_gaussian_batched(const GaussItem* items, BTable t, hipStream_t s);
hipError_t launch_reduce_batched(const ReduceItem* items, BTable t, hipStream_t s);
hipError_t launch_col_dot_batched(const ColDotItem* items, BTable t, hipStream_t s);
hipError_t launch_cg_alpha_batched(const CgItem* items, int G, hipStream_t s);
hipError_t launch_cg_update1_batched(const CgItem* items, BTable t, hipStream_t s);
hipError_t launch_cg_scalar_batched(const CgItem* items, int G, hipStream_t s);
hipError_t launch_cg_update2_batched(const CgItem* items, BTable t, hipStream_t s);
hipError_t launch_labels_batched(const LabelItem* items, BTable t, hipStream_t s);
constexpr int kElemsPerUnit = 1024;  // gaussian / update2 / labels: elements per work unit

// Work list for per-item unit counts, chunks of up to `chunk` units.
void build_work(const int* units, int G, int chunk, bool xcd, std::vector<Work>& out);

// Process-wide kernel tuning (csc_set_tuning).
struct Tuning {
  int xcd = 1;
  int nt = 0;
};
Tuning tuning();

int rows_per_tile(int pw);
int tiles_for(const Layout& L);

hipError_t launch_cheb_step(const StepArgs& a, int epi, bool first, bool last, hipStream_t s);

// Laplacian scaling.
hipError_t launch_degree_scale(int n, const int* row_ptr, const int* col, const float* w,
                               float* dinv_sqrt, hipStream_t s);
hipError_t launch_adjacency_values(int n, const int* row_ptr, const int* col, const float* w,
                                   const float* dinv_sqrt, float* val, hipStream_t s);
hipError_t launch_check_graph_strict(int n, const int* row_ptr, const int* col, const float* w,
                                     int* flag, hipStream_t s);
hipError_t launch_check_csr(int n, int nnz, const int* row_ptr, const int* col, int* flag,
                            hipStream_t s);

// Random blocks.
// The signals of passes t, t + 1, ..., t + G - 1 (each an n x nc block of
// sub-stream t + j, exactly as launch_gaussian_panels draws it) side by side:
// pass j in columns [j nc4, j nc4 + nc) of the G nc4-column layout L, the
// other columns zero.
hipError_t launch_gaussian_group(const Layout& L, uint64_t seed, uint32_t t, uint32_t stream_id,
                                 int nc, int nc4, float* out, hipStream_t s);
hipError_t launch_gaussian_panels(const Layout& L, uint64_t seed, uint32_t t, uint32_t stream_id,
                                  float* out, hipStream_t s);
hipError_t launch_gaussian_rows(int n_rows, int w, uint64_t seed, uint32_t t, uint32_t stream_id,
                                float* R, int ld, hipStream_t s);

// Layout conversion and row scaling.
hipError_t launch_pack(const Layout& L, const float* X, int ld, float* out, hipStream_t s);
// columns [0, wc) between a wide layout Lw and a compact layout Lc of the same rows
hipError_t launch_to_compact(const Layout& Lc, float* dst, const Layout& Lw, const float* src,
                             int wc, hipStream_t s);
hipError_t launch_from_compact(const Layout& Lc, const float* src, const Layout& Lw, float* dst,
                               int wc, hipStream_t s);
hipError_t launch_unpack(const Layout& L, const float* in, float* Y, int ld, int normalize,
                         hipStream_t s);
hipError_t launch_normalize_rows(int n_rows, int w, float* Y, int ld, hipStream_t s,
                                double* sq = nullptr);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int* p, size_t n, int v, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_slot_map(int n_rows, const int* rows, int n, int* slot, int* bad,
                           hipStream_t s);

// Deterministic reductions: out[v] = sum_t part[v * len + t], fixed order.
hipError_t launch_reduce(const double* part, int len, int nvec, double* out, hipStream_t s);
// part[c * chunks + chunk] = sum over the chunk's rows of A(i, c) * B(i, c),
// chunks = col_dot_chunks(L) (at most tiles_for(L)) of col_dot_rows(L) rows;
// launch_reduce(part, col_dot_chunks(L), w, out) then gives the column sums.
int col_dot_chunks(const Layout& L);
int col_dot_rows(const Layout& L);
hipError_t launch_col_dot(const Layout& L, const float* A, const float* B, double* part,
                          hipStream_t s);

// Sampling by smallest keys.
int sample_chunks(int N);
hipError_t launch_sample_count(int N, uint64_t seed, uint64_t thresh, int* counts, hipStream_t s);
hipError_t launch_scan_counts(const int* counts, int nchunks, int* offsets, int* total,
                              hipStream_t s);
hipError_t launch_sample_write(int N, uint64_t seed, uint64_t thresh, const int* offsets,
                               uint64_t* keys, int* idx, hipStream_t s);
size_t sort_pairs_temp_bytes(int count);
hipError_t sort_pairs(void* temp, size_t temp_bytes, const uint64_t* kin, uint64_t* kout,
                      const int* vin, int* vout, int count, hipStream_t s);

// Conjugate gradient.
hipError_t launch_cg_scatter(const Layout& L, int n, const int* idx, const int* lab,
                             const float* wts, float* R, float* P, float* mask, int* bad,
                             hipStream_t s);
hipError_t launch_cg_alpha(int k, const double* rr, const double* pAp, int* active,
                           double* alpha, int* breakdown, hipStream_t s);
hipError_t launch_cg_update1(const Layout& L, const float* AP, const float* P, float* X, float* R,
                             const double* alpha, double* part, hipStream_t s);
hipError_t launch_cg_scalar(int k, const double* rrn, double* rr, const double* bnorm2,
                            double* beta, int* active, int* iters, double* relres, int it,
                            double tol, int* nactive, hipStream_t s);
hipError_t launch_cg_update2(const Layout& L, const float* R, float* P, const double* beta,
                             const int* active, hipStream_t s);
hipError_t launch_labels(const Layout& L, const float* X, const double* colnorm2, int* labels,
                         float* Xout, int ldx, const int* out_map, hipStream_t s);

// Block products (block.hip).  Gram G = A^T B of the first ka and kb columns
// of two N-row panel-major blocks (float64 sums in a fixed order, row-major
// with leading dimension ldg); part holds gram_part_elems(L, max(ka, kb))
// doubles.  lower (ka == kb): only the 128 x 128 tiles on and below the
// diagonal are summed, and an entry above them is set to its mirror, which
// a Gram that is symmetric (A = B) or whose upper triangle is never read
// does not notice.  amask, bmask: bit t set when 128-column tile t of A (B)
// is read afterwards; the other tiles' entries are left unspecified (all
// bits are taken as set past 64 tiles).  Block product Out = c0 In0 +
// In1[:, :kin] S with S float64 kin x kout (leading dimension lds), every
// stored column written, except the 128-column tiles whose bit in cmask is
// clear, which keep their contents.
constexpr int kBlockTile = 128;  // column tile of the Gram and block-product kernels
struct GramPlan {
  int tiles_a = 0, tiles_b = 0, tiles = 0, chunks = 0, rows_per_chunk = 0;
  bool lower = false;
};
GramPlan gram_plan(const Layout& L, int ka, int kb, bool lower = false);
size_t gram_part_elems(const Layout& L, int kmax);
hipError_t launch_gram(const Layout& L, const float* A, const float* B, int ka, int kb,
                       double* part, double* G, int ldg, hipStream_t s, bool lower = false,
                       uint64_t amask = ~0ull, uint64_t bmask = ~0ull);
// Z = R / (mask_i + gamma) row by row (Jacobi preconditioner of the interpolation).
hipError_t launch_jacobi(const Layout& L, const float* R, const float* mask, float gamma, float* Z,
                         hipStream_t s);
// CSC_TUNE_BLOCK_PRODUCT: block products with float32 sums (true) or float64 sums
bool block_product_f32();
// f32: float32 sums for this product whatever the knob says
hipError_t launch_block_mul(const Layout& L, float c0, const float* In0, const float* In1,
                            const double* S, int kin, int kout, int lds, float* Out,
                            hipStream_t s, bool f32 = false, uint64_t cmask = ~0ull);

// Row schedule of a CSR graph (order.hip): chunks of kSchedChunk rows, each
// by decreasing degree, ties by index.
constexpr int kSchedChunk = 4096;
hipError_t launch_row_schedule(int n, const int* row_ptr, int* sched, hipStream_t s);

// Node orders (order.hip).  order[r] = node placed at position r.
hipError_t launch_perm_inverse(int N, const int* order, int* inv, int* bad, hipStream_t s);
hipError_t launch_perm_check(int N, const int* inv, int* bad, hipStream_t s);
size_t perm_graph_temp_bytes(int N);
hipError_t perm_graph(int N, const int* order, const int* inv, const int* row_ptr, const int* col,
                      const float* val, int* row_ptr_out, int* col_out, float* val_out, int* deg,
                      void* temp, size_t temp_bytes, hipStream_t s);
hipError_t launch_map_indices(int n, int N, const int* inv, const int* idx, int* out,
                              hipStream_t s);
hipError_t launch_gather_rows(int n, int d, const float* F, size_t ldf, const int* rows, int N,
                              float* out, int ldo, int* bad, hipStream_t s);
hipError_t launch_nearest_centroid(int N, int d, const float* F, size_t ldf, const float* C,
                                   const int* usable, int k, int* labels, hipStream_t s);
size_t sort_labels_temp_bytes(int N);
hipError_t sort_labels(void* temp, size_t temp_bytes, const int* kin, int* kout, const int* vin,
                       int* vout, int N, int key_bits, hipStream_t s);
hipError_t launch_iota(int N, int* out, hipStream_t s);
hipError_t launch_density_keys(int N, const double* w, uint64_t seed, uint64_t* keys, int* vals,
                               hipStream_t s);
hipError_t launch_sum_f64(const double* x, int N, double* part, int nparts, double* out,
                          hipStream_t s);
hipError_t launch_decoder_weights(int n, const int* idx, const double* w, const double* sum, int N,
                                  float* out, hipStream_t s);

}  // namespace csc
