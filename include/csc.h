/*
 * csc.h - C ABI of libcsc, the MI355X (gfx950) hot path of compressive
 * spectral clustering (Tremblay, Puy, Gribonval, Vandergheynst, ICML 2016).
 *
 * The calls follow the statement of Alg. 2: the input is the normalized
 * Laplacian L of an undirected graph and the number of clusters k, with
 * parameters n (sampled nodes), d (random signals), p (polynomial order) and
 * gamma (regularisation).  Steps 1, 3-5 and 7 run on the GPU; step 6 (k-means
 * on an n x d matrix) runs on the host inside the library.
 *
 * Conventions shared by every call
 * --------------------------------
 * Return value: a csc_status.  CSC_OK and the CSC_W_* warnings leave every
 *   output valid; CSC_E_* errors leave outputs unspecified.  The message of
 *   the last error of the calling thread is returned by csc_last_error().
 * Pointers: "device" pointers are HIP device allocations on the current
 *   device; "host" pointers are ordinary host memory.  The caller owns every
 *   buffer; the library never allocates device memory and never frees caller
 *   memory.  Scratch memory is a caller-provided device workspace of at least
 *   the size returned by the matching csc_*_workspace_bytes() call, aligned to
 *   256 bytes.
 * Streams: all device work is ordered on the hipStream_t passed as `stream`
 *   (NULL = the null stream).  Calls that return host scalars synchronise that
 *   stream before returning; the others return as soon as the work is queued.
 * Dense blocks: node-major float32, row i of an N x w block starts at
 *   ptr + i*ld, ld >= w.
 * Determinism: the same inputs, seeds and parameters give bit-identical
 *   outputs on the same device (no floating-point atomics; every reduction
 *   runs in a fixed order).
 * Random numbers: Philox4x64-10 (Salmon et al., SC'11) with key (seed, 0).
 *   Gaussian entry (i, j) of an N x w block for sub-stream t of stream S uses
 *   counter (i*w + j, t, S, 0) and the Box-Muller transform in float64 of the
 *   first two output words x0, x1:
 *   u1 = ((x0>>11)+1) 2^-53, u2 = (x1>>11) 2^-53,
 *   z = sqrt(-2 ln u1) cos(2 pi u2) / sqrt(w), rounded to float32.
 *   Streams: COUNT = 1 (eigencount signals, t = dichotomy step), FEAT = 2
 *   (feature signals, t = 0), SAMPLE = 3 (sampling keys), KMEANS = 4.
 * Thread safety: calls are reentrant when they use distinct workspaces (the
 *   batched calls take turns while recording a HIP graph on the library's
 *   capture stream).  Tuning, damping and filter-form settings are
 *   process-wide and read when a call starts; changing them while another
 *   thread's call runs is not supported.
 */
#ifndef CSC_H
#define CSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t csc_status;

enum {
  CSC_OK = 0,
  CSC_E_INVALID_ARG = 1,      /* bad size, pointer, parameter or workspace   */
  CSC_E_GRAPH = 2,            /* malformed CSR (range, order, self-loop)      */
  CSC_E_HIP = 3,              /* a HIP runtime call failed                    */
  CSC_E_OOM = 4,              /* host memory exhausted                        */
  CSC_W_NOT_CONVERGED = 5,    /* CG reached max_iter; outputs still valid     */
  CSC_W_BISECT_EXHAUSTED = 6, /* dichotomy used max_steps; lambda = upper end */
  CSC_W_BRACKET_MISS = 7      /* given bracket did not hold lambda_k; the
                                 search fell back to [0, 2]                   */
};

enum { CSC_STREAM_COUNT = 1, CSC_STREAM_FEAT = 2, CSC_STREAM_SAMPLE = 3, CSC_STREAM_KMEANS = 4 };

/* A = D^-1/2 W D^-1/2 of an undirected graph in CSR form (device pointers).
 * L = I - A is never stored.  row_ptr[n+1] non-decreasing with row_ptr[0] = 0,
 * col[nnz] in [0, n), val[nnz] = A_ij.  dinv_sqrt[n] = D_ii^-1/2 (0 for an
 * isolated node) is kept for reference; the filters only read val. */
typedef struct csc_graph {
  int32_t n;
  int32_t nnz;
  const int32_t* row_ptr;
  const int32_t* col;
  const float* val;
  const float* dinv_sqrt;
  /* Row walk of the step kernels, or NULL for the natural order: a
   * permutation of [0, n) from csc_row_schedule.  Rows of one wave are
   * taken from consecutive entries, so rows of similar degree share a wave;
   * results do not depend on it (each row still sums its neighbours in CSR
   * order; only the grouping of float64 partial sums changes). */
  const int32_t* sched;
} csc_graph;

/* Message of the last error returned on the calling thread ("" if none). */
const char* csc_last_error(void);

/* Library version, major*10000 + minor*100 + patch. */
int32_t csc_version(void);

/* Tuning.  Dense blocks inside the library are stored as panels of PW
 * columns (PW a multiple of 4 in [4, 256]); a Chebyshev step gathers
 * neighbour rows of one panel at a time.  csc_set_panel_width(pw) forces PW for every later
 * call of this process (0 restores the built-in choice); workspace sizes
 * returned by the csc_*_workspace_bytes calls cover every PW.
 * csc_get_panel_width(n, nnz, w) returns the PW the library will use for an
 * n x w block of a graph with nnz stored entries. */
csc_status csc_set_panel_width(int32_t pw);
int32_t csc_get_panel_width(int32_t n, int64_t nnz, int32_t w);

/* Damping of the Chebyshev coefficients used by every call that builds a
 * low-pass from lambda (eigencount, dichotomy, features, interpolation,
 * csc_jackson_coeffs): CSC_DAMP_JACKSON (default) multiplies c_m by the
 * Jackson factors g_m (Sec. 4.3); CSC_DAMP_NONE keeps the plain truncated
 * Chebyshev series c_m, which overshoots near lambda_c (Gibbs) and can make
 * 1 - h~ indefinite, so the interpolation may stop with
 * CSC_W_NOT_CONVERGED.  Process-wide; for comparisons of the two filters. */
enum { CSC_DAMP_JACKSON = 0, CSC_DAMP_NONE = 1 };
csc_status csc_set_damping(int32_t damping);
int32_t csc_get_damping(void);

/* Evaluation form of the accumulated filters (Sec. 2.1, fast graph filtering):
 * the features h~(L) R of every node and the CG operator's h~(L) P.
 * CSC_FORM_FORWARD: the three-term recurrence T_{m+1} = 2 (L - I) T_m - T_{m-1}
 *   with a running sum Y += a_m T_m (per step: the gathered T_m, T_{m-1}, the
 *   written T_{m+1}, Y read and written: five block accesses);
 * CSC_FORM_CLENSHAW (default): Clenshaw's backward recurrence
 *   b_m = a_m R + 2 (L - I) b_{m+1} - b_{m+2}, h~(L) R = a_0 R + (L - I) b_1 - b_2
 *   (gathered b_{m+1}, b_{m+2}, R, written b_m: four accesses).
 * Both take p products by A; results agree to float32 rounding (not bit for
 * bit).  Moment passes (eigencount) and sampled-row feature passes always use
 * the forward recurrence.  Process-wide. */
enum { CSC_FORM_FORWARD = 0, CSC_FORM_CLENSHAW = 1 };
csc_status csc_set_filter_form(int32_t form);
int32_t csc_get_filter_form(void);

/* Kernel tuning knobs, process-wide; results do not depend on them, except
 * for CSC_TUNE_BLOCK_PRODUCT (rounding only, see below).
 * CSC_TUNE_PANEL_WIDTH: as csc_set_panel_width.
 * CSC_TUNE_XCD_ORDER (0/1/2, default 1): how row tiles are spread over the
 *   8 XCDs of the GPU (workgroup b runs on XCD b mod 8): 0 round-robin; 1
 *   each XCD walks a contiguous range of panel-major row tiles; 2 each XCD
 *   keeps one eighth of the rows and all XCDs walk the panels in step.
 * CSC_TUNE_NONTEMPORAL (0/1, default 0): non-temporal loads and stores for
 *   the streamed blocks (T_{m-1}, T_{m+1}, accumulators).
 * CSC_TUNE_HIP_GRAPHS (0/1, default 1): the batched calls record their
 *   repeated passes (eigencount passes, CG iterations) once as a HIP graph
 *   and replay it; 0 launches every kernel directly.
 * CSC_TUNE_ROW_SCHED (0/1/2, default 1): when the step kernels follow the
 *   graph's row schedule (csc_graph.sched, when set): 0 never, 1 when a wave
 *   holds exactly 8 rows (panel widths 29 to 32, the only shape where the
 *   degree-sorted walk was measured to pay), 2 whenever a wave holds several
 *   rows.
 * CSC_TUNE_COUNT_GROUP (1..4, default 4): the dichotomies
 *   (csc_estimate_lambda_k, csc_estimate_lambda_k_learned) run this many
 *   consecutive tests' eigencount passes as one wider pass (their signals do
 *   not depend on the earlier counts; each test's moments are kept apart), so
 *   a search computes up to this many - 1 passes it does not use.  Each
 *   test keeps its own signals, tested point and decision rule; its count
 *   equals the count of one pass per test up to the order of the float64
 *   moment sums (a wider pass groups them differently), so only a count
 *   within that rounding of k - 1/2 or k + 1/2 can decide differently.
 * CSC_TUNE_BATCH_COUNT_GROUP (1..4, default 1): the same for the batched
 *   dichotomy (csc_estimate_lambda_k_batched); a batch already fills the GPU
 *   with one test per graph per pass, so by default no passes are computed
 *   ahead there.  With equal group sizes the batched and the single calls
 *   give the same results bit for bit; at the defaults (4 and 1) their
 *   counts agree up to the order of float64 sums, as above.
 * CSC_TUNE_BLOCK_PRODUCT (0/1, default 0): the block CG's residual update
 *   R -= Q alpha (Sec. 4.4's interpolation solve): 0 forms each output
 *   element as a float64 sum of exact products of the float32 entries and
 *   the float64 k x k step matrix, rounded once to float32 (float64 matrix
 *   cores); 1 rounds the step matrix to float32 and sums in float32 (float32
 *   matrix cores).  X += P alpha always takes float32 sums (the precision
 *   form's float32 vector updates), and so do P = Z T and Z += P beta in
 *   CSC_CG_BLOCK_JACOBI (CSC_CG_BLOCK keeps float64 sums for them).  This
 *   knob changes the rounding of the solve (not the
 *   tolerance it meets); the Gram matrices (inner products) stay float64
 *   either way.
 * csc_get_tuning returns the current value (-1 for an unknown key).
 */
enum {
  CSC_TUNE_PANEL_WIDTH = 0,
  CSC_TUNE_XCD_ORDER = 1,
  CSC_TUNE_NONTEMPORAL = 2,
  CSC_TUNE_HIP_GRAPHS = 3,
  CSC_TUNE_ROW_SCHED = 4,
  CSC_TUNE_COUNT_GROUP = 5,
  CSC_TUNE_BATCH_COUNT_GROUP = 6,
  CSC_TUNE_BLOCK_PRODUCT = 7
};
csc_status csc_set_tuning(int32_t key, int32_t value);
int32_t csc_get_tuning(int32_t key);

/* Autotuner.  csc_autotune times one kind of Chebyshev step (as in
 * csc_cheb_steps: 0 accumulate, 1 moments, 2 CG operator, 3 Clenshaw step,
 * 4 moments of a group of dichotomy tests side by side) on graph g at block
 * width w for candidate panel widths (the six best of the built-in cost
 * model and every multiple of 32 columns that pads w less than twofold) and
 * both XCD orders, `reps` launches each, timed with HIP events on `stream`.
 * The fastest panel width is recorded for the shape bucket (floor(log2 N),
 * rounded mean degree, w) and used by every later call of the process on a
 * graph of that bucket; pw_out / xcd_out / us_out (host, or NULL) receive the
 * winner and its microseconds per launch.  The XCD-order knob is left as it
 * was (pass xcd_out to csc_set_tuning to apply it).  ws:
 * csc_cheb_steps_workspace_bytes(N, w).  Synchronises.  csc_autotune_clear
 * forgets every recorded bucket. */
csc_status csc_autotune(const csc_graph* g, int32_t w, int32_t kind, int32_t reps,
                        int32_t* pw_out, int32_t* xcd_out, double* us_out, void* ws,
                        size_t ws_bytes, void* stream);
void csc_autotune_clear(void);

/* ------------------------------------------------------------------------
 * Normalized adjacency (Sec. 2.1): D_ii = sum_{j != i} W_ij accumulated in
 * float64, s_i = D_ii^-1/2 (0 when D_ii = 0, so that an isolated node has
 * L_ii = 1), val_out[e] = s_i W_ij s_j for each stored entry e = (i, j), and 0
 * for a stored diagonal entry.
 * row_ptr, col, w, val_out, dinv_sqrt_out: device.  w = NULL means W_ij = 1.
 * When `check` is non-zero the CSR is validated first (row_ptr monotone,
 * row_ptr[0] = 0, row_ptr[n] = nnz, columns in range) and CSC_E_GRAPH is
 * returned on failure; this synchronises the stream.  check = 2 also
 * requires the undirected graph of Sec. 2.1 without self-loops: no stored
 * diagonal entry, columns strictly increasing in each row, and W symmetric
 * (every stored (i, j) has a stored (j, i) of the same weight); without it a
 * stored diagonal entry is accepted and its value set to 0, and symmetry is
 * the caller's promise.
 */
csc_status csc_laplacian_from_adjacency(int32_t n, int32_t nnz, const int32_t* row_ptr,
                                        const int32_t* col, const float* w, float* val_out,
                                        float* dinv_sqrt_out, int32_t check, void* stream);

/* Row schedule for csc_graph.sched: rows in chunks of 4096 consecutive
 * indices, within a chunk by decreasing degree (row_ptr[i+1] - row_ptr[i]),
 * ties by index.  A wave of a step kernel walks several consecutive rows of
 * the schedule, so it no longer waits on the one high-degree row among
 * low-degree ones (skewed degree distributions), while rows stay within
 * 4096 of their place (the node order's locality is kept).
 * row_ptr, sched: device (sched int32[n]).  The CSR must be valid (see
 * csc_laplacian_from_adjacency).
 * skew_out: host double or NULL: how much longer the natural order keeps a
 *   wave of 8 rows busy than its mean, sum over groups of 8 consecutive rows
 *   of 8 * max degree divided by nnz (1 for equal degrees, about 1.4 for a
 *   Poisson(16) SBM, 3.4 for the 1e6-node Chung-Lu graph); requesting it
 *   synchronises the stream and needs ws (256 bytes of device memory),
 *   otherwise ws may be NULL and nothing synchronises.
 * The schedule pays off where that skew is large and a wave holds 8 rows or
 * more (panel widths up to 32): measured on MI355X, the moment step at width
 * 28 of the 1e6-node Chung-Lu graph drops from 820 to 664 us, while on the
 * 1e5-node SBM the schedule costs 4%. */
csc_status csc_row_schedule(int32_t n, const int32_t* row_ptr, int32_t* sched, double* skew_out,
                            void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Jackson-Chebyshev coefficients a_0..a_p (host, float64) of the order-p
 * approximation of the ideal low-pass h_lc of Eq. (1) (Sec. 4.3) in the basis
 * T_m(lambda - 1):  theta = arccos(lc - 1), c_0 = 1 - theta/pi,
 * c_m = -2 sin(m theta)/(m pi), g_m = [(p+2-m) cos(m a) + sin(m a) cot a]/(p+2)
 * with a = pi/(p+2), a_m = g_m c_m.  lc in [0, 2], p >= 0.  a_out: host[p+1].
 */
csc_status csc_jackson_coeffs(double lambda_c, int32_t p, double* a_out);

/* ------------------------------------------------------------------------
 * Gaussian signal block (Sec. 3.1, Alg. 2 step 3): R[i*ld + j] for i < n_rows,
 * j < w, variance 1/w, drawn as in the header comment with sub-stream t of
 * stream `stream_id`.  R: device.
 */
csc_status csc_gaussian_block(int32_t n_rows, int32_t w, uint64_t seed, uint32_t t,
                              uint32_t stream_id, float* R, int32_t ld, void* stream);

/* ------------------------------------------------------------------------
 * Polynomial filtering (Sec. 2.1, fast graph filtering) of a given block:
 * Y = sum_{m=0}^{p} coeffs[m] T_m(L - I) X by the recurrence T_0 = X,
 * T_1 = -A X, T_{m+1} = -2 A T_m - T_{m-1}, in float32.
 * X, Y: device, N x w node-major with leading dimension ld (X and Y may not
 * overlap).  coeffs: host[p+1].  ws: csc_filter_workspace_bytes(N, w).
 */
size_t csc_filter_workspace_bytes(int32_t n, int32_t w);
csc_status csc_filter_block(const csc_graph* g, const double* coeffs, int32_t p, const float* X,
                            int32_t w, int32_t ld, float* Y, void* ws, size_t ws_bytes,
                            void* stream);

/* ------------------------------------------------------------------------
 * Feature pass, Alg. 2 steps 2-4: draws the N x d block R of stream FEAT
 * (sub-stream 0), filters it by the order-p Jackson-Chebyshev low-pass at
 * lambda_c, and writes rows of h~(L) R, scaled to unit length when
 * `normalize` is non-zero (a zero row stays zero).
 * rows = NULL: all N rows, Y is N x d.  Otherwise rows (device, n_rows
 * distinct indices in [0, N)) selects the rows written, Y[s] = row rows[s]
 * (Alg. 2 step 5 keeps only the sampled rows); the recurrence still runs
 * over the whole graph.  Y: device, ld >= d.  ws: csc_filter_workspace_bytes.
 */
csc_status csc_filter(const csc_graph* g, double lambda_c, int32_t p, int32_t d, uint64_t seed,
                      const int32_t* rows, int32_t n_rows, int32_t normalize, float* Y,
                      int32_t ld, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * csc_filter without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Arguments, outputs and errors as csc_filter; the
 * scratch memory is a fixed array inside the library, one per device
 * (csc_filter_noalloc_max_bytes() = 128 MiB), held from the first call on
 * that device until the process ends.  The call allocates no device memory
 * and calls no allocating routine.  A call whose workspace need (the
 * csc_filter layout at the chosen panel width, about 16 N d bytes, e.g.
 * N = 1e5 with d = 47 needs 77 MB) exceeds the array returns
 * CSC_E_INVALID_ARG before any device work; p must lie in [1, 4096].  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (other threads or streams) race and give undefined results; the
 * array keeps the last call's contents and each call initialises what it
 * reads.  The results are bit-identical to csc_filter's.
 */
size_t csc_filter_noalloc_max_bytes(void);
csc_status csc_filter_noalloc(const csc_graph* g, double lambda_c, int32_t p, int32_t d,
                              uint64_t seed, const int32_t* rows, int32_t n_rows,
                              int32_t normalize, float* Y, int32_t ld, void* stream);

/* ------------------------------------------------------------------------
 * Eigencount (Sec. 4.3): Hutchinson estimate of the number of eigenvalues of
 * L in [0, lambda], count = sum_{i,l} R_il (h~_lambda(L) R)_il, with R the
 * N x n_signals block of stream COUNT, sub-stream t.  It is evaluated as
 * sum_m a_m mu_m with the moments mu_m = <R, T_m(L - I) R> accumulated in
 * float64 on the GPU from float32 recurrences.
 * count_out: host scalar.  moments_out: host[p+1] or NULL.
 * ws: csc_estimate_workspace_bytes(N, n_signals, p).  Synchronises.
 */
size_t csc_estimate_workspace_bytes(int32_t n, int32_t n_signals, int32_t p);
csc_status csc_eigencount(const csc_graph* g, double lambda, int32_t p, int32_t n_signals,
                          uint64_t seed, uint32_t t, double* count_out, double* moments_out,
                          void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * lambda_k by eigencount dichotomy (Alg. 2 step 1, Sec. 4.3).  Starting from
 * the bracket [lo, hi] (bracket = host[2], or NULL for [0, 2]), step
 * t = 1, 2, ... tests mid = (lo + hi)/2 with fresh signals (sub-stream t):
 * if floor(count + 1/2) = k it returns mid; if count < k then lo = mid, else
 * hi = mid.  After max_steps tests it returns hi with CSC_W_BISECT_EXHAUSTED.
 * With a caller bracket the search runs inside it; if it uses max_steps
 * tests whose counts all fell on one side of k (lambda_k lies outside the
 * bracket), it restarts from [0, 2] with the next sub-streams and returns
 * CSC_W_BRACKET_MISS (steps_out counts the tests of both searches).
 * lambda_out, steps_out: host scalars.  trace_out: host[4*max_steps] receiving
 * (mid, count) of every tested point (up to 2*max_steps tests when a caller
 * bracket misses), or NULL.  moments_out: host[p+1]
 * receiving the moments of the first tested point, or NULL.
 * ws: csc_estimate_workspace_bytes(N, n_signals, p).  Synchronises.  The
 * signals of test t + 1 are drawn into ws on a library-owned second stream
 * while test t runs; events order it after the caller's earlier work on
 * `stream` and make `stream` wait for it before returning, so the caller sees
 * the usual stream order (the same holds for csc_estimate_lambda_k_learned).
 */
/* One-pass form of the dichotomy (kernel polynomial method).  The count of
 * Sec. 4.3 written in the Chebyshev basis, count(lambda) = sum_m a_m(lambda)
 * mu_m with mu_m = <R, T_m(L - I) R>, holds for every lambda with the same
 * signals, so one moment pass (the signals of the plain search's first test,
 * sub-stream 1) serves every tested point and the dichotomy, with the same
 * rules as csc_estimate_lambda_k, runs on the host from the moments.
 * Arguments and outputs as csc_estimate_lambda_k (steps_out counts tested
 * points; one pass is run whatever their number; moments_out receives the
 * pass's moments).  Returns CSC_W_BISECT_EXHAUSTED after max_steps tests.
 * ws: csc_estimate_workspace_bytes(N, n_signals, p).  Synchronises. */
csc_status csc_estimate_lambda_k_kpm(const csc_graph* g, int32_t k, int32_t p, int32_t n_signals,
                                     uint64_t seed, int32_t max_steps, double* lambda_out,
                                     int32_t* steps_out, double* trace_out, double* moments_out,
                                     void* ws, size_t ws_bytes, void* stream);

csc_status csc_estimate_lambda_k(const csc_graph* g, int32_t k, int32_t p, int32_t n_signals,
                                 uint64_t seed, int32_t max_steps, const double* bracket,
                                 double* lambda_out, int32_t* steps_out, double* trace_out,
                                 double* moments_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Uniform sampling without replacement (Sec. 3.2.2, Eq. (4)): node i gets the
 * 64-bit key x0 of counter (i, 0, SAMPLE, 0); idx[0..n) lists the n nodes
 * with the smallest (key, i) pairs in increasing order.  Integer-only, hence
 * bit-exact across implementations.  1 <= n <= N.  idx: device int32[n].
 * ws: csc_sample_workspace_bytes(N, n).  Synchronises.
 */
size_t csc_sample_workspace_bytes(int32_t N, int32_t n);
csc_status csc_sample(int32_t N, int32_t n, uint64_t seed, int32_t* idx, void* ws,
                      size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * k-means on the n sampled features (Alg. 2 step 6), on the host in float64:
 * `replicates` runs of k-means++ seeding (uniform draws at counter
 * (c, r, KMEANS, 0), u = (x0>>11) 2^-53) followed by Lloyd iterations (at most
 * max_iter; empty clusters re-seeded with the farthest point); the run with
 * the smallest inertia is kept.  Squared distances sum coordinates in order,
 * centroids sum points in index order, ties go to the lowest index.
 * F: host n x d (float32 with leading dimension ld for the first call, float64
 * for the _f64 call).  labels: host int32[n].  inertia_out: host or NULL.
 */
csc_status csc_kmeans_reduced(const float* F, int32_t n, int32_t d, int32_t ld, int32_t k,
                              int32_t replicates, int32_t max_iter, uint64_t seed,
                              int32_t* labels, double* inertia_out);
csc_status csc_kmeans_reduced_f64(const double* F, int32_t n, int32_t d, int32_t ld, int32_t k,
                                  int32_t replicates, int32_t max_iter, uint64_t seed,
                                  int32_t* labels, double* inertia_out);

/* The k-means++ seeding alone (the first phase of csc_kmeans_reduced /
 * csc_kmeans_reduced_device, same draws and sums): picks[r*k + c] (host
 * int32[replicates*k]) receives the index of the point chosen as centre c of
 * replicate r.  The library forms the seeding's running sums of the D^2
 * weights in blocks of 32 points (the block's offset plus the running sum
 * inside it), which is the index-order prefix sum up to rounding, so a pick
 * can differ from one made with the plain prefix sum only where u_c times
 * the total lies within that rounding (at most 4 n 2^-53 of the total) of a
 * running sum.  csc_kmeans_seeds works on host float64 F (n x d, leading
 * dimension ld); csc_kmeans_seeds_device on device float32 F with the
 * workspace of csc_kmeans_device_workspace_bytes(n, d, k, replicates), and
 * synchronises. */
csc_status csc_kmeans_seeds(const double* F, int32_t n, int32_t d, int32_t ld, int32_t k,
                            int32_t replicates, uint64_t seed, int32_t* picks);
csc_status csc_kmeans_seeds_device(const float* F, int32_t n, int32_t d, int32_t ld, int32_t k,
                                   int32_t replicates, uint64_t seed, int32_t* picks, void* ws,
                                   size_t ws_bytes, void* stream);

/* Community cores (the paper's conclusion: repeat the filtering with new
 * signals and the clustering of the sampled nodes, keep the nodes always
 * clustered together, interpolate from these stable cores only).  labels:
 * host T x n (run t's k-means labels of the n sampled nodes, row t).  Two
 * nodes share a class iff their labels agree in every run; the cores are the
 * k largest classes (ties: the class whose first member comes first), and
 * core_labels (host int32[n]) gets c for members of core c (0 = largest),
 * -1 for nodes outside the cores.  Host only. */
csc_status csc_community_cores(int32_t n, int32_t T, int32_t k, const int32_t* labels,
                               int32_t* core_labels);

/* The same k-means on the GPU, for float32 features already in device
 * memory: one workgroup per replicate, the same sums in the same order, so
 * labels and inertia are bit-identical to csc_kmeans_reduced's.
 * F: device n x d with leading dimension ld.  labels: HOST int32[n].
 * inertia_out: host or NULL.  ws: csc_kmeans_device_workspace_bytes(n, d, k,
 * replicates).  Synchronises. */
size_t csc_kmeans_device_workspace_bytes(int32_t n, int32_t d, int32_t k, int32_t replicates);
csc_status csc_kmeans_reduced_device(const float* F, int32_t n, int32_t d, int32_t ld, int32_t k,
                                     int32_t replicates, int32_t max_iter, uint64_t seed,
                                     int32_t* labels, double* inertia_out, void* ws,
                                     size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Interpolation, Eq. (5), and hard labels (Alg. 2 step 7, Sec. 4.1).
 * Solves (diag(mask) + gamma (I - h~(L))) X = B for the k columns of
 * B[idx[s], labels_r[s]] = 1 (mask_i = 1 iff i is in idx), h~ the order-p
 * Jackson-Chebyshev low-pass at lambda_k, by conjugate gradient per column in
 * lockstep: float32 vectors and recurrences, float64 inner products, step
 * sizes and residual norms; column j stops when ||r_j|| / ||b_j|| <= tol.
 * Then labels[i] = argmax_j X_ij / ||X_j|| (ties and zero columns -> lowest j).
 * idx, labels_r: device int32[n] (idx distinct, labels_r in [0, k)).
 * weights: device float[n] or NULL (all 1).  Fidelity weight w_s of sampled
 *   node idx[s]: the system becomes (M^T W M + gamma g~(L)) X = M^T W B, the
 *   weighted fidelity term that goes with variable-density sampling
 *   (csc_sample_density's decoder weights).
 * X: device N x k with leading dimension ldx >= k.  labels: device int32[N].
 * iters_out: host int32[k] or NULL; relres_out: host double[k] or NULL.
 * order: device int32[N] permutation of [0, N), or NULL.  With an order the
 *   solve runs on a copy of the graph permuted so that row r is node order[r]
 *   (neighbours kept in CSR order), which only changes where rows sit in
 *   memory (see csc_community_order); X and labels are written in the
 *   caller's node numbering either way.  Per-element products are unchanged;
 *   the float64 column sums run in the new row order.  An order that is not a
 *   permutation returns CSC_E_INVALID_ARG.
 * method: CSC_CG_COLUMNS runs the k conjugate gradients above side by side
 *   (columns never mix).  CSC_CG_BLOCK solves the k columns as one block CG
 *   (O'Leary 1980) in its breakdown-free form (Ji and Li 2017): the search
 *   block is the rank-revealing orthonormalisation of R + P beta (columns
 *   scaled to unit norm, pivoted Cholesky of their float64 Gram matrix, pivots
 *   below 1e-10 dropped), step matrices from float64 Gram matrices solved on
 *   the host; one Chebyshev pass per iteration serves every column, and the
 *   block Krylov space usually needs far fewer iterations.
 *   CSC_CG_BLOCK_JACOBI is the same block CG preconditioned by the diagonal
 *   D = diag(mask) + gamma I (the operator's diagonal without the small
 *   h~(L)_ii terms): the next search block comes from D^-1 R instead of R.
 *   The sampled rows (~1 + gamma) and the unsampled ones (~gamma) then share
 *   one scale, which leaves only about k small eigenvalues for the block
 *   Krylov space to resolve.  All three stop when
 *   every column has ||r_j|| / ||b_j|| <= tol (recursive residuals); iters_out
 *   gives the iteration at which each column first met it.  In the block
 *   forms a column that has met it leaves the search block (its X and
 *   residual keep the values it converged with), and a search block narrower
 *   than k runs its Chebyshev pass on a compact copy of its live columns.
 *   All solve the same system; X agrees to the accuracy the tolerance
 *   implies.  In the block forms the update X += P alpha runs on a
 *   library-owned second stream while the host works out the next step
 *   matrix; events order it after the work it reads and make `stream` wait
 *   for it before X or P is touched again, so the caller sees the usual
 *   stream order.
 * ws: csc_interpolate_workspace_bytes(N, nnz, k, n) (covers every form).
 * Synchronises.  Returns CSC_W_NOT_CONVERGED if a column reached max_iter or
 * the block iteration broke down (outputs still hold the last iterate).
 */
enum { CSC_CG_COLUMNS = 0, CSC_CG_BLOCK = 1, CSC_CG_BLOCK_JACOBI = 2 };
size_t csc_interpolate_workspace_bytes(int32_t N, int64_t nnz, int32_t k, int32_t n);
csc_status csc_interpolate(const csc_graph* g, const int32_t* order, int32_t method,
                           double lambda_k, int32_t p, double gamma, const int32_t* idx,
                           const int32_t* labels_r, const float* weights, int32_t n, int32_t k,
                           double tol,
                           int32_t max_iter, float* X, int32_t ldx, int32_t* labels,
                           int32_t* iters_out, double* relres_out, void* ws, size_t ws_bytes,
                           void* stream);

/* ------------------------------------------------------------------------
 * Community order of the nodes, a memory layout for the interpolation (the
 * paper fixes no node order).  Each node gets the label of the nearest
 * centroid (squared Euclidean distance in float32, coordinates summed in
 * order, ties to the lowest label) among the centroids of the k-means of
 * Alg. 2 step 6: centroid c is the float64 mean, rounded to float32, of the
 * rows F[idx[s]] with labels_r[s] = c (empty clusters are skipped).  order
 * lists the nodes by that label, ties in index order.  Listing communities
 * contiguously lets the gathers of a Chebyshev step hit the L2 of the XCD
 * that walks a community's rows.
 * F: device N x d, leading dimension ldf (the normalized features of every
 *   node, csc_filter with rows = NULL), d <= 128.  idx: device int32[n].
 *   labels_r: HOST int32[n] in [0, k) (csc_kmeans_reduced's output).
 * g: the graph (N = g->n nodes).  order: device int32[N].  node_labels: device
 *   int32[N] (the nearest-centroid label of every node) or NULL.
 * same_label_frac: host double or NULL: the fraction of stored edges whose
 *   ends share a label, i.e. of the gathers an XCD can serve from the rows it
 *   walks itself; on graphs without such structure the order only moves
 *   hubs around and callers should keep the natural order.
 * ws: csc_community_order_workspace_bytes(N, d, k, n).  Synchronises.
 */
size_t csc_community_order_workspace_bytes(int32_t N, int32_t d, int32_t k, int32_t n);
csc_status csc_community_order(const csc_graph* g, const float* F, int64_t ldf, int32_t d,
                               const int32_t* idx, const int32_t* labels_r, int32_t n, int32_t k,
                               int32_t* order, int32_t* node_labels, double* same_label_frac,
                               void* ws, size_t ws_bytes, void* stream);

/* Variable-density sampling (Alg. 2 step 5 with the sampling distribution
 * that Sec. 3.2.3 points to: p_i proportional to the local cumulative
 * coherence v_k(i)^2, estimated by the squared row norms of the filtered
 * signals, Sec. 4.1).  n distinct nodes by successive sampling, as an
 * exponential race: node i gets the float64 key E_i / w_i with
 * E_i = -ln(u_i), u_i = ((x0 >> 11) + 1) 2^-53 from Philox at counter
 * (i, 1, SAMPLE, 0) (+inf when w_i <= 0); idx lists the n smallest
 * (key, index) pairs in increasing order.
 * w: device double[N] (csc_normalize_rows' squared norms).  idx: device
 * int32[n].  dec_weights: device float[n] or NULL: the decoder weights
 * 1 / (N p_i) = (sum(w) / N) / w_i of the sampled nodes (0 where w_i = 0),
 * for csc_interpolate.  ws: csc_sample_density_workspace_bytes(N).
 * Synchronises. */
size_t csc_sample_density_workspace_bytes(int32_t N);
csc_status csc_sample_density(int32_t N, int32_t n, uint64_t seed, const double* w, int32_t* idx,
                              float* dec_weights, void* ws, size_t ws_bytes, void* stream);

/* Unit-length rows in place (Alg. 2 step 4), with the same arithmetic as
 * csc_filter's normalisation: s_i = sum_j Y_ij^2 in float64, Y_ij <- Y_ij / sqrt(s_i)
 * (a zero row stays zero).  sqnorm: device double[n_rows] receiving s_i, or
 * NULL.  Y: device n_rows x d with leading dimension ld. */
csc_status csc_normalize_rows(float* Y, int64_t ld, int32_t n_rows, int32_t d, double* sqnorm,
                              void* stream);

/* Rows of a device block: out[s, :] = F[rows[s], :] for s < n (Alg. 2 step 5,
 * the sampled features F_Omega from the features of every node).  F: device
 * N x d with leading dimension ldf; rows: device int32[n]; out: device n x d
 * with leading dimension ldo.  Returns CSC_E_INVALID_ARG if a row index lies
 * outside [0, N).  ws: 256 bytes of device memory.  Synchronises. */
csc_status csc_gather_rows(const float* F, int64_t ldf, int32_t N, int32_t d, const int32_t* rows,
                           int32_t n, float* out, int32_t ldo, void* ws, size_t ws_bytes,
                           void* stream);

/* ------------------------------------------------------------------------
 * Batched form: the same steps for G graphs of uneven size at once.  Every
 * Chebyshev step, reduction and CG update is one kernel launch covering all
 * graphs (workgroups stride over a table of per-graph work units); the
 * repeated passes (one eigencount pass per dichotomy step, one CG iteration)
 * are recorded once as a HIP graph and replayed (CSC_TUNE_HIP_GRAPHS).
 * Graph g follows exactly the arithmetic of the single-graph call with the
 * same arguments, so its outputs are bit-identical to that call's; for the
 * dichotomy this holds when CSC_TUNE_BATCH_COUNT_GROUP equals
 * CSC_TUNE_COUNT_GROUP (at the defaults, 1 and 4, counts agree up to the
 * order of float64 sums; see CSC_TUNE_COUNT_GROUP).
 * `graphs` is a host array of G csc_graph (device pointers inside); every
 * other per-graph array below is a host array indexed by g, and "device
 * per-graph" means a host array of G device pointers.  Workspaces: device, at
 * least the size returned by the matching *_workspace_bytes_batched call.
 * Per-graph statuses are written to status_out[g].
 *
 * csc_estimate_lambda_k_batched: csc_estimate_lambda_k for every graph
 * (k[g], n_signals[g], seeds[g], brackets[2g..2g+1] or NULL for [0, 2]), or
 * csc_estimate_lambda_k_learned when mlp_params (device) is given instead of
 * brackets; each dichotomy round runs one batched eigencount pass for the
 * graphs still searching (and one batched network evaluation after the
 * first).  lambda_out, steps_out, status_out: host[G]; trace_out:
 * host[G][2*max_steps][2] or NULL; moments_out: host[G][p+1] or NULL.
 * Its workspace size depends on CSC_TUNE_BATCH_COUNT_GROUP (a pass carries
 * that many tests per graph): query it after setting the knob; a call whose
 * workspace is smaller than the current setting needs returns
 * CSC_E_INVALID_ARG.
 * Synchronises.
 */
size_t csc_estimate_workspace_bytes_batched(const csc_graph* graphs, int32_t G,
                                            const int32_t* n_signals, int32_t p);
csc_status csc_estimate_lambda_k_batched(const csc_graph* graphs, int32_t G, const int32_t* k,
                                         int32_t p, const int32_t* n_signals,
                                         const uint64_t* seeds, int32_t max_steps,
                                         const double* brackets, const float* mlp_params,
                                         double* lambda_out,
                                         int32_t* steps_out, double* trace_out,
                                         double* moments_out, int32_t* status_out, void* ws,
                                         size_t ws_bytes, void* stream);

/* csc_filter_batched: csc_filter for every graph (lambda[g], d[g], seeds[g],
 * rows[g] device per-graph with n_rows[g] entries, or NULL for all N_g rows;
 * output Y[g] device per-graph n_rows[g] (or N_g) x d[g] with ld[g]).
 * Results are bit-identical to csc_filter's. */
size_t csc_filter_workspace_bytes_batched(const csc_graph* graphs, int32_t G, const int32_t* d,
                                          int32_t p);
csc_status csc_filter_batched(const csc_graph* graphs, int32_t G, const double* lambda,
                              int32_t p, const int32_t* d, const uint64_t* seeds,
                              const int32_t* const* rows, const int32_t* n_rows,
                              int32_t normalize, float* const* Y, const int32_t* ld, void* ws,
                              size_t ws_bytes, void* stream);

/* csc_interpolate_batched: csc_interpolate for every graph (lambda[g],
 * idx[g] / labels_r[g] device per-graph of n[g] entries, k[g]); all graphs'
 * CG iterations advance together, a graph leaving the batch once its columns
 * converge (or after max_iter iterations).  X: device per-graph N_g x k[g]
 * with ldx[g] (X or X[g] may be NULL), labels: device per-graph int32[N_g].
 * iters_out / relres_out: host arrays of sum_g k[g] entries (graph-major) or
 * NULL.  order: NULL, or per-graph device int32[N_g] node orders (entries
 * may be NULL); weights: NULL, or per-graph device float[n[g]] (entries may
 * be NULL); method: as in csc_interpolate.  Returns CSC_W_NOT_CONVERGED if any
 * graph did not converge. */
size_t csc_interpolate_workspace_bytes_batched(const csc_graph* graphs, int32_t G,
                                               const int32_t* k, int32_t p);
csc_status csc_interpolate_batched(const csc_graph* graphs, int32_t G, const int32_t* const* order,
                                   int32_t method, const double* lambda, int32_t p, double gamma,
                                   const int32_t* const* idx,
                                   const int32_t* const* labels_r, const float* const* weights,
                                   const int32_t* n,
                                   const int32_t* k, double tol, int32_t max_iter,
                                   float* const* X, const int32_t* ldx, int32_t* const* labels,
                                   int32_t* iters_out, double* relres_out, int32_t* status_out,
                                   void* ws, size_t ws_bytes, void* stream);

/* csc_kmeans_reduced_batched: csc_kmeans_reduced for G independent float32
 * inputs F[g] (host n[g] x d[g], leading dimension d[g]) with k[g] and
 * seeds[g]; the (graph, replicate) runs share one pool of host threads.
 * labels[g]: host int32[n[g]]; inertia_out: host[G] or NULL. */
csc_status csc_kmeans_reduced_batched(int32_t G, const float* const* F, const int32_t* n,
                                      const int32_t* d, const int32_t* k, int32_t replicates,
                                      int32_t max_iter, const uint64_t* seeds,
                                      int32_t* const* labels, double* inertia_out);

/* csc_kmeans_reduced_device_batched: csc_kmeans_reduced_device for G inputs
 * (F[g] device n[g] x d[g], leading dimension d[g]) in one launch of
 * G * replicates workgroups.  labels[g]: HOST int32[n[g]]; inertia_out: host[G]
 * or NULL.  ws: csc_kmeans_device_workspace_bytes_batched(...). */
size_t csc_kmeans_device_workspace_bytes_batched(int32_t G, const int32_t* n, const int32_t* d,
                                                 const int32_t* k, int32_t replicates);
csc_status csc_kmeans_reduced_device_batched(int32_t G, const float* const* F, const int32_t* n,
                                             const int32_t* d, const int32_t* k,
                                             int32_t replicates, int32_t max_iter,
                                             const uint64_t* seeds, int32_t* const* labels,
                                             double* inertia_out, void* ws, size_t ws_bytes,
                                             void* stream);

/* ------------------------------------------------------------------------
 * Learned lambda_k bracket.  The paper notes that a better estimate of
 * lambda_k would help the method (Sec. 5.2); this network proposes a bracket
 * for the dichotomy of Sec. 4.3 from the first eigencount pass.
 * A 52 -> 128 -> 128 -> 2 perceptron with GELU activations, float32, trained
 * and run on the GPU.  Parameters: one flat device array of
 * csc_mlp_param_count() = 23554 floats, W1 (52 x 128, row = input), b1 (128),
 * W2 (128 x 128), b2 (128), W3 (128 x 2), b3 (2).
 *
 * csc_mlp_features: the 52 inputs (host float[52]) from the moments
 *   mu_0..mu_p (host, p >= 50) of one eigencount pass: g_m mu_m / mu_0 for
 *   m = 1..50 (g_m the Jackson factors of order 50), ln N / 10 and k / N.
 * csc_mlp_forward: Y (device B x 2) for inputs X (device B x 52).
 * csc_count_root: lambda_0, the root of the count curve
 *   c(lambda) = sum_m a_m(lambda) mu_m of one eigencount pass (host moments
 *   mu_0..mu_p; 50 halvings of [0, 2]), and s = sqrt(2k / n_signals) /
 *   c'(lambda_0) clipped to [1e-4, 0.5]: the spread of lambda implied by the
 *   count's standard deviation.  The network's two outputs y are offsets in
 *   units of s: the bracket is [lambda_0 + s min(y), lambda_0 + s max(y)].
 * csc_mlp_loss_grad: mean pinball loss of output 0 at tau = 0.02 and output 1
 *   at tau = 0.98 against target (device float[B]) and its gradient with
 *   respect to the parameters (device float[23554]); loss_out: host or NULL
 *   (synchronises when given).  Every sum runs in a fixed order.
 * csc_mlp_adam_step: Adam (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected,
 *   step counted from 1) on params with moment buffers m, v (device, zeroed
 *   before the first step).
 * Workspace for forward / loss_grad: csc_mlp_workspace_bytes(B).
 */
int32_t csc_mlp_param_count(void);
size_t csc_mlp_workspace_bytes(int32_t B);
csc_status csc_mlp_features(const double* moments, int32_t p, int32_t N, int32_t k, float* x_out);
csc_status csc_count_root(const double* moments, int32_t p, int32_t k, int32_t n_signals,
                          double* lambda0_out, double* scale_out);
csc_status csc_mlp_forward(const float* params, const float* X, int32_t B, float* Y, void* ws,
                           size_t ws_bytes, void* stream);
csc_status csc_mlp_loss_grad(const float* params, const float* X, const float* target, int32_t B,
                             float* grad, double* loss_out, void* ws, size_t ws_bytes,
                             void* stream);
csc_status csc_mlp_adam_step(float* params, const float* grad, float* m, float* v, int32_t step,
                             float lr, void* stream);

/* csc_estimate_lambda_k_learned: the dichotomy of csc_estimate_lambda_k
 * started from a learned bracket.  Its first pass is the plain dichotomy's
 * first test (lambda = 1, sub-stream 1); if that does not stop the search,
 * the network maps that pass's moments to offsets around the pass's own count
 * root (csc_count_root), giving [lo, hi], intersected with the half of [0, 2]
 * the first count selects.  The dichotomy then runs inside with fresh
 * signals (sub-streams 2, 3, ...), stopping as the plain one does; if the
 * first four tests inside the bracket all fall on one side of k (the
 * interval is then a sixteenth of the bracket), the interval reopens once
 * towards the rest of the half: from the bracket's upper end to the top of
 * the half when the counts were below k, from the bottom of the half to its
 * lower end when above (CSC_W_BRACKET_MISS).  If the network's bracket cut
 * to the half is narrower than 1/1024, the bracket is lambda_0 (moved into
 * the half) plus or minus max(s, 1/1024), cut to the half.  steps_out counts
 * every pass (max_steps in total).
 * params: device.  trace_out: host[2*max_steps] or NULL; bracket_out: host[2]
 * or NULL.  p >= 50.  ws: csc_estimate_workspace_bytes_learned.  Synchronises.
 */
size_t csc_estimate_workspace_bytes_learned(int32_t n, int32_t n_signals, int32_t p);
csc_status csc_estimate_lambda_k_learned(const csc_graph* g, int32_t k, int32_t p,
                                         int32_t n_signals, uint64_t seed, int32_t max_steps,
                                         const float* params, double* lambda_out,
                                         int32_t* steps_out, double* trace_out,
                                         double* bracket_out, void* ws, size_t ws_bytes,
                                         void* stream);

/* ------------------------------------------------------------------------
 * Measurement hook (not a step of Alg. 2).  Launches exactly `steps`
 * Chebyshev-step kernels of one kind on an N x w block held in the workspace,
 * so that a caller can time one kernel with events on `stream`:
 * kind 0: T_{m+1} = -2 A T_m - T_{m-1} with Y += c T_{m+1} (feature and CG
 *         passes), kind 1: the same recurrence with the float64 moment
 *         epilogue (eigencount passes), kind 2: the last CG step (operator
 *         and per-column p^T A p partials), kind 3: a Clenshaw step, kind 4:
 *         the moment step of a group of CSC_TUNE_COUNT_GROUP eigencount tests
 *         side by side (w must be that group size times a multiple of 4),
 *         kind 5: the sparse product alone, T_{m+1} = A T_m (the CSR read,
 *         the gathered rows and one block written: the floor under every
 *         step kind at that width).
 * prepare != 0 first fills the block with a Gaussian block and zeroes the
 * other buffers (these launches precede the timed ones; call once with
 * steps = 0 and prepare = 1, then time calls with prepare = 0).
 * ws: csc_cheb_steps_workspace_bytes(N, w).
 */
size_t csc_cheb_steps_workspace_bytes(int32_t n, int32_t w);
csc_status csc_cheb_steps(const csc_graph* g, int32_t w, int32_t kind, int32_t prepare,
                          int32_t steps, void* ws, size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CSC_H */
