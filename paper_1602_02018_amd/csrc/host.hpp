// Host-side helpers shared by the single-graph and the batched C calls.
#pragma once

#include <functional>
#include <vector>

#include "kernels.hpp"

namespace csc {

hipStream_t as_stream(void* s);
csc_status check_graph(const csc_graph* g);
csc_status check_ws(void* ws, size_t ws_bytes, size_t need);
void jackson_lowpass(double lc, int p, double* a);
double count_from_moments(double lambda, int p, const double* mom);
void apply_tuning(StepArgs& sa);
// The row schedule the step kernels follow on g at layout L (or NULL).
const int* step_sched(const csc_graph& g, const Layout& L);
size_t filter_bytes(const Layout& L);
size_t count_bytes(const Layout& L, int p, int group = 1);
// Eigencount passes t0, t0 + 1, ... (the dichotomy of Sec. 4.3) on a count
// workspace (count_bytes): after each pass, more(t, moments) says whether
// another follows.  Pass t + 1's signals are drawn on a second stream while
// pass t runs.
csc_status count_passes(const csc_graph& g, int n_signals, int p, uint64_t seed, uint32_t t0,
                        void* ws, size_t ws_bytes, hipStream_t s,
                        const std::function<bool(uint32_t, const double*)>& more);
// A moment pass of order p runs moment_steps(p) = ceil(p/2) Chebyshev steps
// and leaves moment_raw(p) = 2 ceil(p/2) + 1 float64 products: raw[0] =
// <T_0, T_0>, raw[2j-1] = <T_{j-1}, T_j>, raw[2j] = <T_j, T_j>.
// moments_from_raw turns them into mu_0..mu_p by the doubling identities
// mu_{2j} = 2 <T_j, T_j> - mu_0 and mu_{2j+1} = 2 <T_j, T_{j+1}> - mu_1.
int moment_steps(int p);
int moment_raw(int p);
// Eigencount passes run together by the dichotomies (at most kMaxCountGroup,
// each n_signals columns rounded up to a multiple of 4).
int count_group();
int batch_count_group();  // tests per pass of the batched dichotomy
inline int round4(int x) { return (x + 3) / 4 * 4; }
void moments_from_raw(const double* raw, int p, double* mom);
size_t interp_bytes(const Layout& L);
int use_hip_graphs();
// Batched step work lists follow the single kernels' XCD-aware order (order != 0).
bool xcd_batched();

// Launch sequence of one pass h~(L) T0 for the accumulating epilogues
// (EPI_Y: Y = h~(L) T0; EPI_CG: the CG operator), in the process-wide form:
// forward recurrence with a running sum, or Clenshaw's backward recurrence.
struct PassStep {
  const float* Tm;
  const float* Tprev;
  float* Tnext;
  float c0, c1;
  int epi;
  bool first, last;
};
enum { FORM_FORWARD = 0, FORM_CLENSHAW = 1 };
int filter_form();
std::vector<PassStep> pass_plan(int epi, const double* a, int p, const float* T0, float* Ta,
                                float* Tb, int form);

// Block conjugate gradient of the interpolation (api.hip), one graph's state;
// the Chebyshev pass Q = M P runs between block_pre and block_post.
struct BlockBufs {
  float *P, *Q, *Ta, *Tb, *X, *R, *Z, *mask;
  double *part, *gpart, *G, *S_t, *S_a, *S_na, *S_b, *rn2;
};
struct BlockState {
  Layout L;
  int k = 0, sr = 0, ndone = 0, nlive = 0;
  double tol = 0.0;
  bool jacobi = false;  // preconditioned form: Z = D^-1 R, D = diag(mask) + gamma I
  int host_threads = 1;  // host threads of the k x k solves (the batched form runs graphs in parallel)
  float gamma = 0.f;
  BlockBufs b{};
  bool finished = false, converged = false, broke = false;
  std::vector<char> done;
  std::vector<int> iters;
  std::vector<double> bn2, relres, G, T, W, C, N, rn2;
  // X += P alpha on the side stream (post_launch_b): `main` waits for `done`
  // before P or S_a change again (post_finish), in block_join, and at the
  // latest when the state goes away
  struct SideX {
    hipEvent_t go = nullptr, done = nullptr;
    hipStream_t main = nullptr;
    bool pending = false;
    SideX() = default;
    SideX(const SideX&) = delete;
    SideX& operator=(const SideX&) = delete;
    ~SideX();
  } sx;
};
csc_status block_init(BlockState& st, const Layout& L, int k, double tol, bool jacobi, float gamma,
                      const BlockBufs& b, const double* bnorm2_dev, hipStream_t s);
csc_status block_pre(BlockState& st, hipStream_t s);
csc_status block_post(BlockState& st, int it, int max_iter, hipStream_t s);
// The stages of block_pre and block_post: the launch stages enqueue device
// work and copies into st's host vectors, the host stages (which touch only
// st) need the stream synchronised after the preceding launch stage.
csc_status pre_launch(BlockState& st, hipStream_t s);
void pre_host(BlockState& st);
csc_status pre_finish(BlockState& st, hipStream_t s);
csc_status post_launch_a(BlockState& st, hipStream_t s);
void post_host_a(BlockState& st);
csc_status post_launch_b(BlockState& st, hipStream_t s);
void post_host_b(BlockState& st, int it, int max_iter);
csc_status post_finish(BlockState& st, hipStream_t s);
void block_finish(BlockState& st, int max_iter);
// the stream waits for an X update still running on the side stream
csc_status block_join(BlockState& st);

// Workspace of permuted_graph, and the graph g permuted to `order` (row r =
// node order[r], neighbours relabelled and kept in CSR order) with the sampled
// indices renumbered, carved from ar; synchronises s to check `order`.
size_t perm_bytes(int N, int64_t nnz, int n);
csc_status permuted_graph(const csc_graph& g, const int* order, const int* idx, int n, Arena& ar,
                          csc_graph& gp, const int*& idxp, hipStream_t s);

// Learned dichotomy (mlp.hip): the bracket from the network outputs y for a
// graph whose first pass at lambda = 1 gave count c1 and moments mom, and the
// update after each later count (true once the count rounds to k).
struct LearnedState {
  double lo = 0, hi = 2, lo0 = 0, hi0 = 2, half_lo = 0, half_hi = 2;
  int inside = 0;  // tests run inside the bracket so far
  bool below = false, above = false, widened = false;
  int status = CSC_OK;
};
void learned_features(const double* mom, int N, int k, float* x);
void learned_begin(LearnedState& S, const double* mom, int p, int k, int n_signals, double c1,
                   const float y[2]);
bool learned_update(LearnedState& S, double mid, double cnt, int k);
size_t mlp_workspace(int B);
hipStream_t capture_stream();

}  // namespace csc
