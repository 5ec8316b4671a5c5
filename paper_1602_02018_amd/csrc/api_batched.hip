// Batched C calls: Alg. 2 steps 1, 3-4 and 7 for G graphs of uneven size and
// width at once.  Every Chebyshev step, reduction and CG update is one launch
// for all graphs (batched.hip); the repeated passes (one eigencount pass per
// dichotomy step, one CG iteration) are recorded once as a HIP graph and
// replayed.  Each graph follows exactly the arithmetic of the single-graph
// calls, so outputs are bit-identical to calling those graph by graph.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <string>
#include <thread>
#include <mutex>
#include <vector>

#include "host.hpp"

namespace csc {
namespace {

// f(g) for every g in idx on up to 16 host threads (each call touches only
// graph g's state); in order on the calling thread for a single graph.
template <class F>
void host_parallel(const std::vector<int>& idx, F f) {
  const int n = (int)idx.size();
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  const int nt = std::min({n, hw, 16});
  if (nt <= 1) {
    for (int g : idx) f(g);
    return;
  }
  std::atomic<int> next{0};
  std::vector<std::thread> pool;
  pool.reserve(nt);
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&] {
      for (int i; (i = next.fetch_add(1)) < n;) f(idx[i]);
    });
  for (auto& th : pool) th.join();
}

struct Captured {
  hipGraphExec_t exec = nullptr;
  Captured() = default;
  Captured(const Captured&) = delete;
  Captured& operator=(const Captured&) = delete;
  ~Captured() {
    if (exec) (void)hipGraphExecDestroy(exec);
  }
};

// Records launch(stream) as a HIP graph on the capture stream.  The stream is
// one per device and process, so concurrent batched calls (distinct
// workspaces, other threads) take turns: the lock spans begin-capture,
// the recorded launches, end-capture and instantiation.
std::mutex g_capture_mu;

template <class F>
csc_status capture(F&& launch, Captured& out) {
  std::lock_guard<std::mutex> lock(g_capture_mu);
  hipStream_t cs = capture_stream();
  if (!cs) {
    set_error("could not create the graph-capture stream");
    return CSC_E_HIP;
  }
  CSC_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  const csc_status st = launch(cs);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &graph);
  if (st != CSC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) {
    set_error(std::string("hipStreamEndCapture failed: ") + hipGetErrorString(e));
    return CSC_E_HIP;
  }
  const hipError_t e2 = hipGraphInstantiate(&out.exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e2 != hipSuccess) {
    out.exec = nullptr;
    set_error(std::string("hipGraphInstantiate failed: ") + hipGetErrorString(e2));
    return CSC_E_HIP;
  }
  return CSC_OK;
}

// Replays the recorded pass (recording it on first use), or launches directly.
template <class F>
csc_status run_pass(F&& launch, Captured& cap, hipStream_t s) {
  if (!use_hip_graphs()) return launch(s);
  if (!cap.exec) CSC_TRY(capture(launch, cap));
  CSC_HIP(hipGraphLaunch(cap.exec, s));
  return CSC_OK;
}

template <class T>
csc_status upload(T* dst, const std::vector<T>& src, hipStream_t s) {
  if (src.empty()) return CSC_OK;
  CSC_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return CSC_OK;
}

// Step kernels take one unit per workgroup, as the single-graph kernels do:
// the rows in flight on an XCD then form the same narrow window of its slab,
// which is what lets the gathers of a community-ordered graph hit in L2 (with
// 8 units per workgroup the window grew eightfold and the batched CG pass ran
// 24% slower than the graphs one by one).
constexpr int kStepChunk = 1;

// Chunk size of the other tables: up to 8 units per workgroup while keeping
// >= 16384 workgroups.
int chunk_for(const std::vector<int>& units) {
  long long tot = 0;
  for (int u : units) tot += u;
  return (int)std::max(1LL, std::min(8LL, tot / 16384));
}

// Work list of a per-graph unit count in the workspace; returns its table.
struct WorkList {
  std::vector<Work> h;
  Work* d = nullptr;
  BTable table() const { return BTable{d, (int)h.size()}; }
};

// xcd: lay the entries out in the XCD-aware order of the single-graph step
// kernels (for tables of panel x tile units).
void plan_work(Arena& ar, const std::vector<int>& units, int chunk, WorkList& wl,
               bool xcd = false) {
  build_work(units.data(), (int)units.size(), chunk, xcd, wl.h);
  wl.d = ar.take<Work>(std::max<size_t>(wl.h.size(), 1));
}

size_t work_bytes(const std::vector<int>& units) {
  size_t n = 0;
  // chunk >= 1 => at most one entry per unit, plus the XCD-aware layout's
  // alignment and padding (at most 15 entries per graph)
  for (int u : units) n += (size_t)u + 16;
  return align_up(std::max<size_t>(n, 1) * sizeof(Work));
}

template <class F>
size_t max_widths(int n, int w, F f) {
  size_t m = 0;
  for (int pw = 4; pw <= 256; pw += 4) m = std::max(m, f(make_layout(n, w, pw)));
  return m;
}

// Largest number of (panel, tile) units and of block elements over all panel widths.
size_t max_units(int n, int w) {
  size_t m = 0;
  for (int pw = 4; pw <= 256; pw += 4) {
    const Layout L = make_layout(n, w, pw);
    m = std::max(m, (size_t)L.np * tiles_for(L));
  }
  return m;
}

size_t max_elems(int n, int w) {
  size_t m = 0;
  for (int pw = 4; pw <= 256; pw += 4) m = std::max(m, make_layout(n, w, pw).elems());
  return m;
}

int elem_units(size_t elems) { return (int)((elems + kElemsPerUnit - 1) / kElemsPerUnit); }

// Block width of a dichotomy pass carrying `group` tests of nc signals each
// (rounded up to a multiple of 4 when several share the pass).
int count_width(int nc, int group) { return group > 1 ? group * round4(nc) : nc; }

csc_status check_graphs(const csc_graph* graphs, int G) {
  CSC_REQUIRE(graphs != nullptr && G >= 1, "need at least one graph");
  for (int g = 0; g < G; ++g) CSC_TRY(check_graph(&graphs[g]));
  return CSC_OK;
}

size_t desc_bytes(int G, int p) {
  size_t b = align_up((size_t)p * G * sizeof(StepArgs)) + align_up(G * sizeof(GaussItem)) +
             2 * align_up(G * sizeof(ReduceItem)) + align_up(G * sizeof(ColDotItem)) +
             align_up(G * sizeof(CgItem)) + align_up(G * sizeof(LabelItem));
  b += 2 * align_up((size_t)G * sizeof(int));  // live flags, scratch flags
  return b + 4096;
}

}  // namespace
}  // namespace csc

using namespace csc;

// ------------------------------------------------------------ dichotomy ---
namespace csc {
namespace {
// Workspace of the batched dichotomy with gs tests per pass.
size_t estimate_bytes_batched(const csc_graph* graphs, int G, const int32_t* n_signals, int p,
                              int gs) {
  size_t b = desc_bytes(G, p) + align_up((size_t)G * gs * moment_raw(p) * sizeof(double));
  b += mlp_workspace(G) + align_up((size_t)G * 54 * sizeof(float)) + 1024;  // learned mode
  std::vector<int> u(G), gu(G), rv(G, gs * moment_raw(p));
  for (int g = 0; g < G; ++g) {
    const int w = count_width(n_signals[g], gs);
    b += max_widths(graphs[g].n, w, [p, gs](const Layout& L) { return count_bytes(L, p, gs); });
    u[g] = (int)std::min<size_t>(max_units(graphs[g].n, w), 1u << 30);
    gu[g] = (int)((max_elems(graphs[g].n, w) + kElemsPerUnit - 1) / kElemsPerUnit);
  }
  return b + work_bytes(u) + work_bytes(gu) + work_bytes(rv);
}
}  // namespace
}  // namespace csc

extern "C" size_t csc_estimate_workspace_bytes_batched(const csc_graph* graphs, int32_t G,
                                                       const int32_t* n_signals, int32_t p) {
  if (!graphs || G < 1 || !n_signals || p < 1) return 0;
  return estimate_bytes_batched(graphs, G, n_signals, p, batch_count_group());
}

extern "C" csc_status csc_estimate_lambda_k_batched(
    const csc_graph* graphs, int32_t G, const int32_t* k, int32_t p, const int32_t* n_signals,
    const uint64_t* seeds, int32_t max_steps, const double* brackets, const float* mlp_params,
    double* lambda_out, int32_t* steps_out, double* trace_out, double* moments_out,
    int32_t* status_out, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graphs(graphs, G));
  CSC_REQUIRE(!(brackets && mlp_params), "give either brackets or mlp_params, not both");
  CSC_REQUIRE(!mlp_params || (p >= 50 && max_steps >= 2),
              "the learned bracket needs p >= 50 and max_steps >= 2");
  CSC_REQUIRE(k && n_signals && seeds && lambda_out && steps_out && status_out,
              "k, n_signals, seeds, lambda_out, steps_out and status_out must be non-NULL");
  CSC_REQUIRE(p >= 1 && max_steps >= 1, "need p >= 1 and max_steps >= 1");
  for (int g = 0; g < G; ++g) {
    CSC_REQUIRE(k[g] >= 1 && k[g] <= graphs[g].n, "k[g] must lie in [1, N_g]");
    CSC_REQUIRE(n_signals[g] >= 1, "n_signals[g] must be >= 1");
    if (brackets)
      CSC_REQUIRE(brackets[2 * g] >= 0.0 && brackets[2 * g + 1] <= 2.0 &&
                      brackets[2 * g] < brackets[2 * g + 1],
                  "brackets must satisfy 0 <= lo < hi <= 2");
  }
  // each round runs `gc` consecutive tests of every graph still searching in
  // one pass (their signals side by side), as the single-graph dichotomy does;
  // the setting is read once, and the workspace is checked against it
  const int gc = batch_count_group();
  CSC_TRY(check_ws(ws, ws_bytes, estimate_bytes_batched(graphs, G, n_signals, p, gc)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);

  std::vector<Layout> L(G);
  const int msteps = moment_steps(p), nraw = moment_raw(p);
  std::vector<int> tiles(G), units(G), gunits(G), rvec(G, gc * nraw);
  std::vector<float*> T0(G), Ta(G), Tb(G);
  std::vector<double*> part(G);
  for (int g = 0; g < G; ++g) {
    const int w = count_width(n_signals[g], gc);
    L[g] = make_layout(graphs[g].n, w, choose_panel_width(graphs[g].n, w, graphs[g].nnz));
    tiles[g] = tiles_for(L[g]);
    units[g] = L[g].np * tiles[g];
    gunits[g] = elem_units(L[g].elems());
    T0[g] = ar.take<float>(L[g].elems());
    Ta[g] = ar.take<float>(L[g].elems());
    Tb[g] = ar.take<float>(L[g].elems());
    part[g] = ar.take<double>((size_t)gc * nraw * units[g] * kMomSlots);
  }
  double* mom = ar.take<double>((size_t)G * gc * nraw);
  StepArgs* d_steps = ar.take<StepArgs>((size_t)msteps * G);
  GaussItem* d_gauss = ar.take<GaussItem>(G);
  ReduceItem* d_red = ar.take<ReduceItem>(G);
  int* d_live = ar.take<int>(G);
  WorkList w_step, w_gauss, w_red;
  plan_work(ar, units, kStepChunk, w_step, xcd_batched());
  plan_work(ar, gunits, chunk_for(gunits), w_gauss);
  plan_work(ar, rvec, 1, w_red);
  float* d_x = ar.take<float>((size_t)G * 52);
  float* d_y = ar.take<float>((size_t)G * 2);
  char* d_mws = ar.take<char>(mlp_workspace(G));
  if (!ar.ok()) {
    set_error("internal: batched workspace plan overflow");
    return CSC_E_INVALID_ARG;
  }

  // per-step descriptors never change between passes
  std::vector<StepArgs> h_steps((size_t)msteps * G);
  std::vector<ReduceItem> h_red(G);
  std::vector<GaussItem> h_gauss(G);
  for (int g = 0; g < G; ++g) {
    for (int m = 0; m < msteps; ++m) {
      StepArgs& a = h_steps[(size_t)m * G + g];
      a.L = L[g];
      a.tiles = tiles[g];
      a.row_ptr = graphs[g].row_ptr;
      a.col = graphs[g].col;
      a.val = graphs[g].val;
      a.sched = step_sched(graphs[g], L[g]);
      a.T0 = T0[g];
      apply_tuning(a);
      a.xcd = 0;
      a.live = d_live + g;
      const bool first = m == 0;
      a.Tm = first ? T0[g] : ((m & 1) ? Ta[g] : Tb[g]);
      a.Tprev = first ? T0[g] : ((m - 1) == 0 ? T0[g] : (((m - 1) & 1) ? Ta[g] : Tb[g]));
      a.Tnext = ((m + 1) & 1) ? Ta[g] : Tb[g];
      const size_t nslots = (size_t)units[g] * kMomSlots;
      a.part = part[g] + (size_t)(2 * m + 1) * nslots;
      a.part2 = part[g] + (size_t)(2 * m + 2) * nslots;
      a.part0 = part[g];
      a.mgroup = gc;
      a.mnc4 = gc > 1 ? round4(n_signals[g]) : n_signals[g];
      a.mstride = (size_t)nraw * nslots;
    }
    h_red[g].part = part[g];
    h_red[g].len = units[g] * kMomSlots;
    h_red[g].out = mom + (size_t)g * gc * nraw;
    h_red[g].live = d_live + g;
    h_gauss[g].L = L[g];
    h_gauss[g].seed = seeds[g];
    h_gauss[g].sid = CSC_STREAM_COUNT;
    h_gauss[g].out = T0[g];
    h_gauss[g].live = d_live + g;
    if (gc > 1) {
      h_gauss[g].nc = n_signals[g];
      h_gauss[g].nc4 = round4(n_signals[g]);
    }
  }
  CSC_TRY(upload(d_steps, h_steps, s));
  CSC_TRY(upload(d_red, h_red, s));
  CSC_TRY(upload(w_step.d, w_step.h, s));
  CSC_TRY(upload(w_gauss.d, w_gauss.h, s));
  CSC_TRY(upload(w_red.d, w_red.h, s));

  auto pass = [&](hipStream_t st) -> csc_status {
    CSC_HIP(launch_gaussian_batched(d_gauss, w_gauss.table(), st));
    for (int m = 0; m < msteps; ++m)
      CSC_HIP(launch_cheb_step_batched(d_steps + (size_t)m * G, w_step.table(),
                                       gc > 1 ? EPI_MOMG : EPI_MOM, m == 0, m + 1 == msteps, st));
    CSC_HIP(launch_reduce_batched(d_red, w_red.table(), st));
    return CSC_OK;
  };

  struct State {
    double lo = 0.0, hi = 2.0;
    int used = 0, t_in = 0, attempt = 0;
    bool below = false, above = false, missed = false, done = false;
    LearnedState ls;  // learned mode, after the first pass
  };
  std::vector<State> st(G);
  for (int g = 0; g < G; ++g)
    if (brackets) {
      st[g].lo = brackets[2 * g];
      st[g].hi = brackets[2 * g + 1];
    }
  std::vector<int> live(G);
  std::vector<double> hraw((size_t)G * gc * nraw), hmom((size_t)G * gc * (p + 1));
  std::vector<float> hx((size_t)G * 52, 0.f), hy((size_t)G * 2, 0.f);
  Captured cap;
  const int rounds = mlp_params ? max_steps : 2 * max_steps;
  for (int round = 0; round < rounds; ++round) {
    int nlive = 0;
    for (int g = 0; g < G; ++g) {
      live[g] = st[g].done ? 0 : 1;
      nlive += live[g];
      h_gauss[g].t = (uint32_t)(st[g].used + 1);
    }
    if (nlive == 0) break;
    CSC_TRY(upload(d_live, live, s));
    CSC_TRY(upload(d_gauss, h_gauss, s));
    CSC_TRY(run_pass(pass, cap, s));
    CSC_HIP(hipMemcpyAsync(hraw.data(), mom, hraw.size() * sizeof(double), hipMemcpyDeviceToHost,
                           s));
    CSC_HIP(hipStreamSynchronize(s));
    for (int g = 0; g < G; ++g)
      if (live[g])
        for (int j = 0; j < gc; ++j)
          moments_from_raw(hraw.data() + ((size_t)g * gc + j) * nraw, p,
                           hmom.data() + ((size_t)g * gc + j) * (p + 1));
    // the round's tests one position at a time, every graph in turn (a graph
    // that finishes leaves the rest of its group unused)
    for (int j = 0; j < gc; ++j) {
      bool need_mlp = false;
      for (int g = 0; g < G; ++g) {
        if (!live[g] || st[g].done) continue;
        State& S = st[g];
        const double* mg = hmom.data() + ((size_t)g * gc + j) * (p + 1);
        const double mid = (mlp_params && S.used > 0) ? 0.5 * (S.ls.lo + S.ls.hi)
                                                      : 0.5 * (S.lo + S.hi);
        const double cnt = count_from_moments(mid, p, mg);
        if (S.used == 0 && moments_out)
          std::memcpy(moments_out + (size_t)g * (p + 1), mg, (p + 1) * sizeof(double));
        if (trace_out) {
          trace_out[((size_t)g * 2 * max_steps + S.used) * 2] = mid;
          trace_out[((size_t)g * 2 * max_steps + S.used) * 2 + 1] = cnt;
        }
        ++S.used;
        ++S.t_in;
        if (mlp_params) {
          // learned mode: the first pass picks the half and feeds the network
          if (S.used == 1) {
            if (std::floor(cnt + 0.5) == (double)k[g]) {
              lambda_out[g] = mid;
              status_out[g] = CSC_OK;
              S.done = true;
            } else {
              learned_features(mg, graphs[g].n, k[g], hx.data() + (size_t)g * 52);
              S.ls.half_lo = cnt;  // first count, consumed by learned_begin below
              need_mlp = true;
            }
            continue;
          }
          if (learned_update(S.ls, mid, cnt, k[g])) {
            lambda_out[g] = mid;
            status_out[g] = S.ls.status;
            S.done = true;
          } else if (S.used == max_steps) {
            lambda_out[g] = S.ls.hi;
            status_out[g] = S.ls.status == CSC_OK ? CSC_W_BISECT_EXHAUSTED : S.ls.status;
            S.done = true;
          }
          continue;
        }
        if (std::floor(cnt + 0.5) == (double)k[g]) {
          lambda_out[g] = mid;
          status_out[g] = S.missed ? CSC_W_BRACKET_MISS : CSC_OK;
          S.done = true;
          continue;
        }
        if (cnt < k[g]) {
          S.lo = mid;
          S.below = true;
        } else {
          S.hi = mid;
          S.above = true;
        }
        if (S.t_in == max_steps) {
          if (brackets && S.attempt == 0 && !(S.below && S.above)) {
            S.missed = true;
            S.attempt = 1;
            S.t_in = 0;
            S.lo = 0.0;
            S.hi = 2.0;
          } else {
            lambda_out[g] = S.hi;
            status_out[g] = S.missed ? CSC_W_BRACKET_MISS : CSC_W_BISECT_EXHAUSTED;
            S.done = true;
          }
        }
      }
      if (need_mlp) {
        CSC_TRY(upload(d_x, hx, s));
        CSC_TRY(csc_mlp_forward(mlp_params, d_x, G, d_y, d_mws, mlp_workspace(G), stream));
        CSC_HIP(hipMemcpyAsync(hy.data(), d_y, hy.size() * sizeof(float),
                               hipMemcpyDeviceToHost, s));
        CSC_HIP(hipStreamSynchronize(s));
        for (int g = 0; g < G; ++g) {
          State& S = st[g];
          if (!live[g] || S.done || S.used != 1) continue;
          const double c1 = S.ls.half_lo;
          learned_begin(S.ls, hmom.data() + ((size_t)g * gc + j) * (p + 1), p, k[g], n_signals[g],
                        c1, hy.data() + (size_t)g * 2);
        }
      }
    }
  }
  for (int g = 0; g < G; ++g) steps_out[g] = st[g].used;
  return CSC_OK;
}

// ---------------------------------------------------------- feature pass ---
extern "C" size_t csc_filter_workspace_bytes_batched(const csc_graph* graphs, int32_t G,
                                                     const int32_t* d, int32_t p) {
  if (!graphs || G < 1 || !d || p < 1) return 0;
  size_t b = desc_bytes(G, p);
  std::vector<int> u(G), gu(G);
  for (int g = 0; g < G; ++g) {
    b += max_widths(graphs[g].n, d[g], [](const Layout& L) { return filter_bytes(L); });
    u[g] = (int)max_units(graphs[g].n, d[g]);
    gu[g] = (int)((max_elems(graphs[g].n, d[g]) + kElemsPerUnit - 1) / kElemsPerUnit);
  }
  // second descriptor set and work list: all-row graphs run the accumulated pass
  return b + align_up((size_t)p * G * sizeof(StepArgs)) + 2 * work_bytes(u) + work_bytes(gu);
}

extern "C" csc_status csc_filter_batched(const csc_graph* graphs, int32_t G, const double* lambda,
                                         int32_t p, const int32_t* d, const uint64_t* seeds,
                                         const int32_t* const* rows, const int32_t* n_rows,
                                         int32_t normalize, float* const* Y, const int32_t* ld,
                                         void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graphs(graphs, G));
  CSC_REQUIRE(lambda && d && seeds && rows && n_rows && Y && ld,
              "lambda, d, seeds, rows, n_rows, Y and ld must be non-NULL");
  CSC_REQUIRE(p >= 1, "p must be >= 1");
  for (int g = 0; g < G; ++g) {
    CSC_REQUIRE(lambda[g] >= 0.0 && lambda[g] <= 2.0, "lambda[g] must lie in [0, 2]");
    CSC_REQUIRE(d[g] >= 1 && ld[g] >= d[g], "need d[g] >= 1 and ld[g] >= d[g]");
    CSC_REQUIRE(Y[g] && (rows[g] == nullptr || (n_rows[g] >= 1 && n_rows[g] <= graphs[g].n)),
                "Y[g] must be non-NULL, and 1 <= n_rows[g] <= N_g when rows[g] is given");
  }
  CSC_TRY(check_ws(ws, ws_bytes, csc_filter_workspace_bytes_batched(graphs, G, d, p)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  std::vector<Layout> L(G);
  std::vector<int> tiles(G), units(G), gunits(G);
  // graphs with sampled rows run the forward recurrence with the sampled-row
  // epilogue; graphs with all rows run the accumulated pass in the process-wide
  // form, exactly as csc_filter does, so every output matches csc_filter's
  std::vector<float*> T0(G), Ta(G), Tb(G), Yi(G);
  std::vector<int*> slot(G);
  std::vector<int> units_s(G, 0), units_a(G, 0);
  for (int g = 0; g < G; ++g) {
    L[g] = make_layout(graphs[g].n, d[g], choose_panel_width(graphs[g].n, d[g], graphs[g].nnz));
    tiles[g] = tiles_for(L[g]);
    units[g] = L[g].np * tiles[g];
    (rows[g] ? units_s : units_a)[g] = units[g];
    gunits[g] = elem_units(L[g].elems());
    T0[g] = ar.take<float>(L[g].elems());
    Ta[g] = ar.take<float>(L[g].elems());
    Tb[g] = ar.take<float>(L[g].elems());
    Yi[g] = ar.take<float>(L[g].elems());
    slot[g] = ar.take<int>(graphs[g].n);
  }
  StepArgs* d_steps = ar.take<StepArgs>((size_t)p * G);
  StepArgs* d_steps_a = ar.take<StepArgs>((size_t)p * G);
  GaussItem* d_gauss = ar.take<GaussItem>(G);
  int* bad = ar.take<int>(G);
  WorkList w_step, w_step_a, w_gauss;
  plan_work(ar, units_s, kStepChunk, w_step, xcd_batched());
  plan_work(ar, units_a, kStepChunk, w_step_a, xcd_batched());
  plan_work(ar, gunits, chunk_for(gunits), w_gauss);
  if (!ar.ok()) {
    set_error("internal: batched workspace plan overflow");
    return CSC_E_INVALID_ARG;
  }
  std::vector<StepArgs> h_steps((size_t)p * G), h_steps_a((size_t)p * G);
  std::vector<GaussItem> h_gauss(G);
  std::vector<double> a(p + 1);
  const int form = filter_form();
  std::vector<PassStep> plan0;
  for (int g = 0; g < G; ++g) {
    jackson_lowpass(lambda[g], p, a.data());
    const std::vector<PassStep> plan = pass_plan(EPI_Y, a.data(), p, T0[g], Ta[g], Tb[g], form);
    if (plan0.empty()) plan0 = plan;
    for (int m = 0; m < p; ++m) {
      StepArgs& x = h_steps_a[(size_t)m * G + g];
      x.L = L[g];
      x.tiles = tiles[g];
      x.row_ptr = graphs[g].row_ptr;
      x.col = graphs[g].col;
      x.val = graphs[g].val;
      x.sched = step_sched(graphs[g], L[g]);
      x.T0 = T0[g];
      x.Y = Yi[g];
      apply_tuning(x);
      x.xcd = 0;
      x.Tm = plan[m].Tm;
      x.Tprev = plan[m].Tprev;
      x.Tnext = plan[m].Tnext;
      x.c0 = plan[m].c0;
      x.c1 = plan[m].c1;
    }
    for (int m = 0; m < p; ++m) {
      StepArgs& x = h_steps[(size_t)m * G + g];
      x.L = L[g];
      x.tiles = tiles[g];
      x.row_ptr = graphs[g].row_ptr;
      x.col = graphs[g].col;
      x.val = graphs[g].val;
      x.sched = step_sched(graphs[g], L[g]);
      x.T0 = T0[g];
      apply_tuning(x);
      x.xcd = 0;
      const bool first = m == 0;
      x.Tm = first ? T0[g] : ((m & 1) ? Ta[g] : Tb[g]);
      x.Tprev = first ? T0[g] : ((m - 1) == 0 ? T0[g] : (((m - 1) & 1) ? Ta[g] : Tb[g]));
      x.Tnext = ((m + 1) & 1) ? Ta[g] : Tb[g];
      x.c0 = (float)a[0];
      x.c1 = (float)a[m + 1];
      x.slot = slot[g];
      x.Ys = Y[g];
      x.lds = ld[g];
    }
    h_gauss[g].L = L[g];
    h_gauss[g].seed = seeds[g];
    h_gauss[g].t = 0;
    h_gauss[g].sid = CSC_STREAM_FEAT;
    h_gauss[g].out = T0[g];
  }
  CSC_TRY(upload(d_steps, h_steps, s));
  CSC_TRY(upload(d_steps_a, h_steps_a, s));
  CSC_TRY(upload(d_gauss, h_gauss, s));
  CSC_TRY(upload(w_step.d, w_step.h, s));
  CSC_TRY(upload(w_step_a.d, w_step_a.h, s));
  CSC_TRY(upload(w_gauss.d, w_gauss.h, s));
  CSC_HIP(launch_fill_i32(bad, G, 0, s));
  for (int g = 0; g < G; ++g) {
    if (rows[g]) {
      CSC_HIP(launch_fill_i32(slot[g], graphs[g].n, -1, s));
      CSC_HIP(launch_slot_map(n_rows[g], rows[g], graphs[g].n, slot[g], bad + g, s));
    }
  }
  std::vector<int> hbad(G);
  CSC_HIP(hipMemcpyAsync(hbad.data(), bad, G * sizeof(int), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  for (int g = 0; g < G; ++g)
    if (hbad[g]) {
      set_error("rows[" + std::to_string(g) + "] holds an index outside [0, N)");
      return CSC_E_INVALID_ARG;
    }
  CSC_HIP(launch_gaussian_batched(d_gauss, w_gauss.table(), s));
  for (int m = 0; m < p; ++m) {
    CSC_HIP(launch_cheb_step_batched(d_steps + (size_t)m * G, w_step.table(), EPI_YS, m == 0,
                                     m + 1 == p, s));
    CSC_HIP(launch_cheb_step_batched(d_steps_a + (size_t)m * G, w_step_a.table(), plan0[m].epi,
                                     plan0[m].first, plan0[m].last, s));
  }
  for (int g = 0; g < G; ++g) {
    if (rows[g]) {
      if (normalize) CSC_HIP(launch_normalize_rows(n_rows[g], d[g], Y[g], ld[g], s));
    } else {
      CSC_HIP(launch_unpack(L[g], Yi[g], Y[g], ld[g], normalize, s));
    }
  }
  return CSC_OK;
}

// --------------------------------------------------------- interpolation ---
extern "C" size_t csc_interpolate_workspace_bytes_batched(const csc_graph* graphs, int32_t G,
                                                          const int32_t* k, int32_t p) {
  if (!graphs || G < 1 || !k || p < 1) return 0;
  size_t b = desc_bytes(G, p) + align_up((size_t)G * 4 * sizeof(int));
  std::vector<int> u(G), kv(G), u2(G), lu(G);
  for (int g = 0; g < G; ++g) {
    b += max_widths(graphs[g].n, k[g], [](const Layout& L) { return interp_bytes(L); });
    b += perm_bytes(graphs[g].n, graphs[g].nnz, graphs[g].n);
    u[g] = (int)max_units(graphs[g].n, k[g]);
    kv[g] = k[g];
    u2[g] = (int)((max_elems(graphs[g].n, k[g]) / 4 + kElemsPerUnit - 1) / kElemsPerUnit);
    lu[g] = (graphs[g].n + 255) / 256;
  }
  return b + work_bytes(u) + work_bytes(kv) + work_bytes(u2) + work_bytes(lu);
}

extern "C" csc_status csc_interpolate_batched(
    const csc_graph* graphs, int32_t G, const int32_t* const* order, int32_t method,
    const double* lambda,
    int32_t p, double gamma, const int32_t* const* idx_in, const int32_t* const* labels_r,
    const float* const* weights, const int32_t* n, const int32_t* k,
    double tol, int32_t max_iter, float* const* X, const int32_t* ldx, int32_t* const* labels,
    int32_t* iters_out, double* relres_out, int32_t* status_out, void* ws, size_t ws_bytes,
    void* stream) {
  clear_error();
  CSC_TRY(check_graphs(graphs, G));
  CSC_REQUIRE(lambda && idx_in && labels_r && n && k && labels && status_out,
              "lambda, idx, labels_r, n, k, labels and status_out must be non-NULL");
  CSC_REQUIRE(p >= 1 && gamma > 0.0 && tol > 0.0 && max_iter >= 1,
              "need p >= 1, gamma > 0, tol > 0, max_iter >= 1");
  CSC_REQUIRE(method == CSC_CG_COLUMNS || method == CSC_CG_BLOCK || method == CSC_CG_BLOCK_JACOBI,
              "method must be CSC_CG_COLUMNS, CSC_CG_BLOCK or CSC_CG_BLOCK_JACOBI");
  for (int g = 0; g < G; ++g) {
    const int N = graphs[g].n;
    CSC_REQUIRE(idx_in[g] && labels_r[g] && labels[g],
                "idx[g], labels_r[g], labels[g] must be non-NULL");
    CSC_REQUIRE(k[g] >= 1 && k[g] <= N && n[g] >= 1 && n[g] <= N,
                "need 1 <= k[g] <= N_g and 1 <= n[g] <= N_g");
    CSC_REQUIRE(lambda[g] >= 0.0 && lambda[g] <= 2.0, "lambda[g] must lie in [0, 2]");
    CSC_REQUIRE(!X || !X[g] || (ldx && ldx[g] >= k[g]), "ldx[g] must be >= k[g]");
  }
  CSC_TRY(check_ws(ws, ws_bytes, csc_interpolate_workspace_bytes_batched(graphs, G, k, p)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);

  struct Buf {
    Layout L;
    int tiles, units, u2;
    size_t wp;
    float *P, *Ta, *Tb, *AP, *Xi, *Rr, *mask;
    double *part, *rr, *rrn, *pAp, *alpha, *beta, *bnorm2, *colnorm2, *relres;
    int *active, *iters;
    float* Z;  // block CG
    double *gpart, *G, *S_t, *S_a, *S_na, *S_b;
  };
  std::vector<Buf> B(G);
  for (int g = 0; g < G; ++g) {
    Buf& b = B[g];
    const int N = graphs[g].n;
    b.L = make_layout(N, k[g], choose_panel_width(N, k[g], graphs[g].nnz));
    b.tiles = tiles_for(b.L);
    b.units = b.L.np * b.tiles;
    b.u2 = elem_units(b.L.elems() / 4);
    b.wp = (size_t)b.L.np * b.L.pw;
    b.P = ar.take<float>(b.L.elems());
    b.Ta = ar.take<float>(b.L.elems());
    b.Tb = ar.take<float>(b.L.elems());
    b.AP = ar.take<float>(b.L.elems());
    b.Xi = ar.take<float>(b.L.elems());
    b.Rr = ar.take<float>(b.L.elems());
    b.mask = ar.take<float>(N);
    b.part = ar.take<double>(b.wp * b.tiles);
    b.rr = ar.take<double>(b.wp);
    b.rrn = ar.take<double>(b.wp);
    b.pAp = ar.take<double>(b.wp);
    b.alpha = ar.take<double>(b.wp);
    b.beta = ar.take<double>(b.wp);
    b.bnorm2 = ar.take<double>(b.wp);
    b.colnorm2 = ar.take<double>(b.wp);
    b.active = ar.take<int>(b.wp);
    b.iters = ar.take<int>(b.wp);
    b.relres = ar.take<double>(b.wp);
    const size_t kk = (size_t)k[g] * k[g];
    b.Z = ar.take<float>(b.L.elems());
    b.gpart = ar.take<double>(gram_part_elems(b.L, b.L.w));
    b.G = ar.take<double>(kk);
    b.S_t = ar.take<double>(kk);
    b.S_a = ar.take<double>(kk);
    b.S_na = ar.take<double>(kk);
    b.S_b = ar.take<double>(kk);
  }
  int* flags = ar.take<int>((size_t)G * 4);  // per graph: nactive, breakdown, bad, it
  int* d_live = ar.take<int>(G);
  StepArgs* d_steps = ar.take<StepArgs>((size_t)p * G);
  ReduceItem* d_red_pap = ar.take<ReduceItem>(G);
  ReduceItem* d_red_rrn = ar.take<ReduceItem>(G);
  CgItem* d_cg = ar.take<CgItem>(G);
  ColDotItem* d_cd = ar.take<ColDotItem>(G);
  LabelItem* d_lab = ar.take<LabelItem>(G);
  std::vector<int> units(G), kvec(G), u2(G), lunits(G);
  for (int g = 0; g < G; ++g) {
    units[g] = B[g].units;
    kvec[g] = k[g];
    u2[g] = B[g].u2;
    lunits[g] = (graphs[g].n + 255) / 256;  // kb_labels: one row per thread, 256 per unit
  }
  WorkList w_step, w_k, w_u2, w_lab;
  plan_work(ar, units, kStepChunk, w_step, xcd_batched());
  plan_work(ar, kvec, 1, w_k);
  plan_work(ar, u2, chunk_for(u2), w_u2);
  plan_work(ar, lunits, chunk_for(lunits), w_lab);
  if (!ar.ok()) {
    set_error("internal: batched workspace plan overflow");
    return CSC_E_INVALID_ARG;
  }
  // graphs with a node order run on their permuted copy
  std::vector<csc_graph> gv(graphs, graphs + G);
  std::vector<const int32_t*> idx(idx_in, idx_in + G);
  for (int g = 0; g < G; ++g)
    if (order && order[g])
      CSC_TRY(permuted_graph(graphs[g], order[g], idx_in[g], n[g], ar, gv[g], idx[g], s));

  // set-up, graph by graph: zero blocks, scatter the right-hand sides, ||b_j||^2
  CSC_HIP(launch_fill_i32(flags, (size_t)G * 4, 0, s));
  std::vector<int> live(G, 1);
  CSC_TRY(upload(d_live, live, s));
  for (int g = 0; g < G; ++g) {
    Buf& b = B[g];
    CSC_HIP(launch_fill_f32(b.P, b.L.elems(), 0.f, s));
    CSC_HIP(launch_fill_f32(b.Xi, b.L.elems(), 0.f, s));
    CSC_HIP(launch_fill_f32(b.Rr, b.L.elems(), 0.f, s));
    CSC_HIP(launch_fill_f32(b.mask, graphs[g].n, 0.f, s));
    CSC_HIP(launch_fill_i32(b.iters, b.wp, 0, s));
    CSC_HIP(launch_fill_f64(b.relres, b.wp, 0.0, s));
    CSC_HIP(launch_cg_scatter(b.L, n[g], idx[g], labels_r[g], weights ? weights[g] : nullptr, b.Rr,
                              b.P, b.mask,
                              flags + 4 * g + 2, s));
    CSC_HIP(launch_col_dot(b.L, b.Rr, b.Rr, b.part, s));
    CSC_HIP(launch_reduce(b.part, col_dot_chunks(b.L), k[g], b.bnorm2, s));
    CSC_HIP(hipMemcpyAsync(b.rr, b.bnorm2, k[g] * sizeof(double), hipMemcpyDeviceToDevice, s));
  }
  std::vector<int> hflags((size_t)G * 4);
  CSC_HIP(hipMemcpyAsync(hflags.data(), flags, hflags.size() * sizeof(int),
                         hipMemcpyDeviceToHost, s));
  std::vector<std::vector<double>> hb(G);
  for (int g = 0; g < G; ++g) {
    hb[g].resize(k[g]);
    CSC_HIP(hipMemcpyAsync(hb[g].data(), B[g].bnorm2, k[g] * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  }
  CSC_HIP(hipStreamSynchronize(s));
  for (int g = 0; g < G; ++g) {
    if (hflags[4 * g + 2]) {
      set_error("idx[" + std::to_string(g) + "] or labels_r[" + std::to_string(g) +
                "] holds a value out of range");
      return CSC_E_INVALID_ARG;
    }
  }
  {
    std::vector<std::vector<int>> ha(G);
    for (int g = 0; g < G; ++g) {
      ha[g].resize(k[g]);
      for (int j = 0; j < k[g]; ++j) ha[g][j] = hb[g][j] > 0.0 ? 1 : 0;
      CSC_HIP(hipMemcpyAsync(B[g].active, ha[g].data(), k[g] * sizeof(int),
                             hipMemcpyHostToDevice, s));
    }
    CSC_HIP(hipStreamSynchronize(s));
  }

  // descriptors of one CG iteration
  const int form = filter_form();
  std::vector<PassStep> plan0;
  std::vector<StepArgs> h_steps((size_t)p * G);
  std::vector<ReduceItem> h_pap(G), h_rrn(G);
  std::vector<CgItem> h_cg(G);
  std::vector<double> a(p + 1);
  for (int g = 0; g < G; ++g) {
    const Buf& b = B[g];
    jackson_lowpass(lambda[g], p, a.data());
    // the same launch sequence as the single-graph pass (epilogue and flags
    // per step depend on p only, so one batched launch per step serves all)
    const std::vector<PassStep> plan_g = pass_plan(EPI_CG, a.data(), p, b.P, b.Ta, b.Tb, form);
    if (g == 0) plan0 = plan_g;
    for (int m = 0; m < p; ++m) {
      StepArgs& x = h_steps[(size_t)m * G + g];
      x.L = b.L;
      x.tiles = b.tiles;
      x.row_ptr = gv[g].row_ptr;
      x.col = gv[g].col;
      x.val = gv[g].val;
      x.sched = step_sched(gv[g], b.L);
      x.T0 = b.P;
      x.Y = b.AP;
      x.mask = b.mask;
      x.gamma = (float)gamma;
      x.part = b.part;
      apply_tuning(x);
      x.xcd = 0;
      x.live = d_live + g;
      const PassStep& ps = plan_g[m];
      x.Tm = ps.Tm;
      x.Tprev = ps.Tprev;
      x.Tnext = ps.Tnext;
      x.c0 = ps.c0;
      x.c1 = ps.c1;
    }
    h_pap[g] = ReduceItem{b.part, b.tiles, b.pAp, d_live + g};
    h_rrn[g] = ReduceItem{b.part, b.tiles, b.rrn, d_live + g};
    CgItem& c = h_cg[g];
    c.L = b.L;
    c.tiles = b.tiles;
    c.k = k[g];
    c.AP = b.AP;
    c.P = b.P;
    c.X = b.Xi;
    c.R = b.Rr;
    c.rr = b.rr;
    c.rrn = b.rrn;
    c.pAp = b.pAp;
    c.alpha = b.alpha;
    c.beta = b.beta;
    c.bnorm2 = b.bnorm2;
    c.active = b.active;
    c.iters = b.iters;
    c.relres = b.relres;
    c.part = b.part;
    c.nactive = flags + 4 * g;
    c.breakdown = flags + 4 * g + 1;
    c.it = flags + 4 * g + 3;
    c.tol = tol;
    c.max_iter = max_iter;
    c.live = d_live + g;
  }
  CSC_TRY(upload(d_steps, h_steps, s));
  CSC_TRY(upload(d_red_pap, h_pap, s));
  CSC_TRY(upload(d_red_rrn, h_rrn, s));
  CSC_TRY(upload(d_cg, h_cg, s));
  CSC_TRY(upload(w_step.d, w_step.h, s));
  CSC_TRY(upload(w_k.d, w_k.h, s));
  CSC_TRY(upload(w_u2.d, w_u2.h, s));
  CSC_TRY(upload(w_lab.d, w_lab.h, s));

  if (method != CSC_CG_COLUMNS) {
    // every graph's block CG; the Chebyshev pass Q = M P of all graphs still
    // iterating is one batched launch per step
    std::vector<BlockState> bs(G);
    for (int g = 0; g < G; ++g) {
      const Buf& b = B[g];
      CSC_TRY(block_init(bs[g], b.L, k[g], tol, method == CSC_CG_BLOCK_JACOBI, (float)gamma,
                         BlockBufs{b.P, b.AP, b.Ta, b.Tb, b.Xi, b.Rr, b.Z, b.mask, b.part,
                                   b.gpart, b.G, b.S_t, b.S_a, b.S_na, b.S_b, b.rrn},
                         b.bnorm2, s));
    }
    auto filter_pass = [&](hipStream_t st) -> csc_status {
      for (int m = 0; m < p; ++m) {
        const PassStep& ps = plan0[m];
        CSC_HIP(launch_cheb_step_batched(d_steps + (size_t)m * G, w_step.table(),
                                         ps.epi, ps.first, ps.last, st));
      }
      return CSC_OK;
    };
    // each stage of the iteration runs for every graph before the next one:
    // one synchronisation per stage, the host algebra of the graphs in parallel
    auto unfinished = [&]() {
      std::vector<int> v;
      for (int g = 0; g < G; ++g)
        if (!bs[g].finished) v.push_back(g);
      return v;
    };
    Captured cap_pass;
    for (int it = 1; it <= max_iter; ++it) {
      std::vector<int> act = unfinished();
      if (act.empty()) break;
      for (int g : act) CSC_TRY(pre_launch(bs[g], s));
      CSC_HIP(hipStreamSynchronize(s));
      host_parallel(act, [&](int g) { pre_host(bs[g]); });
      bool any = false;
      for (int g = 0; g < G; ++g) {
        live[g] = bs[g].finished ? 0 : 1;
        any = any || live[g];
        if (live[g]) CSC_TRY(pre_finish(bs[g], s));
      }
      if (!any) break;
      CSC_TRY(upload(d_live, live, s));
      CSC_TRY(run_pass(filter_pass, cap_pass, s));
      act = unfinished();
      for (int g : act) CSC_TRY(post_launch_a(bs[g], s));
      CSC_HIP(hipStreamSynchronize(s));
      host_parallel(act, [&](int g) { post_host_a(bs[g]); });
      act = unfinished();
      if (act.empty()) continue;
      for (int g : act) CSC_TRY(post_launch_b(bs[g], s));
      CSC_HIP(hipStreamSynchronize(s));
      host_parallel(act, [&](int g) { post_host_b(bs[g], it, max_iter); });
      for (int g : unfinished()) CSC_TRY(post_finish(bs[g], s));
    }
    std::vector<ColDotItem> h_cd(G);
    std::vector<ReduceItem> h_cn(G);
    std::vector<LabelItem> h_lab(G);
    for (int g = 0; g < G; ++g) {
      CSC_TRY(block_join(bs[g]));
      block_finish(bs[g], max_iter);
      const Buf& b = B[g];
      h_cd[g] = ColDotItem{b.L, col_dot_chunks(b.L), col_dot_rows(b.L), b.Xi, b.Xi, b.part,
                           nullptr};
      h_cn[g] = ReduceItem{b.part, col_dot_chunks(b.L), b.colnorm2, nullptr};
      h_lab[g] = LabelItem{b.L, b.Xi, b.colnorm2, labels[g], X ? X[g] : nullptr,
                           (X && X[g]) ? ldx[g] : 0, order ? order[g] : nullptr};
    }
    CSC_TRY(upload(d_cd, h_cd, s));
    CSC_TRY(upload(d_red_pap, h_cn, s));
    CSC_TRY(upload(d_lab, h_lab, s));
    CSC_HIP(launch_col_dot_batched(d_cd, w_step.table(), s));
    CSC_HIP(launch_reduce_batched(d_red_pap, w_k.table(), s));
    CSC_HIP(launch_labels_batched(d_lab, w_lab.table(), s));
    CSC_HIP(hipStreamSynchronize(s));
    csc_status worst = CSC_OK;
    size_t off = 0;
    for (int g = 0; g < G; ++g) {
      if (iters_out) std::memcpy(iters_out + off, bs[g].iters.data(), k[g] * sizeof(int));
      if (relres_out) std::memcpy(relres_out + off, bs[g].relres.data(), k[g] * sizeof(double));
      off += k[g];
      const bool ok = bs[g].converged && !bs[g].broke;
      status_out[g] = ok ? CSC_OK : CSC_W_NOT_CONVERGED;
      if (!ok) worst = CSC_W_NOT_CONVERGED;
    }
    return worst;
  }

  auto iteration = [&](hipStream_t st) -> csc_status {
    for (int m = 0; m < p; ++m) {
      const PassStep& ps = plan0[m];
      CSC_HIP(launch_cheb_step_batched(d_steps + (size_t)m * G, w_step.table(),
                                       ps.epi, ps.first, ps.last, st));
    }
    CSC_HIP(launch_reduce_batched(d_red_pap, w_k.table(), st));
    CSC_HIP(launch_cg_alpha_batched(d_cg, G, st));
    CSC_HIP(launch_cg_update1_batched(d_cg, w_step.table(), st));
    CSC_HIP(launch_reduce_batched(d_red_rrn, w_k.table(), st));
    CSC_HIP(launch_cg_scalar_batched(d_cg, G, st));
    CSC_HIP(launch_cg_update2_batched(d_cg, w_u2.table(), st));
    return CSC_OK;
  };
  Captured cap;
  for (int it = 1; it <= max_iter; ++it) {
    CSC_TRY(run_pass(iteration, cap, s));
    CSC_HIP(hipMemcpyAsync(live.data(), d_live, G * sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    bool any = false;
    for (int g = 0; g < G; ++g) any = any || live[g];
    if (!any) break;
  }

  // column norms of X and hard labels
  std::vector<ColDotItem> h_cd(G);
  std::vector<ReduceItem> h_cn(G);
  std::vector<LabelItem> h_lab(G);
  for (int g = 0; g < G; ++g) {
    const Buf& b = B[g];
    h_cd[g] = ColDotItem{b.L, col_dot_chunks(b.L), col_dot_rows(b.L), b.Xi, b.Xi, b.part, nullptr};
    h_cn[g] = ReduceItem{b.part, col_dot_chunks(b.L), b.colnorm2, nullptr};
    h_lab[g] = LabelItem{b.L, b.Xi, b.colnorm2, labels[g], X ? X[g] : nullptr,
                         (X && X[g]) ? ldx[g] : 0, order ? order[g] : nullptr};
  }
  CSC_TRY(upload(d_cd, h_cd, s));
  CSC_TRY(upload(d_red_pap, h_cn, s));
  CSC_TRY(upload(d_lab, h_lab, s));
  CSC_HIP(launch_col_dot_batched(d_cd, w_step.table(), s));
  CSC_HIP(launch_reduce_batched(d_red_pap, w_k.table(), s));
  CSC_HIP(launch_labels_batched(d_lab, w_lab.table(), s));

  CSC_HIP(hipMemcpyAsync(hflags.data(), flags, hflags.size() * sizeof(int),
                         hipMemcpyDeviceToHost, s));
  size_t off = 0;
  std::vector<std::vector<int>> hit(G);
  std::vector<std::vector<double>> hrel(G);
  for (int g = 0; g < G; ++g) {
    hit[g].resize(k[g]);
    hrel[g].resize(k[g]);
    CSC_HIP(hipMemcpyAsync(hit[g].data(), B[g].iters, k[g] * sizeof(int), hipMemcpyDeviceToHost,
                           s));
    CSC_HIP(hipMemcpyAsync(hrel[g].data(), B[g].relres, k[g] * sizeof(double),
                           hipMemcpyDeviceToHost, s));
  }
  CSC_HIP(hipStreamSynchronize(s));
  csc_status worst = CSC_OK;
  for (int g = 0; g < G; ++g) {
    if (iters_out) std::memcpy(iters_out + off, hit[g].data(), k[g] * sizeof(int));
    if (relres_out) std::memcpy(relres_out + off, hrel[g].data(), k[g] * sizeof(double));
    off += k[g];
    const bool unfinished = hflags[4 * g] > 0 || hflags[4 * g + 1] != 0;
    status_out[g] = unfinished ? CSC_W_NOT_CONVERGED : CSC_OK;
    if (unfinished) worst = CSC_W_NOT_CONVERGED;
  }
  return worst;
}
