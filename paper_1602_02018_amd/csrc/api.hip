// C ABI of libcsc: argument checks, workspace carving and the host side of
// Alg. 2 (dichotomy loop, CG loop).  Every arithmetic step on graph-sized data
// runs in the kernels of kernels.hip.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <tuple>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <thread>
#include <vector>

#include "dense.hpp"
#include "host.hpp"

namespace csc {

// largest polynomial order of csc_filter_noalloc (its coefficients live on the stack)
constexpr int kNoallocMaxOrder = 4096;

namespace {
thread_local std::string g_error;
std::atomic<int> g_panel_override{0};
std::atomic<int> g_tune_xcd{1};
std::atomic<int> g_filter_form{FORM_CLENSHAW};
std::atomic<int> g_damping{CSC_DAMP_JACKSON};
std::atomic<int> g_tune_nt{0};
std::atomic<int> g_tune_graphs{1};
std::atomic<int> g_tune_sched{1};
std::atomic<int> g_tune_group{4};
std::atomic<int> g_tune_bgroup{1};
std::atomic<int> g_tune_bprod{0};
}  // namespace

bool block_product_f32() { return g_tune_bprod.load() != 0; }

void set_error(const std::string& msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

Tuning tuning() {
  Tuning t;
  t.xcd = g_tune_xcd.load();
  t.nt = g_tune_nt.load();
  return t;
}

int use_hip_graphs() { return g_tune_graphs.load(); }
int count_group() { return g_tune_group.load(); }
int batch_count_group() { return g_tune_bgroup.load(); }
bool xcd_batched() { return g_tune_xcd.load() != 0; }

// Stream used only to record HIP graphs (kernels are captured, never run on
// it); one per device, default priority, kept for the life of the process.
hipStream_t capture_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

// Second stream for work that overlaps the caller's stream (the signals of
// the next eigencount pass); one per device, default priority, kept for the
// life of the process.  Ordering with the caller's stream goes through events.
hipStream_t side_stream() {
  static std::mutex mu;
  static hipStream_t streams[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev] && hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking) != hipSuccess)
    streams[dev] = nullptr;
  return streams[dev];
}

void apply_tuning(StepArgs& sa) {
  const Tuning t = tuning();
  sa.xcd = t.xcd;
  sa.nt = t.nt;
}

const int* step_sched(const csc_graph& g, const Layout& L) {
  if (!g.sched || L.pw < 4) return nullptr;
  const int mode = g_tune_sched.load();
  const int rows_per_wave = 64 / (L.pw / 4);
  if (mode == 2 && rows_per_wave >= 2) return g.sched;
  // measured on a 1e6-node power-law graph: the degree-sorted walk gains only
  // where a wave holds exactly 8 rows (panels of 29-32 columns; moment step
  // 1.23x, Clenshaw step 1.04x) and loses 5-38% at every other width, most
  // where a wave holds many short rows (64 rows per wave: 868 vs 540 us)
  if (mode == 1 && rows_per_wave == 8) return g.sched;
  return nullptr;
}

// Panel width PW = 4 * lanes-per-row.  A Chebyshev step is bound by the
// 128-byte cache lines it gathers: a neighbour row of PW floats starting at
// byte offset 4*PW*j touches (4PW + 128 - gcd(4PW, 128)) / 128 lines on
// average.  The choice minimises, per row and step, gathered line bytes
// (deg * 128 * lines per panel) + streamed bytes (16 per padded column)
// + CSR bytes re-read for every panel (8 deg + 4).
double panel_cost(int n, int w, long long nnz, int pw);

namespace {
// Autotuner results: panel width per shape bucket (log2 N, rounded mean
// degree, width).  Written by csc_autotune, read by every later call.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned;

std::tuple<int, int, int> shape_key(int n, int w, long long nnz) {
  int lg = 0;
  while ((1LL << (lg + 1)) <= (long long)n) ++lg;
  const int deg = n > 0 ? (int)std::lround((double)nnz / n) : 0;
  return std::make_tuple(lg, deg, w);
}
}  // namespace

int choose_panel_width(int n, int w, long long nnz) {
  const int o = g_panel_override.load();
  if (o) return o;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    auto it = g_tuned.find(shape_key(n, w, nnz));
    if (it != g_tuned.end()) return it->second;
  }
  int arg = 4;
  double best = 0.0;
  for (int pw = 4; pw <= 256; pw += 4) {
    const double c = panel_cost(n, w, nnz, pw);
    if (pw == 4 || c < best) {
      best = c;
      arg = pw;
    }
  }
  return arg;
}

double panel_cost(int n, int w, long long nnz, int pw) {
  const double deg = n > 0 ? (double)nnz / n : 16.0;
  const int np = (w + pw - 1) / pw;
  const int b = 4 * pw;
  int g = 128;
  while (b % g) g >>= 1;
  const double lines = (double)(b + 128 - g) / 128.0;
  return np * (deg * 128.0 * lines + 16.0 * pw + 8.0 * deg + 4.0);
}

Layout make_layout(int n, int w, int pw) {
  Layout L;
  L.n = n;
  L.w = w;
  L.pw = pw;
  L.np = (w + pw - 1) / pw;
  return L;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

csc_status check_graph(const csc_graph* g) {
  CSC_REQUIRE(g != nullptr, "graph is NULL");
  CSC_REQUIRE(g->n >= 1, "graph must have at least one node");
  CSC_REQUIRE(g->nnz >= 0, "nnz must be non-negative");
  CSC_REQUIRE(g->row_ptr != nullptr, "graph row_ptr is NULL");
  CSC_REQUIRE(g->nnz == 0 || (g->col != nullptr && g->val != nullptr),
              "graph col/val are NULL");
  return CSC_OK;
}

csc_status check_ws(void* ws, size_t ws_bytes, size_t need) {
  if (need == 0) return CSC_OK;
  CSC_REQUIRE(ws != nullptr, "workspace is NULL");
  CSC_REQUIRE(((uintptr_t)ws % 256) == 0, "workspace must be 256-byte aligned");
  if (ws_bytes < need) {
    set_error("workspace too small: need " + std::to_string(need) + " bytes, got " +
              std::to_string(ws_bytes));
    return CSC_E_INVALID_ARG;
  }
  return CSC_OK;
}

// Jackson-Chebyshev coefficients of the ideal low-pass at lc (Sec. 4.3).
void jackson_lowpass(double lc, int p, double* a) {
  const bool damp = g_damping.load() == CSC_DAMP_JACKSON;
  const double pi = 3.14159265358979323846;
  double xc = lc - 1.0;
  xc = xc < -1.0 ? -1.0 : (xc > 1.0 ? 1.0 : xc);
  const double th = std::acos(xc);
  const double al = pi / (p + 2);
  for (int m = 0; m <= p; ++m) {
    const double c = m == 0 ? 1.0 - th / pi : -2.0 * std::sin(m * th) / (m * pi);
    const double g = ((p + 2 - m) * std::cos(m * al) + std::sin(m * al) / std::tan(al)) / (p + 2);
    a[m] = damp ? g * c : c;
  }
}

namespace {

// Buffers of one p-step pass.
struct Pass {
  const float* T0 = nullptr;
  float* Ta = nullptr;
  float* Tb = nullptr;
  float* Y = nullptr;
  double* part = nullptr;  // EPI_MOM: moment_raw(p) x nblocks kMomSlots; EPI_CG: columns x tiles
  const int* slot = nullptr;
  float* Ys = nullptr;
  int lds = 0;
  const float* mask = nullptr;
  float gamma = 0.f;
  int mgroup = 1;  // EPI_MOM: passes side by side, mnc4 columns each
  int mnc4 = 0;
  int form = -1;   // EPI_Y / EPI_CG: filter form of this pass (-1: the process-wide setting)
};

}  // namespace

int filter_form() { return g_filter_form.load(); }

std::vector<PassStep> pass_plan(int epi, const double* a, int p, const float* T0, float* Ta,
                                float* Tb, int form) {
  std::vector<PassStep> out;
  if (form == FORM_CLENSHAW) {
    // b_m = a_m T0 + 2 (L - I) b_{m+1} - b_{m+2} for m = p-1 .. 1 (b_p = a_p T0
    // is folded into the coefficients, never stored), then
    // h~(L) T0 = a_0 T0 + (L - I) b_1 - b_2; b_m lives in Ta (m odd) or Tb.
    auto buf = [&](int m) { return (m & 1) ? Ta : Tb; };
    for (int m = p - 1; m >= 0; --m) {
      PassStep st;
      const bool top = m + 1 == p;
      st.Tm = top ? T0 : buf(m + 1);
      st.c1 = (float)((m >= 1 ? -2.0 : -1.0) * (top ? a[p] : 1.0));
      st.c0 = (float)(a[m] - (m + 2 == p ? a[p] : 0.0));
      st.first = !(m + 2 <= p - 1);  // no stored b_{m+2}
      st.Tprev = st.first ? nullptr : buf(m + 2);
      st.Tnext = m >= 1 ? buf(m) : nullptr;
      st.last = m == 0;
      st.epi = m >= 1 ? EPI_CLEN : (epi == EPI_CG ? EPI_CLEN_CG : EPI_CLEN_Y);
      out.push_back(st);
    }
    return out;
  }
  for (int m = 0; m < p; ++m) {  // step m produces T_{m+1}
    PassStep st;
    st.first = m == 0;
    st.last = m + 1 == p;
    st.Tm = st.first ? T0 : ((m & 1) ? Ta : Tb);
    st.Tprev = st.first ? T0 : ((m - 1) == 0 ? T0 : (((m - 1) & 1) ? Ta : Tb));
    st.Tnext = ((m + 1) & 1) ? Ta : Tb;
    st.c0 = (float)a[0];
    st.c1 = (float)a[m + 1];
    st.epi = (epi == EPI_CG && st.last) ? EPI_CG : EPI_Y;
    out.push_back(st);
  }
  return out;
}

namespace {

// h~(L) applied to T0 by the Chebyshev recurrence; `epi` selects the
// consumer of each T_{m+1}.  For epi == EPI_CG the steps before the last
// accumulate into Y and the last one forms the CG operator.
csc_status chebyshev_pass(const csc_graph& g, const Layout& L, const double* a, int p, int epi,
                          const Pass& b, hipStream_t s) {
  StepArgs sa;
  sa.L = L;
  sa.tiles = tiles_for(L);
  sa.row_ptr = g.row_ptr;
  sa.col = g.col;
  sa.val = g.val;
  sa.sched = step_sched(g, L);
  sa.T0 = b.T0;
  sa.Y = b.Y;
  sa.slot = b.slot;
  sa.Ys = b.Ys;
  sa.lds = b.lds;
  sa.mask = b.mask;
  sa.gamma = b.gamma;
  apply_tuning(sa);
  const size_t nblocks = (size_t)L.np * sa.tiles;
  if (epi == EPI_Y || epi == EPI_CG) {
    for (const PassStep& st : pass_plan(epi, a, p, b.T0, b.Ta, b.Tb,
                                        b.form >= 0 ? b.form : filter_form())) {
      sa.Tm = st.Tm;
      sa.Tprev = st.Tprev;
      sa.Tnext = st.Tnext;
      sa.c0 = st.c0;
      sa.c1 = st.c1;
      sa.part = b.part;
      CSC_HIP(launch_cheb_step(sa, st.epi, st.first, st.last, s));
    }
    return CSC_OK;
  }
  if (epi == EPI_MOM && b.mgroup > 1) epi = EPI_MOMG;
  const int steps = (epi == EPI_MOM || epi == EPI_MOMG) ? moment_steps(p) : p;
  for (int m = 0; m < steps; ++m) {  // step m produces T_{m+1}
    const bool first = m == 0, last = m + 1 == steps;
    sa.Tm = first ? b.T0 : ((m & 1) ? b.Ta : b.Tb);
    sa.Tprev = first ? b.T0 : ((m - 1) == 0 ? b.T0 : (((m - 1) & 1) ? b.Ta : b.Tb));
    sa.Tnext = ((m + 1) & 1) ? b.Ta : b.Tb;
    sa.c0 = (float)a[0];
    sa.c1 = (float)a[m + 1];
    int e = epi;
    if (epi == EPI_MOM || epi == EPI_MOMG) {
      const size_t nslots = nblocks * kMomSlots;
      sa.part = b.part + (size_t)(2 * m + 1) * nslots;
      sa.part2 = b.part + (size_t)(2 * m + 2) * nslots;
      sa.part0 = b.part;
      sa.mgroup = b.mgroup;
      sa.mnc4 = b.mnc4;
      sa.mstride = (size_t)moment_raw(p) * nslots;
    } else if (epi == EPI_CG) {
      e = last ? EPI_CG : EPI_Y;
      sa.part = b.part;
    }
    CSC_HIP(launch_cheb_step(sa, e, first, last, s));
  }
  return CSC_OK;
}

}  // namespace

// ------------------------------------------------------ workspace plans ---
size_t filter_bytes(const Layout& L) {
  size_t b = 0;
  b += 4 * align_up(L.bytes());                // T0, Ta, Tb, Y
  b += align_up((size_t)L.n * sizeof(int));    // slot map
  b += align_up(4 * sizeof(int));              // bad-index flag
  return b + 256;
}

int moment_steps(int p) { return (p + 1) / 2; }
int moment_raw(int p) { return 2 * moment_steps(p) + 1; }

void moments_from_raw(const double* raw, int p, double* mom) {
  mom[0] = raw[0];
  if (p >= 1) mom[1] = raw[1];
  for (int m = 2; m <= p; ++m)
    mom[m] = (m & 1) ? 2.0 * raw[m] - raw[1] : 2.0 * raw[m] - raw[0];
}

size_t count_bytes(const Layout& L, int p, int group) {
  const size_t nblocks = (size_t)L.np * tiles_for(L);
  size_t b = 4 * align_up(L.bytes());  // two signal blocks, two recurrence blocks
  b += align_up((size_t)group * moment_raw(p) * nblocks * kMomSlots * sizeof(double));
  b += align_up((size_t)group * moment_raw(p) * sizeof(double));
  return b + 256;
}

size_t interp_bytes(const Layout& L) {
  const size_t tiles = tiles_for(L), wp = (size_t)L.np * L.pw, kk = (size_t)L.w * L.w;
  size_t b = 6 * align_up(L.bytes());
  b += align_up((size_t)L.n * sizeof(float));          // mask
  b += align_up(wp * tiles * sizeof(double));          // column partials
  b += 7 * align_up(wp * sizeof(double));              // rr rrn pAp alpha beta bnorm2 colnorm2
  b += 2 * align_up(wp * sizeof(int));                 // active iters
  b += align_up(wp * sizeof(double));                  // relres
  b += align_up(4 * sizeof(int));                      // nactive, breakdown
  // block CG: Z, Gram partials, Gram results, four small coefficient matrices
  b += align_up(L.bytes()) + align_up(gram_part_elems(L, L.w) * sizeof(double));
  b += 5 * align_up(kk * sizeof(double));
  return b + 256;
}

namespace {
template <class F>
size_t max_over_widths(int n, int w, F f) {
  size_t m = 0;
  for (int pw = 4; pw <= 256; pw += 4) m = std::max(m, f(make_layout(n, w, pw)));
  return m;
}

// ------------------------------------------------------------ eigencount ---
struct CountBuffers {
  float* T0;
  float* T0n;  // the next pass's signals (dichotomy)
  float* Ta;
  float* Tb;
  double* part;
  double* mom;
};

CountBuffers carve_count(Arena& ar, const Layout& L, int p, int group = 1) {
  const size_t nblocks = (size_t)L.np * tiles_for(L);
  CountBuffers c;
  c.T0 = ar.take<float>(L.elems());
  c.T0n = ar.take<float>(L.elems());
  c.Ta = ar.take<float>(L.elems());
  c.Tb = ar.take<float>(L.elems());
  c.part = ar.take<double>((size_t)group * moment_raw(p) * nblocks * kMomSlots);
  c.mom = ar.take<double>((size_t)group * moment_raw(p));
  return c;
}

// Draws eigencount signal blocks on the side stream, ordered against the
// caller's stream s by events: the side stream starts after s's earlier work
// (the workspace may still be in use), s waits for a draw before the pass
// that reads it and, when this object goes, for the last draw.  Off (draw()
// does nothing and passes draw their own signals) without a side stream or
// events.
// How a count pass lays out its signals: one test (g == 1: n_signals
// columns, drawn by launch_gaussian_panels) or g consecutive tests side by
// side, nc4 columns each.
struct CountGroup {
  int g = 1, nc = 1, nc4 = 1;
};

hipError_t draw_count_signals(const Layout& L, const CountGroup& cg, uint64_t seed, uint32_t t,
                              float* out, hipStream_t s) {
  if (cg.g == 1) return launch_gaussian_panels(L, seed, t, CSC_STREAM_COUNT, out, s);
  return launch_gaussian_group(L, seed, t, CSC_STREAM_COUNT, cg.nc, cg.nc4, out, s);
}

class SignalAhead {
 public:
  explicit SignalAhead(hipStream_t s) : s_(s), s2_(side_stream()) {
    if (!s2_) return;
    if (hipEventCreateWithFlags(&start_, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&drawn_, hipEventDisableTiming) != hipSuccess ||
        hipEventRecord(start_, s_) != hipSuccess || hipStreamWaitEvent(s2_, start_, 0) != hipSuccess)
      s2_ = nullptr;
  }
  ~SignalAhead() {
    if (s2_ && pending_) (void)hipStreamWaitEvent(s_, drawn_, 0);
    if (start_) (void)hipEventDestroy(start_);
    if (drawn_) (void)hipEventDestroy(drawn_);
  }
  SignalAhead(const SignalAhead&) = delete;
  SignalAhead& operator=(const SignalAhead&) = delete;
  bool on() const { return s2_ != nullptr; }
  csc_status draw(const Layout& L, const CountGroup& cg, uint64_t seed, uint32_t t, float* out) {
    if (!s2_) return CSC_OK;
    CSC_HIP(draw_count_signals(L, cg, seed, t, out, s2_));
    CSC_HIP(hipEventRecord(drawn_, s2_));
    pending_ = true;
    return CSC_OK;
  }
  // s waits for the last draw
  csc_status wait() {
    if (!s2_ || !pending_) return CSC_OK;
    CSC_HIP(hipStreamWaitEvent(s_, drawn_, 0));
    pending_ = false;
    return CSC_OK;
  }

 private:
  hipStream_t s_;
  hipStream_t s2_;
  hipEvent_t start_ = nullptr, drawn_ = nullptr;
  bool pending_ = false;
};

// One eigencount pass on the signals of pass t: drawn into c.T0 first, or
// already in T0 (drawn ahead by the caller) when T0 is given.
// With a group, the passes of tests t .. t + g - 1 at once, moments of test
// t + j in mom_host[j (p + 1) ..].  `between` runs on the host as soon as the
// pass's steps are enqueued: before the copy of the moments, which, into
// pageable host memory, returns only once the pass has run (work that
// `between` enqueues on another stream then overlaps the pass).
csc_status moments_pass(const csc_graph& g, const Layout& L, int p, uint64_t seed, uint32_t t,
                        const CountBuffers& c, double* mom_host, hipStream_t s,
                        const float* T0 = nullptr,
                        const std::function<csc_status()>& between = nullptr,
                        const CountGroup& cg = CountGroup{}) {
  const size_t nblocks = (size_t)L.np * tiles_for(L);
  if (!T0) CSC_HIP(draw_count_signals(L, cg, seed, t, c.T0, s));
  Pass b;
  b.T0 = T0 ? T0 : c.T0;
  b.Ta = c.Ta;
  b.Tb = c.Tb;
  b.part = c.part;
  b.mgroup = cg.g;
  b.mnc4 = cg.nc4;
  std::vector<double> zero(p + 1, 0.0);
  CSC_TRY(chebyshev_pass(g, L, zero.data(), p, EPI_MOM, b, s));
  if (between) CSC_TRY(between());
  const int nraw = moment_raw(p);
  CSC_HIP(launch_reduce(c.part, (int)(nblocks * kMomSlots), cg.g * nraw, c.mom, s));
  std::vector<double> raw((size_t)cg.g * nraw);
  CSC_HIP(hipMemcpyAsync(raw.data(), c.mom, raw.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  for (int j = 0; j < cg.g; ++j)
    moments_from_raw(raw.data() + (size_t)j * nraw, p, mom_host + (size_t)j * (p + 1));
  return CSC_OK;
}

}  // namespace

double count_from_moments(double lambda, int p, const double* mom) {
  std::vector<double> a(p + 1);
  jackson_lowpass(lambda, p, a.data());
  double c = 0.0;
  for (int m = 0; m <= p; ++m) c += a[m] * mom[m];
  return c;
}

csc_status count_passes(const csc_graph& g, int n_signals, int p, uint64_t seed, uint32_t t0,
                        void* ws, size_t ws_bytes, hipStream_t s,
                        const std::function<bool(uint32_t, const double*)>& more) {
  CountGroup cg;
  cg.g = count_group();
  cg.nc = n_signals;
  cg.nc4 = cg.g > 1 ? round4(n_signals) : n_signals;
  const int w = cg.g * cg.nc4;
  const Layout L = make_layout(g.n, w, choose_panel_width(g.n, w, g.nnz));
  CSC_TRY(check_ws(ws, ws_bytes, count_bytes(L, p, cg.g)));
  Arena ar(ws, ws_bytes);
  const CountBuffers c = carve_count(ar, L, p, cg.g);
  // the signals of the next group of tests are drawn on a second stream
  // while the current group runs (they do not depend on its counts); the two
  // signal blocks alternate
  SignalAhead ahead(s);
  float* blocks[2] = {c.T0, c.T0n};
  CSC_TRY(ahead.draw(L, cg, seed, t0, blocks[0]));
  std::vector<double> mom((size_t)cg.g * (p + 1));
  for (uint32_t t = t0, k = 0;; t += (uint32_t)cg.g, ++k) {
    const float* cur = blocks[k & 1];
    CSC_TRY(ahead.wait());
    // the group is enqueued first, then the next draw, so that it starts as
    // early as possible
    CSC_TRY(moments_pass(g, L, p, seed, t, c, mom.data(), s, ahead.on() ? cur : nullptr,
                         [&] { return ahead.draw(L, cg, seed, t + cg.g, blocks[(k + 1) & 1]); },
                         cg));
    for (int j = 0; j < cg.g; ++j)
      if (!more(t + (uint32_t)j, mom.data() + (size_t)j * (p + 1))) return CSC_OK;
  }
}

}  // namespace csc

using namespace csc;

// ===================================================================== ABI ==
extern "C" const char* csc_last_error(void) { return g_error.c_str(); }

extern "C" int32_t csc_version(void) { return 100; }

extern "C" csc_status csc_set_panel_width(int32_t pw) {
  clear_error();
  CSC_REQUIRE(pw == 0 || (pw >= 4 && pw <= 256 && pw % 4 == 0),
              "panel width must be 0 or a multiple of 4 in [4, 256]");
  g_panel_override.store(pw);
  return CSC_OK;
}

extern "C" int32_t csc_get_panel_width(int32_t n, int64_t nnz, int32_t w) {
  return choose_panel_width(n, w, nnz);
}

extern "C" csc_status csc_set_damping(int32_t damping) {
  clear_error();
  CSC_REQUIRE(damping == CSC_DAMP_JACKSON || damping == CSC_DAMP_NONE,
              "damping must be CSC_DAMP_JACKSON or CSC_DAMP_NONE");
  g_damping.store(damping);
  return CSC_OK;
}

extern "C" int32_t csc_get_damping(void) { return g_damping.load(); }

extern "C" csc_status csc_set_filter_form(int32_t form) {
  clear_error();
  CSC_REQUIRE(form == CSC_FORM_FORWARD || form == CSC_FORM_CLENSHAW,
              "form must be CSC_FORM_FORWARD or CSC_FORM_CLENSHAW");
  g_filter_form.store(form);
  return CSC_OK;
}

extern "C" int32_t csc_get_filter_form(void) { return g_filter_form.load(); }

extern "C" csc_status csc_set_tuning(int32_t key, int32_t value) {
  clear_error();
  switch (key) {
    case CSC_TUNE_PANEL_WIDTH:
      return csc_set_panel_width(value);
    case CSC_TUNE_XCD_ORDER:
      CSC_REQUIRE(value >= 0 && value <= 2, "value must be 0, 1 or 2");
      g_tune_xcd.store(value);
      return CSC_OK;
    case CSC_TUNE_NONTEMPORAL:
      CSC_REQUIRE(value == 0 || value == 1, "value must be 0 or 1");
      g_tune_nt.store(value);
      return CSC_OK;
    case CSC_TUNE_HIP_GRAPHS:
      CSC_REQUIRE(value == 0 || value == 1, "value must be 0 or 1");
      g_tune_graphs.store(value);
      return CSC_OK;
    case CSC_TUNE_ROW_SCHED:
      CSC_REQUIRE(value >= 0 && value <= 2, "value must be 0, 1 or 2");
      g_tune_sched.store(value);
      return CSC_OK;
    case CSC_TUNE_COUNT_GROUP:
      CSC_REQUIRE(value >= 1 && value <= kMaxCountGroup, "value must lie in 1..4");
      g_tune_group.store(value);
      return CSC_OK;
    case CSC_TUNE_BATCH_COUNT_GROUP:
      CSC_REQUIRE(value >= 1 && value <= kMaxCountGroup, "value must lie in 1..4");
      g_tune_bgroup.store(value);
      return CSC_OK;
    case CSC_TUNE_BLOCK_PRODUCT:
      CSC_REQUIRE(value == 0 || value == 1, "value must be 0 or 1");
      g_tune_bprod.store(value);
      return CSC_OK;
    default:
      CSC_REQUIRE(false, "unknown tuning key");
  }
}

extern "C" int32_t csc_get_tuning(int32_t key) {
  switch (key) {
    case CSC_TUNE_PANEL_WIDTH: return g_panel_override.load();
    case CSC_TUNE_XCD_ORDER: return g_tune_xcd.load();
    case CSC_TUNE_NONTEMPORAL: return g_tune_nt.load();
    case CSC_TUNE_HIP_GRAPHS: return g_tune_graphs.load();
    case CSC_TUNE_ROW_SCHED: return g_tune_sched.load();
    case CSC_TUNE_COUNT_GROUP: return g_tune_group.load();
    case CSC_TUNE_BATCH_COUNT_GROUP: return g_tune_bgroup.load();
    case CSC_TUNE_BLOCK_PRODUCT: return g_tune_bprod.load();
    default: return -1;
  }
}

extern "C" csc_status csc_laplacian_from_adjacency(int32_t n, int32_t nnz, const int32_t* row_ptr,
                                                   const int32_t* col, const float* w,
                                                   float* val_out, float* dinv_sqrt_out,
                                                   int32_t check, void* stream) {
  clear_error();
  CSC_REQUIRE(n >= 1 && nnz >= 0, "n must be >= 1 and nnz >= 0");
  CSC_REQUIRE(row_ptr && dinv_sqrt_out, "row_ptr and dinv_sqrt_out must be non-NULL");
  CSC_REQUIRE(nnz == 0 || (col && val_out), "col and val_out must be non-NULL");
  hipStream_t s = as_stream(stream);
  if (check) {
    int* flag = nullptr;
    // the flag lives in the output array of scales until the check is done
    flag = reinterpret_cast<int*>(dinv_sqrt_out);
    CSC_HIP(launch_fill_i32(flag, 1, 0, s));
    CSC_HIP(launch_check_csr(n, nnz, row_ptr, col, flag, s));
    int h = 0;
    CSC_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (h) {
      set_error("malformed CSR (flags " + std::to_string(h) +
                "): row_ptr must start at 0, end at nnz and be non-decreasing; columns in [0, n)");
      return CSC_E_GRAPH;
    }
    if (check >= 2 && nnz > 0) {
      CSC_HIP(launch_fill_i32(flag, 1, 0, s));
      CSC_HIP(launch_check_graph_strict(n, row_ptr, col, w, flag, s));
      CSC_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
      CSC_HIP(hipStreamSynchronize(s));
      if (h) {
        std::string why;
        if (h & 16) why += " a self-loop (stored diagonal entry);";
        if (h & 32) why += " a row whose columns are not strictly increasing;";
        if (h & 64) why += " W not symmetric (entry (j, i) missing or with another weight);";
        set_error("graph rejected:" + why);
        return CSC_E_GRAPH;
      }
    }
  }
  CSC_HIP(launch_degree_scale(n, row_ptr, col, w, dinv_sqrt_out, s));
  if (nnz > 0) CSC_HIP(launch_adjacency_values(n, row_ptr, col, w, dinv_sqrt_out, val_out, s));
  return CSC_OK;
}

extern "C" csc_status csc_jackson_coeffs(double lambda_c, int32_t p, double* a_out) {
  clear_error();
  CSC_REQUIRE(a_out != nullptr, "a_out is NULL");
  CSC_REQUIRE(p >= 0, "p must be >= 0");
  CSC_REQUIRE(lambda_c >= 0.0 && lambda_c <= 2.0, "lambda_c must lie in [0, 2]");
  jackson_lowpass(lambda_c, p, a_out);
  return CSC_OK;
}

extern "C" csc_status csc_gaussian_block(int32_t n_rows, int32_t w, uint64_t seed, uint32_t t,
                                         uint32_t stream_id, float* R, int32_t ld, void* stream) {
  clear_error();
  CSC_REQUIRE(n_rows >= 0 && w >= 1 && ld >= w, "need n_rows >= 0, w >= 1, ld >= w");
  CSC_REQUIRE(R != nullptr || n_rows == 0, "R is NULL");
  if (n_rows == 0) return CSC_OK;
  CSC_HIP(launch_gaussian_rows(n_rows, w, seed, t, stream_id, R, ld, as_stream(stream)));
  return CSC_OK;
}

extern "C" size_t csc_filter_workspace_bytes(int32_t n, int32_t w) {
  if (n < 1 || w < 1) return 0;
  return max_over_widths(n, w, [](const Layout& L) { return filter_bytes(L); });
}

namespace {
csc_status filter_common(const csc_graph* g, const double* a, int p, int w, const float* Xin,
                         int ldx, bool draw, uint64_t seed, const int32_t* rows, int n_rows,
                         int normalize, float* Y, int ld, void* ws, size_t ws_bytes,
                         hipStream_t s) {
  const int n = g->n;
  const Layout L = make_layout(n, w, choose_panel_width(n, w, g->nnz));
  CSC_TRY(check_ws(ws, ws_bytes, filter_bytes(L)));
  Arena ar(ws, ws_bytes);
  float* T0 = ar.take<float>(L.elems());
  float* Ta = ar.take<float>(L.elems());
  float* Tb = ar.take<float>(L.elems());
  float* Yi = ar.take<float>(L.elems());
  int* slot = ar.take<int>(n);
  int* bad = ar.take<int>(4);
  if (draw)
    CSC_HIP(launch_gaussian_panels(L, seed, 0, CSC_STREAM_FEAT, T0, s));
  else
    CSC_HIP(launch_pack(L, Xin, ldx, T0, s));
  Pass b;
  b.T0 = T0;
  b.Ta = Ta;
  b.Tb = Tb;
  if (rows) {
    CSC_HIP(launch_fill_i32(slot, n, -1, s));
    CSC_HIP(launch_fill_i32(bad, 1, 0, s));
    CSC_HIP(launch_slot_map(n_rows, rows, n, slot, bad, s));
    int hbad = 0;
    CSC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (hbad) {
      set_error("rows holds an index outside [0, N)");
      return CSC_E_INVALID_ARG;
    }
    b.slot = slot;
    b.Ys = Y;
    b.lds = ld;
    CSC_TRY(chebyshev_pass(*g, L, a, p, EPI_YS, b, s));
    if (normalize) CSC_HIP(launch_normalize_rows(n_rows, w, Y, ld, s));
  } else {
    b.Y = Yi;
    CSC_TRY(chebyshev_pass(*g, L, a, p, EPI_Y, b, s));
    CSC_HIP(launch_unpack(L, Yi, Y, ld, normalize, s));
  }
  return CSC_OK;
}
}  // namespace

extern "C" csc_status csc_filter_block(const csc_graph* g, const double* coeffs, int32_t p,
                                       const float* X, int32_t w, int32_t ld, float* Y, void* ws,
                                       size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(coeffs && X && Y, "coeffs, X and Y must be non-NULL");
  CSC_REQUIRE(p >= 1, "p must be >= 1");
  CSC_REQUIRE(w >= 1 && ld >= w, "need w >= 1 and ld >= w");
  return filter_common(g, coeffs, p, w, X, ld, false, 0, nullptr, 0, 0, Y, ld, ws, ws_bytes,
                       as_stream(stream));
}

extern "C" csc_status csc_filter(const csc_graph* g, double lambda_c, int32_t p, int32_t d,
                                 uint64_t seed, const int32_t* rows, int32_t n_rows,
                                 int32_t normalize, float* Y, int32_t ld, void* ws,
                                 size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(Y != nullptr, "Y is NULL");
  CSC_REQUIRE(p >= 1, "p must be >= 1");
  CSC_REQUIRE(d >= 1 && ld >= d, "need d >= 1 and ld >= d");
  CSC_REQUIRE(lambda_c >= 0.0 && lambda_c <= 2.0, "lambda_c must lie in [0, 2]");
  CSC_REQUIRE(rows == nullptr || (n_rows >= 1 && n_rows <= g->n),
              "n_rows must lie in [1, N] when rows is given");
  std::vector<double> a(p + 1);
  jackson_lowpass(lambda_c, p, a.data());
  return filter_common(g, a.data(), p, d, nullptr, 0, true, seed, rows, n_rows, normalize, Y, ld,
                       ws, ws_bytes, as_stream(stream));
}

// ----------------------------------------------- feature pass, no alloc ---
namespace {
// Scratch of csc_filter_noalloc: one array per device, held for the life of
// the process.  Host code never passes the array's name to a kernel (on the
// host it is only a stand-in for the symbol); it uses the device address
// returned by hipGetSymbolAddress, looked up once per device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

csc_status scratch_for_current_device(void** out) {
  int dev = 0;
  CSC_HIP(hipGetDevice(&dev));
  CSC_REQUIRE(dev >= 0 && dev < kMaxDevices, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
      return CSC_E_HIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return CSC_OK;
}
}  // namespace

extern "C" size_t csc_filter_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" csc_status csc_filter_noalloc(const csc_graph* g, double lambda_c, int32_t p, int32_t d,
                                         uint64_t seed, const int32_t* rows, int32_t n_rows,
                                         int32_t normalize, float* Y, int32_t ld, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(Y != nullptr, "Y is NULL");
  CSC_REQUIRE(p >= 1 && p <= kNoallocMaxOrder, "p must lie in [1, 4096]");
  CSC_REQUIRE(d >= 1 && ld >= d, "need d >= 1 and ld >= d");
  CSC_REQUIRE(lambda_c >= 0.0 && lambda_c <= 2.0, "lambda_c must lie in [0, 2]");
  CSC_REQUIRE(rows == nullptr || (n_rows >= 1 && n_rows <= g->n),
              "n_rows must lie in [1, N] when rows is given");
  const Layout L = make_layout(g->n, d, choose_panel_width(g->n, d, g->nnz));
  const size_t need = filter_bytes(L);
  if (need > kScratchBytes) {
    set_error("csc_filter_noalloc: this graph and width need " + std::to_string(need) +
              " bytes of scratch, more than the library's fixed " + std::to_string(kScratchBytes) +
              "; use csc_filter with a workspace");
    return CSC_E_INVALID_ARG;
  }
  void* ws = nullptr;
  CSC_TRY(scratch_for_current_device(&ws));
  double a[kNoallocMaxOrder + 1];
  jackson_lowpass(lambda_c, p, a);
  return filter_common(g, a, p, d, nullptr, 0, true, seed, rows, n_rows, normalize, Y, ld, ws,
                       kScratchBytes, as_stream(stream));
}

extern "C" size_t csc_estimate_workspace_bytes(int32_t n, int32_t n_signals, int32_t p) {
  if (n < 1 || n_signals < 1 || p < 1) return 0;
  size_t b = max_over_widths(n, n_signals, [p](const Layout& L) { return count_bytes(L, p); });
  for (int g = 2; g <= kMaxCountGroup; ++g)  // grouped dichotomy passes
    b = std::max(b, max_over_widths(n, g * round4(n_signals),
                                    [p, g](const Layout& L) { return count_bytes(L, p, g); }));
  return b;
}

extern "C" csc_status csc_eigencount(const csc_graph* g, double lambda, int32_t p,
                                     int32_t n_signals, uint64_t seed, uint32_t t,
                                     double* count_out, double* moments_out, void* ws,
                                     size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(count_out != nullptr, "count_out is NULL");
  CSC_REQUIRE(p >= 1 && n_signals >= 1, "need p >= 1 and n_signals >= 1");
  CSC_REQUIRE(lambda >= 0.0 && lambda <= 2.0, "lambda must lie in [0, 2]");
  const Layout L = make_layout(g->n, n_signals, choose_panel_width(g->n, n_signals, g->nnz));
  CSC_TRY(check_ws(ws, ws_bytes, count_bytes(L, p)));
  Arena ar(ws, ws_bytes);
  const CountBuffers c = carve_count(ar, L, p);
  std::vector<double> mom(p + 1);
  CSC_TRY(moments_pass(*g, L, p, seed, t, c, mom.data(), as_stream(stream)));
  *count_out = count_from_moments(lambda, p, mom.data());
  if (moments_out) std::memcpy(moments_out, mom.data(), (p + 1) * sizeof(double));
  return CSC_OK;
}

extern "C" csc_status csc_estimate_lambda_k_kpm(const csc_graph* g, int32_t k, int32_t p,
                                                int32_t n_signals, uint64_t seed,
                                                int32_t max_steps, double* lambda_out,
                                                int32_t* steps_out, double* trace_out,
                                                double* moments_out, void* ws, size_t ws_bytes,
                                                void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(lambda_out && steps_out, "lambda_out and steps_out must be non-NULL");
  CSC_REQUIRE(k >= 1 && k <= g->n, "k must lie in [1, N]");
  CSC_REQUIRE(p >= 1 && n_signals >= 1 && max_steps >= 1,
              "need p >= 1, n_signals >= 1 and max_steps >= 1");
  const Layout L = make_layout(g->n, n_signals, choose_panel_width(g->n, n_signals, g->nnz));
  CSC_TRY(check_ws(ws, ws_bytes, count_bytes(L, p)));
  Arena ar(ws, ws_bytes);
  const CountBuffers c = carve_count(ar, L, p);
  std::vector<double> mom(p + 1);
  CSC_TRY(moments_pass(*g, L, p, seed, 1, c, mom.data(), as_stream(stream)));
  if (moments_out) std::memcpy(moments_out, mom.data(), (p + 1) * sizeof(double));
  double lo = 0.0, hi = 2.0;
  for (int t = 1; t <= max_steps; ++t) {
    const double mid = 0.5 * (lo + hi);
    const double cnt = count_from_moments(mid, p, mom.data());
    if (trace_out) {
      trace_out[2 * (t - 1)] = mid;
      trace_out[2 * (t - 1) + 1] = cnt;
    }
    if (std::floor(cnt + 0.5) == (double)k) {
      *lambda_out = mid;
      *steps_out = t;
      return CSC_OK;
    }
    if (cnt < k)
      lo = mid;
    else
      hi = mid;
  }
  *lambda_out = hi;
  *steps_out = max_steps;
  return CSC_W_BISECT_EXHAUSTED;
}

extern "C" csc_status csc_estimate_lambda_k(const csc_graph* g, int32_t k, int32_t p,
                                            int32_t n_signals, uint64_t seed, int32_t max_steps,
                                            const double* bracket, double* lambda_out,
                                            int32_t* steps_out, double* trace_out,
                                            double* moments_out, void* ws, size_t ws_bytes,
                                            void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(lambda_out && steps_out, "lambda_out and steps_out must be non-NULL");
  CSC_REQUIRE(k >= 1 && k <= g->n, "k must lie in [1, N]");
  CSC_REQUIRE(p >= 1 && n_signals >= 1 && max_steps >= 1,
              "need p >= 1, n_signals >= 1, max_steps >= 1");
  double lo = 0.0, hi = 2.0;
  if (bracket) {
    CSC_REQUIRE(bracket[0] >= 0.0 && bracket[1] <= 2.0 && bracket[0] < bracket[1],
                "bracket must satisfy 0 <= lo < hi <= 2");
    lo = bracket[0];
    hi = bracket[1];
  }
  // pass `used + 1` tests the midpoint of the current bracket; with a caller
  // bracket that the first max_steps passes never straddle, the search
  // restarts once from [0, 2]
  int used = 0, in_attempt = 0, attempt = 0;
  bool below = false, above = false, missed = false, found = false;
  double found_lambda = 0.0;
  auto more = [&](uint32_t, const double* mom) -> bool {
    const double mid = 0.5 * (lo + hi);
    if (used == 0 && moments_out) std::memcpy(moments_out, mom, (p + 1) * sizeof(double));
    const double cnt = count_from_moments(mid, p, mom);
    if (trace_out) {
      trace_out[2 * used] = mid;
      trace_out[2 * used + 1] = cnt;
    }
    ++used;
    ++in_attempt;
    if (std::floor(cnt + 0.5) == (double)k) {
      found = true;
      found_lambda = mid;
      return false;
    }
    if (cnt < k) {
      lo = mid;
      below = true;
    } else {
      hi = mid;
      above = true;
    }
    if (in_attempt < max_steps) return true;
    // exhausted: with a caller bracket, a one-sided history means lambda_k lies outside
    if (bracket && attempt == 0 && !(below && above)) {
      missed = true;
      lo = 0.0;
      hi = 2.0;
      attempt = 1;
      in_attempt = 0;
      return true;
    }
    return false;
  };
  CSC_TRY(count_passes(*g, n_signals, p, seed, 1, ws, ws_bytes, as_stream(stream), more));
  *lambda_out = found ? found_lambda : hi;
  *steps_out = used;
  if (found) return missed ? CSC_W_BRACKET_MISS : CSC_OK;
  return missed ? CSC_W_BRACKET_MISS : CSC_W_BISECT_EXHAUSTED;
}

extern "C" size_t csc_sample_workspace_bytes(int32_t N, int32_t n) {
  if (N < 1 || n < 1) return 0;
  const int nch = sample_chunks(N);
  size_t b = 2 * align_up((size_t)nch * sizeof(int)) + align_up(4 * sizeof(int));
  b += 2 * align_up((size_t)N * sizeof(uint64_t)) + 2 * align_up((size_t)N * sizeof(int));
  b += align_up(sort_pairs_temp_bytes(N));
  return b + 256;
}

extern "C" csc_status csc_sample(int32_t N, int32_t n, uint64_t seed, int32_t* idx, void* ws,
                                 size_t ws_bytes, void* stream) {
  clear_error();
  CSC_REQUIRE(N >= 1 && n >= 1 && n <= N, "need 1 <= n <= N");
  CSC_REQUIRE(idx != nullptr, "idx is NULL");
  CSC_TRY(check_ws(ws, ws_bytes, csc_sample_workspace_bytes(N, n)));
  hipStream_t s = as_stream(stream);
  const int nch = sample_chunks(N);
  Arena ar(ws, ws_bytes);
  int* counts = ar.take<int>(nch);
  int* offsets = ar.take<int>(nch);
  int* total = ar.take<int>(4);
  uint64_t* kin = ar.take<uint64_t>(N);
  uint64_t* kout = ar.take<uint64_t>(N);
  int* vin = ar.take<int>(N);
  int* vout = ar.take<int>(N);
  const size_t temp_bytes = sort_pairs_temp_bytes(N);
  void* temp = ar.take<char>(temp_bytes);
  // Keys are uniform on [0, 2^64); keep those below a threshold expected to
  // admit n + 8 sqrt(n) + 64 nodes and widen it if fewer than n made it.
  double frac = ((double)n + 8.0 * std::sqrt((double)n) + 64.0) / (double)N;
  for (int attempt = 0; attempt < 64; ++attempt) {
    const uint64_t thresh =
        frac >= 1.0 ? ~0ull : (uint64_t)std::ldexp(frac, 64);
    CSC_HIP(launch_sample_count(N, seed, thresh, counts, s));
    CSC_HIP(launch_scan_counts(counts, nch, offsets, total, s));
    int h_total = 0;
    CSC_HIP(hipMemcpyAsync(&h_total, total, sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (h_total < n) {
      frac *= 2.0;
      continue;
    }
    if (sort_pairs_temp_bytes(h_total) > temp_bytes) {
      set_error("internal: sort scratch too small");
      return CSC_E_INVALID_ARG;
    }
    CSC_HIP(launch_sample_write(N, seed, thresh, offsets, kin, vin, s));
    CSC_HIP(sort_pairs(temp, temp_bytes, kin, kout, vin, vout, h_total, s));
    CSC_HIP(hipMemcpyAsync(idx, vout, (size_t)n * sizeof(int), hipMemcpyDeviceToDevice, s));
    CSC_HIP(hipStreamSynchronize(s));
    return CSC_OK;
  }
  set_error("sampling threshold did not admit n keys");
  return CSC_E_INVALID_ARG;
}

namespace csc {
size_t perm_bytes(int N, int64_t nnz, int n) {
  size_t b = align_up(((size_t)N + 1) * sizeof(int)) + align_up((size_t)nnz * sizeof(int));
  b += align_up((size_t)nnz * sizeof(float)) + 2 * align_up((size_t)N * sizeof(int));
  b += align_up((size_t)n * sizeof(int)) + align_up(perm_graph_temp_bytes(N));
  return b + align_up(4 * sizeof(int));
}

// The graph permuted to `order` (row r = node order[r], neighbours relabelled
// and kept in CSR order) and the sampled indices in the new numbering, in
// workspace carved from ar.
csc_status permuted_graph(const csc_graph& g, const int* order, const int* idx, int n, Arena& ar,
                          csc_graph& gp, const int*& idxp, hipStream_t s) {
  const int N = g.n;
  int* rp = ar.take<int>((size_t)N + 1);
  int* col = ar.take<int>((size_t)g.nnz);
  float* val = ar.take<float>((size_t)g.nnz);
  int* inv = ar.take<int>(N);
  int* deg = ar.take<int>(N);
  int* idx2 = ar.take<int>(n);
  const size_t temp_bytes = perm_graph_temp_bytes(N);
  void* temp = ar.take<char>(temp_bytes);
  int* bad = ar.take<int>(4);
  if (!ar.ok()) {
    set_error("internal: permutation workspace overflow");
    return CSC_E_INVALID_ARG;
  }
  CSC_HIP(launch_fill_i32(bad, 1, 0, s));
  CSC_HIP(launch_fill_i32(inv, N, -1, s));
  CSC_HIP(launch_perm_inverse(N, order, inv, bad, s));
  CSC_HIP(launch_perm_check(N, inv, bad, s));
  int hbad = 0;
  CSC_HIP(hipMemcpyAsync(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  CSC_REQUIRE(!hbad, "order is not a permutation of [0, N)");
  CSC_HIP(perm_graph(N, order, inv, g.row_ptr, g.col, g.val, rp, col, val, deg, temp, temp_bytes,
                     s));
  CSC_HIP(launch_map_indices(n, N, inv, idx, idx2, s));
  gp = g;
  gp.row_ptr = rp;
  gp.col = col;
  gp.val = val;
  gp.dinv_sqrt = nullptr;
  gp.sched = nullptr;  // the community order is the walk
  idxp = idx2;
  return CSC_OK;
}

namespace {

csc_status download(std::vector<double>& h, const double* d, size_t n, hipStream_t s) {
  h.resize(n);
  CSC_HIP(hipMemcpyAsync(h.data(), d, n * sizeof(double), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  return CSC_OK;
}

csc_status upload_d(double* d, const std::vector<double>& h, hipStream_t s) {
  CSC_HIP(hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
  return CSC_OK;
}

}  // namespace

// Block conjugate gradient on the k columns of R = B at once, in the
// breakdown-free form (Ji and Li, 2017): the search block P is the
// orthonormalised (rank-revealing) Z + P beta, so columns that converge or
// become dependent leave the search space instead of breaking it.  Z is the
// residual block R, or in the preconditioned form D^-1 R with the Jacobi
// diagonal D = diag(mask) + gamma I of the operator (its diagonal up to the
// small h~(L)_ii terms): that maps the sampled rows (~1 + gamma) and the
// unsampled rows (~gamma) to a common scale.  Every iteration costs one
// Chebyshev pass (Q = M P) plus a few Gram matrices and block products; the
// small k x k algebra runs on the host in float64.  block_pre forms P before
// the pass, block_post the rest after it.
csc_status block_init(BlockState& st, const Layout& L, int k, double tol, bool jacobi, float gamma,
                      const BlockBufs& b, const double* bnorm2_dev, hipStream_t s) {
  st.L = L;
  st.k = k;
  st.tol = tol;
  st.jacobi = jacobi;
  st.gamma = gamma;
  st.b = b;
  CSC_TRY(download(st.bn2, bnorm2_dev, (size_t)k, s));
  st.done.assign(k, 0);
  st.iters.assign(k, 0);
  st.relres.assign(k, 0.0);
  st.ndone = st.nlive = 0;
  for (int j = 0; j < k; ++j) {
    if (st.bn2[j] > 0.0)
      ++st.nlive;
    else
      st.done[j] = 1;
  }
  st.finished = st.converged = st.nlive == 0;
  st.broke = false;
  if (jacobi)
    CSC_HIP(launch_jacobi(L, b.R, b.mask, gamma, b.Z, s));
  else
    CSC_HIP(hipMemcpyAsync(b.Z, b.R, L.bytes(), hipMemcpyDeviceToDevice, s));
  return CSC_OK;
}

// Each iteration runs in stages: a launch stage only enqueues device work
// and copies into st's host vectors, a host stage runs the k x k algebra on
// what the previous launch stage brought back (the caller synchronises the
// stream in between).  block_pre and block_post chain the stages of one
// graph; the batched form runs each stage for all graphs, one
// synchronisation per stage and the host stages in parallel.
// Bit t set when 128-column tile t of the k columns holds a column still in
// the search: the Gram entries and block-product columns of the other tiles
// are never read (done columns are zeroed out of G and have zero step
// coefficients), so their kernels skip them.
uint64_t live_tiles(const BlockState& st) {
  uint64_t m = 0;
  for (int j = 0; j < st.k; ++j)
    if (!st.done[j]) m |= 1ull << std::min(j / kBlockTile, 63);
  return m;
}

// Tiles covering columns [0, w).
uint64_t prefix_tiles(int w) {
  const int t = (w + kBlockTile - 1) / kBlockTile;
  return t >= 64 ? ~0ull : (1ull << t) - 1;
}

csc_status pre_launch(BlockState& st, hipStream_t s) {
  const BlockBufs& b = st.b;
  const int k = st.k;
  // symmetric: the tiles on and below the diagonal, the rest mirrored
  const uint64_t live = live_tiles(st);
  CSC_HIP(launch_gram(st.L, b.Z, b.Z, k, k, b.gpart, b.G, k, s, /*lower=*/true, live, live));
  st.G.resize((size_t)k * k);
  CSC_HIP(hipMemcpyAsync(st.G.data(), b.G, st.G.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  return CSC_OK;
}

void pre_host(BlockState& st) {
  // columns that met the tolerance leave the search space; their X and R
  // stay as they were when they converged (post_host_a)
  const int k = st.k;
  for (int j = 0; j < k; ++j)
    if (st.done[j])
      for (int i = 0; i < k; ++i) st.G[(size_t)j * k + i] = st.G[(size_t)i * k + j] = 0.0;
  st.sr = dense::orth_transform(st.G, st.k, 1e-10, st.T);
  if (st.sr == 0) {  // Z = 0: every residual column vanished
    st.finished = true;
    st.converged = true;
  }
}

csc_status pre_finish(BlockState& st, hipStream_t s) {
  const BlockBufs& b = st.b;
  const int k = st.k;
  CSC_TRY(upload_d(b.S_t, st.T, s));
  // P's columns past sr are read by nothing (passes, Grams and products all
  // stop at sr; a full-width pass leaves them in columns nobody reads)
  CSC_HIP(launch_block_mul(st.L, 0.f, nullptr, b.Z, b.S_t, k, st.sr, k, b.P, s,
                           /*f32=*/st.jacobi, prefix_tiles(st.sr)));
  return CSC_OK;
}

// W = P^T Q (s x s) and P^T R (s x k, parked in S_b, which is free until beta)
csc_status post_launch_a(BlockState& st, hipStream_t s) {
  const BlockBufs& b = st.b;
  const int k = st.k, sr = st.sr;
  // the Cholesky factorisation reads W's lower triangle only
  CSC_HIP(launch_gram(st.L, b.P, b.Q, sr, sr, b.gpart, b.G, sr, s, /*lower=*/true));
  CSC_HIP(launch_gram(st.L, b.P, b.R, sr, k, b.gpart, b.S_b, k, s, false, ~0ull, live_tiles(st)));
  st.W.resize((size_t)sr * sr);
  st.C.resize((size_t)sr * k);
  CSC_HIP(hipMemcpyAsync(st.W.data(), b.G, st.W.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipMemcpyAsync(st.C.data(), b.S_b, st.C.size() * sizeof(double), hipMemcpyDeviceToHost,
                         s));
  return CSC_OK;
}

// alpha = W^{-1} P^T R (and -alpha); a W that is not positive definite ends the solve
void post_host_a(BlockState& st) {
  const int k = st.k, sr = st.sr;
  if (!dense::cholesky(st.W, sr, sr)) {
    st.finished = true;
    st.broke = true;
    return;
  }
  dense::chol_solve(st.W, sr, sr, st.C, k, 1.0, st.host_threads);
  for (int j = 0; j < k; ++j)
    if (st.done[j])
      for (int r = 0; r < sr; ++r) st.C[(size_t)r * k + j] = 0.0;
  st.N = st.C;
  for (auto& v : st.N) v = -v;
}

// X += P alpha feeds nothing back into the iteration: it runs on the side
// stream once the main stream has brought back what the host needs (launched
// last in post_launch_b), so that it fills the GPU while the host works out
// beta; the main stream waits for it before P or S_a change again
// (post_finish) or X is read (block_join).  Without a side stream it runs in
// line.
csc_status launch_x_update(BlockState& st, hipStream_t s) {
  const BlockBufs& b = st.b;
  BlockState::SideX& x = st.sx;
  hipStream_t s2 = side_stream();
  if (s2 && !x.go) {
    if (hipEventCreateWithFlags(&x.go, hipEventDisableTiming) != hipSuccess) {
      x.go = nullptr;
    } else if (hipEventCreateWithFlags(&x.done, hipEventDisableTiming) != hipSuccess) {
      (void)hipEventDestroy(x.go);
      x.go = x.done = nullptr;
    }
  }
  if (!s2 || !x.go) {
    CSC_HIP(launch_block_mul(st.L, 1.f, b.X, b.P, b.S_a, st.sr, st.k, st.k, b.X, s, /*f32=*/true,
                             live_tiles(st)));
    return CSC_OK;
  }
  CSC_HIP(hipEventRecord(x.go, s));
  CSC_HIP(hipStreamWaitEvent(s2, x.go, 0));
  x.main = s;
  x.pending = true;
  CSC_HIP(launch_block_mul(st.L, 1.f, b.X, b.P, b.S_a, st.sr, st.k, st.k, b.X, s2, /*f32=*/true,
                           live_tiles(st)));
  CSC_HIP(hipEventRecord(x.done, s2));
  return CSC_OK;
}

csc_status block_join(BlockState& st) {
  if (!st.sx.pending) return CSC_OK;
  st.sx.pending = false;
  CSC_HIP(hipStreamWaitEvent(st.sx.main, st.sx.done, 0));
  return CSC_OK;
}

BlockState::SideX::~SideX() {
  if (pending && main && done) (void)hipStreamWaitEvent(main, done, 0);
  if (go) (void)hipEventDestroy(go);
  if (done) (void)hipEventDestroy(done);
}

// X += P alpha, R -= Q alpha; the column norms of R, and the next search
// block's Gram Q^T Z formed before the convergence check so that both come
// back in one round trip (after the last iteration it goes unused).
// Precision of the right products: the residual recurrence R -= Q alpha
// decides convergence and sums in float64 (CSC_TUNE_BLOCK_PRODUCT = 1:
// float32, which was measured to cost the 1e5-node SBM a fourth iteration);
// X += P alpha (X feeds nothing back) takes the precision form's float32
// sums on the float32 matrix cores; so do P = Z T and Z += P beta (the search
// directions) in the Jacobi-preconditioned form, whose 3-4 iterations were
// measured unchanged by it (iteration counts, residuals, labels).  The plain
// block CG keeps float64 sums for the directions: over its 13 or more
// iterations float32 directions moved the iterate by ~1e-3.
csc_status post_launch_b(BlockState& st, hipStream_t s) {
  const BlockBufs& b = st.b;
  const Layout& L = st.L;
  const int k = st.k, sr = st.sr;
  CSC_TRY(upload_d(b.S_a, st.C, s));
  CSC_TRY(upload_d(b.S_na, st.N, s));
  const uint64_t live = live_tiles(st);
  CSC_HIP(launch_block_mul(L, 1.f, b.R, b.Q, b.S_na, sr, k, k, b.R, s, false, live));
  CSC_HIP(launch_col_dot(L, b.R, b.R, b.part, s));
  CSC_HIP(launch_reduce(b.part, col_dot_chunks(L), k, b.rn2, s));
  if (st.jacobi) CSC_HIP(launch_jacobi(L, b.R, b.mask, st.gamma, b.Z, s));
  CSC_HIP(launch_gram(L, b.Q, st.jacobi ? b.Z : b.R, sr, k, b.gpart, b.G, k, s, false, ~0ull,
                      live));
  st.rn2.resize(k);
  st.C.resize((size_t)sr * k);
  CSC_HIP(hipMemcpyAsync(st.rn2.data(), b.rn2, (size_t)k * sizeof(double), hipMemcpyDeviceToHost,
                         s));
  CSC_HIP(hipMemcpyAsync(st.C.data(), b.G, st.C.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  CSC_TRY(launch_x_update(st, s));  // after the copies: it runs while the host works
  return CSC_OK;
}

// every column: ||r_j|| <= tol ||b_j||; then beta = -W^{-1} Q^T Z unless done
void post_host_b(BlockState& st, int it, int max_iter) {
  const int k = st.k;
  for (int j = 0; j < k; ++j) {
    if (st.bn2[j] <= 0.0) continue;
    st.relres[j] = std::sqrt(st.rn2[j] / st.bn2[j]);
    if (!st.done[j] && st.relres[j] <= st.tol) {
      st.done[j] = 1;
      st.iters[j] = it;
      ++st.ndone;
    }
  }
  if (st.ndone == st.nlive) {
    st.finished = st.converged = true;
    return;
  }
  if (it == max_iter) {
    st.finished = true;
    return;
  }
  dense::chol_solve(st.W, st.sr, st.sr, st.C, k, -1.0, st.host_threads);
}

// Z = Z + P beta  (Z = R, or D^-1 R)
csc_status post_finish(BlockState& st, hipStream_t s) {
  const BlockBufs& b = st.b;
  const int k = st.k, sr = st.sr;
  CSC_TRY(block_join(st));
  CSC_TRY(upload_d(b.S_b, st.C, s));
  CSC_HIP(launch_block_mul(st.L, 1.f, st.jacobi ? b.Z : b.R, b.P, b.S_b, sr, k, k, b.Z, s,
                           /*f32=*/st.jacobi, live_tiles(st)));
  return CSC_OK;
}

// Q = M P for the block CG.  P's live columns are its first sr; when they are
// fewer than the block's width the pass runs on a compact copy of them (a
// layout of width sr with its own panel width, or an n-vector for a single
// column in Clenshaw's form) and only those columns of Q are written back
// (the block CG reads no column of Q beyond sr).  Every
// element sums its row's neighbours in CSR order whatever the layout, so Q
// is the same either way; a block whose columns have partly converged costs
// a pass of its live width.
// Buffers: in Clenshaw's form the compact P sits in Q's buffer (Q is written
// only by the copy back), the recurrence in Ta / Tb, and the last step, which
// reads b_2 and writes its output element by element in the same lane, writes
// the compact Q over b_2; the forward form keeps two compact blocks in each of
// Ta and Tb, so it compacts only blocks at most half as wide.
static csc_status block_pass(const csc_graph& g, const Layout& L, const double* a, int p,
                             const Pass& pb, int sr, hipStream_t s) {
  if (sr < 1 || sr >= L.w) return chebyshev_pass(g, L, a, p, EPI_CG, pb, s);
  const int form = filter_form();
  // a single live column in Clenshaw's form runs as an n-vector (the steps'
  // single-column path); otherwise a panel layout of the live width
  const Layout Lc = sr == 1 && form == FORM_CLENSHAW
                        ? make_layout(L.n, 1, 1)
                        : make_layout(L.n, sr, choose_panel_width(L.n, sr, g.nnz));
  // the compact blocks live in the wide blocks' buffers, and a compact pass
  // given a partial buffer writes its column partials into the wide pass's
  if (Lc.elems() > L.elems() ||
      (pb.part && (size_t)Lc.np * Lc.pw * tiles_for(Lc) > (size_t)L.np * L.pw * tiles_for(L)))
    return chebyshev_pass(g, L, a, p, EPI_CG, pb, s);
  Pass pc = pb;
  float* Pc;
  float* Qc;
  const std::vector<PassStep> plan = pass_plan(EPI_CG, a, p, pb.T0, pb.Ta, pb.Tb, form);
  if (form == FORM_CLENSHAW && !plan.empty() && plan.back().epi == EPI_CLEN_CG &&
      (plan.back().Tprev == pb.Tb || plan.back().Tprev == nullptr) && plan.back().Tm != pb.Tb) {
    Pc = pb.Y;
    Qc = pb.Tb;  // b_2's buffer at the last step
  } else {
    const size_t half = (Lc.elems() + 63) / 64 * 64;
    if (2 * half > L.elems()) return chebyshev_pass(g, L, a, p, EPI_CG, pb, s);
    Pc = pb.Ta;
    Qc = pb.Ta + half;
    pc.Ta = pb.Tb;
    pc.Tb = pb.Tb + half;
  }
  pc.T0 = Pc;
  pc.Y = Qc;
  pc.form = form;  // the buffer plan above holds for this form only
  CSC_HIP(launch_to_compact(Lc, Pc, L, pb.T0, sr, s));
  CSC_TRY(chebyshev_pass(g, Lc, a, p, EPI_CG, pc, s));
  CSC_HIP(launch_from_compact(Lc, Qc, L, pb.Y, sr, s));
  return CSC_OK;
}

csc_status block_pre(BlockState& st, hipStream_t s) {
  CSC_TRY(pre_launch(st, s));
  CSC_HIP(hipStreamSynchronize(s));
  pre_host(st);
  if (st.finished) return CSC_OK;
  return pre_finish(st, s);
}

csc_status block_post(BlockState& st, int it, int max_iter, hipStream_t s) {
  CSC_TRY(post_launch_a(st, s));
  CSC_HIP(hipStreamSynchronize(s));
  post_host_a(st);
  if (st.finished) return CSC_OK;
  CSC_TRY(post_launch_b(st, s));
  CSC_HIP(hipStreamSynchronize(s));
  post_host_b(st, it, max_iter);
  if (st.finished) return CSC_OK;
  return post_finish(st, s);
}

void block_finish(BlockState& st, int max_iter) {
  for (int j = 0; j < st.k; ++j)
    if (!st.done[j]) st.iters[j] = max_iter;
}

}  // namespace csc

extern "C" size_t csc_interpolate_workspace_bytes(int32_t N, int64_t nnz, int32_t k, int32_t n) {
  if (N < 1 || nnz < 0 || k < 1 || n < 1) return 0;
  return max_over_widths(N, k, [](const Layout& L) { return interp_bytes(L); }) +
         perm_bytes(N, nnz, n);
}

extern "C" csc_status csc_interpolate(const csc_graph* g_in, const int32_t* order,
                                      int32_t method, double lambda_k, int32_t p, double gamma,
                                      const int32_t* idx_in, const int32_t* labels_r,
                                      const float* weights, int32_t n,
                                      int32_t k, double tol, int32_t max_iter, float* X,
                                      int32_t ldx, int32_t* labels, int32_t* iters_out,
                                      double* relres_out, void* ws, size_t ws_bytes,
                                      void* stream) {
  clear_error();
  CSC_TRY(check_graph(g_in));
  const int N = g_in->n;
  const csc_graph* g = g_in;
  const int32_t* idx = idx_in;
  CSC_REQUIRE(idx_in && labels_r && labels, "idx, labels_r and labels must be non-NULL");
  CSC_REQUIRE(k >= 1 && k <= N && n >= 1 && n <= N, "need 1 <= k <= N and 1 <= n <= N");
  CSC_REQUIRE(p >= 1 && gamma > 0.0 && tol > 0.0 && max_iter >= 1,
              "need p >= 1, gamma > 0, tol > 0, max_iter >= 1");
  CSC_REQUIRE(lambda_k >= 0.0 && lambda_k <= 2.0, "lambda_k must lie in [0, 2]");
  CSC_REQUIRE(X == nullptr || ldx >= k, "ldx must be >= k");
  CSC_REQUIRE(method == CSC_CG_COLUMNS || method == CSC_CG_BLOCK || method == CSC_CG_BLOCK_JACOBI,
              "method must be CSC_CG_COLUMNS, CSC_CG_BLOCK or CSC_CG_BLOCK_JACOBI");
  const Layout L = make_layout(N, k, choose_panel_width(N, k, g->nnz));
  CSC_TRY(check_ws(ws, ws_bytes, interp_bytes(L) + (order ? perm_bytes(N, g->nnz, n) : 0)));
  hipStream_t s = as_stream(stream);
  const int tiles = tiles_for(L);
  const size_t wp = (size_t)L.np * L.pw;
  Arena ar(ws, ws_bytes);
  csc_graph gperm;
  if (order) {
    Arena tail(static_cast<char*>(ws) + interp_bytes(L), ws_bytes - interp_bytes(L));
    CSC_TRY(permuted_graph(*g_in, order, idx_in, n, tail, gperm, idx, s));
    g = &gperm;
  }
  float* P = ar.take<float>(L.elems());
  float* Ta = ar.take<float>(L.elems());
  float* Tb = ar.take<float>(L.elems());
  float* AP = ar.take<float>(L.elems());
  float* Xi = ar.take<float>(L.elems());
  float* Rr = ar.take<float>(L.elems());
  float* mask = ar.take<float>(N);
  double* part = ar.take<double>(wp * tiles);
  double* rr = ar.take<double>(wp);
  double* rrn = ar.take<double>(wp);
  double* pAp = ar.take<double>(wp);
  double* alpha = ar.take<double>(wp);
  double* beta = ar.take<double>(wp);
  double* bnorm2 = ar.take<double>(wp);
  double* colnorm2 = ar.take<double>(wp);
  int* active = ar.take<int>(wp);
  int* iters = ar.take<int>(wp);
  double* relres = ar.take<double>(wp);
  int* flags = ar.take<int>(4);  // nactive, breakdown
  float* Zb = ar.take<float>(L.elems());
  double* gpart = ar.take<double>(gram_part_elems(L, L.w));
  double* Gd = ar.take<double>((size_t)k * k);
  double* S_t = ar.take<double>((size_t)k * k);
  double* S_a = ar.take<double>((size_t)k * k);
  double* S_na = ar.take<double>((size_t)k * k);
  double* S_b = ar.take<double>((size_t)k * k);

  CSC_HIP(launch_fill_f32(P, L.elems(), 0.f, s));
  CSC_HIP(launch_fill_f32(Xi, L.elems(), 0.f, s));
  CSC_HIP(launch_fill_f32(Rr, L.elems(), 0.f, s));
  CSC_HIP(launch_fill_f32(mask, N, 0.f, s));
  CSC_HIP(launch_fill_i32(iters, wp, 0, s));
  CSC_HIP(launch_fill_f64(relres, wp, 0.0, s));
  CSC_HIP(launch_fill_i32(flags, 4, 0, s));
  CSC_HIP(launch_cg_scatter(L, n, idx, labels_r, weights, Rr, P, mask, flags + 2, s));
  CSC_HIP(launch_col_dot(L, Rr, Rr, part, s));
  CSC_HIP(launch_reduce(part, col_dot_chunks(L), k, bnorm2, s));
  // rr = bnorm2; active = bnorm2 > 0 (beta doubles as the activity probe)
  CSC_HIP(hipMemcpyAsync(rr, bnorm2, k * sizeof(double), hipMemcpyDeviceToDevice, s));
  {
    std::vector<double> hb(k);
    CSC_HIP(hipMemcpyAsync(hb.data(), bnorm2, k * sizeof(double), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    int hbad = 0;
    CSC_HIP(hipMemcpyAsync(&hbad, flags + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (hbad) {
      set_error("idx or labels_r holds a value out of range");
      return CSC_E_INVALID_ARG;
    }
    std::vector<int> ha(k);
    for (int j = 0; j < k; ++j) ha[j] = hb[j] > 0.0 ? 1 : 0;
    CSC_HIP(hipMemcpyAsync(active, ha.data(), k * sizeof(int), hipMemcpyHostToDevice, s));
    CSC_HIP(hipStreamSynchronize(s));
  }

  std::vector<double> a(p + 1);
  jackson_lowpass(lambda_k, p, a.data());
  if (method != CSC_CG_COLUMNS) {
    BlockState bs;
    CSC_TRY(block_init(bs, L, k, tol, method == CSC_CG_BLOCK_JACOBI, (float)gamma,
                       BlockBufs{P, AP, Ta, Tb, Xi, Rr, Zb, mask, part, gpart, Gd, S_t, S_a, S_na,
                                 S_b, rrn},
                       bnorm2, s));
    bs.host_threads = (int)std::min(8u, std::max(1u, std::thread::hardware_concurrency()));
    Pass pb;
    pb.T0 = P;
    pb.Ta = Ta;
    pb.Tb = Tb;
    pb.Y = AP;
    pb.part = nullptr;  // the block CG takes P^T Q from a Gram, not the pass's column partials
    pb.mask = mask;
    pb.gamma = (float)gamma;
    for (int it = 1; it <= max_iter && !bs.finished; ++it) {
      CSC_TRY(block_pre(bs, s));
      if (bs.finished) break;
      CSC_TRY(block_pass(*g, L, a.data(), p, pb, bs.sr, s));  // Q = M P
      CSC_TRY(block_post(bs, it, max_iter, s));
    }
    CSC_TRY(block_join(bs));
    block_finish(bs, max_iter);
    CSC_HIP(launch_col_dot(L, Xi, Xi, part, s));
    CSC_HIP(launch_reduce(part, col_dot_chunks(L), k, colnorm2, s));
    CSC_HIP(launch_labels(L, Xi, colnorm2, labels, X, ldx, order, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (iters_out) std::memcpy(iters_out, bs.iters.data(), k * sizeof(int));
    if (relres_out) std::memcpy(relres_out, bs.relres.data(), k * sizeof(double));
    if (bs.broke) {
      set_error("block CG breakdown: P^T M P is not positive definite");
      return CSC_W_NOT_CONVERGED;
    }
    return bs.converged ? CSC_OK : CSC_W_NOT_CONVERGED;
  }
  Pass b;
  b.T0 = P;
  b.Ta = Ta;
  b.Tb = Tb;
  b.Y = AP;
  b.part = part;
  b.mask = mask;
  b.gamma = (float)gamma;
  int it = 0, nactive = 1;
  for (it = 1; it <= max_iter; ++it) {
    CSC_TRY(chebyshev_pass(*g, L, a.data(), p, EPI_CG, b, s));
    CSC_HIP(launch_reduce(part, tiles, k, pAp, s));
    CSC_HIP(launch_cg_alpha(k, rr, pAp, active, alpha, flags + 1, s));
    CSC_HIP(launch_cg_update1(L, AP, P, Xi, Rr, alpha, part, s));
    CSC_HIP(launch_reduce(part, tiles, k, rrn, s));
    CSC_HIP(launch_cg_scalar(k, rrn, rr, bnorm2, beta, active, iters, relres, it, tol, flags, s));
    CSC_HIP(launch_cg_update2(L, Rr, P, beta, active, s));
    CSC_HIP(hipMemcpyAsync(&nactive, flags, sizeof(int), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    if (nactive == 0) break;
  }
  CSC_HIP(launch_col_dot(L, Xi, Xi, part, s));
  CSC_HIP(launch_reduce(part, col_dot_chunks(L), k, colnorm2, s));
  CSC_HIP(launch_labels(L, Xi, colnorm2, labels, X, ldx, order, s));
  std::vector<int> hit(k);
  std::vector<double> hrel(k);
  int breakdown = 0;
  CSC_HIP(hipMemcpyAsync(hit.data(), iters, k * sizeof(int), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipMemcpyAsync(hrel.data(), relres, k * sizeof(double), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipMemcpyAsync(&breakdown, flags + 1, sizeof(int), hipMemcpyDeviceToHost, s));
  CSC_HIP(hipStreamSynchronize(s));
  if (iters_out) std::memcpy(iters_out, hit.data(), k * sizeof(int));
  if (relres_out) std::memcpy(relres_out, hrel.data(), k * sizeof(double));
  if (breakdown) {
    set_error("CG breakdown: p^T A p <= 0 in some column");
    return CSC_W_NOT_CONVERGED;
  }
  return nactive > 0 ? CSC_W_NOT_CONVERGED : CSC_OK;
}

namespace {
size_t steps_bytes(const Layout& L) {
  const size_t tiles = tiles_for(L), wp = (size_t)L.np * L.pw;
  size_t b = 4 * align_up(L.bytes());                       // T0, Ta, Tb, Y
  b += align_up((size_t)L.n * sizeof(float));               // mask
  // column partials (kinds 0, 2), or the moment partials of up to
  // kMaxCountGroup tests (kinds 1, 4)
  b += align_up(std::max(wp * tiles, (size_t)L.np * tiles * kMomSlots * kMaxCountGroup) *
                sizeof(double));
  return b + 256;
}
}  // namespace

extern "C" size_t csc_cheb_steps_workspace_bytes(int32_t n, int32_t w) {
  if (n < 1 || w < 1) return 0;
  return max_over_widths(n, w, [](const Layout& L) { return steps_bytes(L); });
}

extern "C" csc_status csc_cheb_steps(const csc_graph* g, int32_t w, int32_t kind, int32_t prepare,
                                     int32_t steps, void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(w >= 1 && steps >= 0, "need w >= 1 and steps >= 0");
  CSC_REQUIRE(kind >= 0 && kind <= 5, "kind must be 0, 1, 2, 3, 4 or 5");
  const int group = kind == 4 ? count_group() : 1;
  CSC_REQUIRE(w % (4 * group) == 0 || kind != 4,
              "kind 4 needs w = group size x a multiple of 4");
  const Layout L = make_layout(g->n, w, choose_panel_width(g->n, w, g->nnz));
  CSC_TRY(check_ws(ws, ws_bytes, steps_bytes(L)));
  hipStream_t s = as_stream(stream);
  const int tiles = tiles_for(L);
  Arena ar(ws, ws_bytes);
  float* T0 = ar.take<float>(L.elems());
  float* Ta = ar.take<float>(L.elems());
  float* Tb = ar.take<float>(L.elems());
  float* Y = ar.take<float>(L.elems());
  float* mask = ar.take<float>(g->n);
  double* part = ar.take<double>(
      std::max((size_t)L.np * L.pw * tiles, (size_t)L.np * tiles * kMomSlots * kMaxCountGroup));
  if (prepare) {
    CSC_HIP(launch_gaussian_panels(L, 1, 0, CSC_STREAM_FEAT, T0, s));
    CSC_HIP(launch_fill_f32(Ta, L.elems(), 0.f, s));
    CSC_HIP(launch_fill_f32(Tb, L.elems(), 0.f, s));
    CSC_HIP(launch_fill_f32(Y, L.elems(), 0.f, s));
    CSC_HIP(launch_fill_f32(mask, g->n, 0.f, s));
  }
  StepArgs sa;
  sa.L = L;
  sa.tiles = tiles;
  sa.row_ptr = g->row_ptr;
  sa.col = g->col;
  sa.val = g->val;
  sa.sched = step_sched(*g, L);
  sa.T0 = T0;
  sa.Y = Y;
  sa.mask = mask;
  sa.gamma = 1e-3f;
  sa.c0 = 0.5f;
  sa.c1 = 0.25f;
  sa.part = part;
  sa.part2 = part;
  sa.part0 = part;
  // kinds 1 and 4: pass j's moment partials at part + j * units * kMomSlots
  // (group <= kMaxCountGroup, within the partial buffer of steps_bytes)
  sa.mgroup = group;
  sa.mnc4 = w / group;
  sa.mstride = (size_t)L.np * tiles * kMomSlots;
  apply_tuning(sa);
  const int epi = kind == 0   ? EPI_Y
                  : kind == 1 ? EPI_MOM
                  : kind == 4 ? (group > 1 ? EPI_MOMG : EPI_MOM)
                  : kind == 5 ? EPI_SPMM
                  : (kind == 2 ? EPI_CG : EPI_CLEN);
  for (int m = 1; m <= steps; ++m) {
    // T_{m+1} from T_m (gathered) and T_{m-1}; buffers alternate as in a pass
    sa.Tm = (m & 1) ? Ta : Tb;
    sa.Tprev = (m & 1) ? Tb : Ta;
    sa.Tnext = (m & 1) ? Tb : Ta;
    if (m == 1) sa.Tm = T0;
    CSC_HIP(launch_cheb_step(sa, epi, false, epi == EPI_CG, s));
  }
  return CSC_OK;
}

extern "C" csc_status csc_autotune(const csc_graph* g, int32_t w, int32_t kind, int32_t reps,
                                   int32_t* pw_out, int32_t* xcd_out, double* us_out, void* ws,
                                   size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(w >= 1 && kind >= 0 && kind <= 4 && reps >= 1, "need w >= 1, kind 0..4, reps >= 1");
  CSC_REQUIRE(kind != 4 || w % (4 * count_group()) == 0,
              "kind 4 needs w = group size x a multiple of 4");
  CSC_REQUIRE(g_panel_override.load() == 0, "a forced panel width is in effect");
  CSC_TRY(check_ws(ws, ws_bytes, csc_cheb_steps_workspace_bytes(g->n, w)));
  hipStream_t s = as_stream(stream);
  // candidates: the six cheapest widths of the cost model and every 128-byte multiple
  std::vector<std::pair<double, int>> ranked;
  for (int pw = 4; pw <= 256; pw += 4) ranked.push_back({panel_cost(g->n, w, g->nnz, pw), pw});
  std::sort(ranked.begin(), ranked.end());
  std::vector<int> cand;
  for (size_t i = 0; i < ranked.size() && cand.size() < 6; ++i) cand.push_back(ranked[i].second);
  for (int pw = 32; pw <= 256; pw += 32)
    if (std::find(cand.begin(), cand.end(), pw) == cand.end() && (w + pw - 1) / pw * pw < 2 * w + 32)
      cand.push_back(pw);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  CSC_HIP(hipEventCreate(&e0));
  CSC_HIP(hipEventCreate(&e1));
  const int xcd_saved = g_tune_xcd.load();
  double best = -1.0;
  int best_pw = cand[0], best_xcd = xcd_saved;
  csc_status st = CSC_OK;
  for (int pw : cand) {
    for (int xcd = 0; xcd <= 1 && st == CSC_OK; ++xcd) {
      g_panel_override.store(pw);
      g_tune_xcd.store(xcd);
      st = csc_cheb_steps(g, w, kind, 1, 2, ws, ws_bytes, stream);  // prepare + warm
      if (st != CSC_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e0, s) != hipSuccess ||
          (st = csc_cheb_steps(g, w, kind, 0, reps, ws, ws_bytes, stream)) != CSC_OK ||
          hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        if (st == CSC_OK) {
          set_error("event timing failed during autotuning");
          st = CSC_E_HIP;
        }
        break;
      }
      const double us = 1000.0 * ms / reps;
      if (best < 0.0 || us < best) {
        best = us;
        best_pw = pw;
        best_xcd = xcd;
      }
    }
    if (st != CSC_OK) break;
  }
  g_panel_override.store(0);
  g_tune_xcd.store(xcd_saved);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != CSC_OK) return st;
  {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tuned[shape_key(g->n, w, g->nnz)] = best_pw;
  }
  if (pw_out) *pw_out = best_pw;
  if (xcd_out) *xcd_out = best_xcd;
  if (us_out) *us_out = best;
  return CSC_OK;
}

extern "C" void csc_autotune_clear(void) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tuned.clear();
}
