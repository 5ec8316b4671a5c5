// The lambda_k bracket network: a 52 -> 128 -> 128 -> 2 GELU perceptron,
// trained and evaluated on the GPU by the kernels below (float32 FMA, every
// sum in a fixed order, no atomics), and the dichotomy that starts from its
// bracket.
//
// Parameters are one flat float array: W1 (52 x 128, row = input), b1 (128),
// W2 (128 x 128), b2 (128), W3 (128 x 2), b3 (2).  Inputs are the
// Jackson-damped Chebyshev moments g_m mu_m / mu_0 (m = 1..50) of the first
// eigencount pass, ln N / 10 and k / N.  The outputs are offsets, in units of
// s = sqrt(2k/n_c) / c'(lambda_0), around the root lambda_0 of that pass's
// own count curve c(lambda) = sum_m a_m(lambda) mu_m.  Training minimises the
// pinball loss of output 0 at tau = 0.02 and output 1 at tau = 0.98 against
// (lambda_k - lambda_0) / s, lambda_k from the plain dichotomy, with Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"

namespace csc {
namespace {

constexpr int kIn = 52, kH = 128, kOut = 2;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kH, kOffW2 = kOffB1 + kH,
              kOffB2 = kOffW2 + kH * kH, kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kOut,
              kParams = kOffB3 + kOut;
constexpr float kTau[2] = {0.02f, 0.98f};

__device__ inline float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }

__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// Z = X W + b (row b of the batch per workgroup, one output per thread);
// A = GELU(Z) when act != 0, else A = Z.
__global__ __launch_bounds__(128) void k_linear(const float* X, int din, const float* W,
                                                const float* bias, int dout, float* Z, float* A,
                                                int act) {
  __shared__ float xs[128];
  const int b = blockIdx.x;
  for (int i = threadIdx.x; i < din; i += blockDim.x) xs[i] = X[(size_t)b * din + i];
  __syncthreads();
  const int o = threadIdx.x;
  if (o >= dout) return;
  float z = bias[o];
  for (int i = 0; i < din; ++i) z = fmaf(xs[i], W[i * dout + o], z);
  Z[(size_t)b * dout + o] = z;
  A[(size_t)b * dout + o] = act ? gelu(z) : z;
}

// dY = d(mean pinball)/dY; per-sample loss into lossb.
__global__ void k_pinball(const float* Y, const float* t, int B, float* dY, double* lossb) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  double l = 0.0;
  for (int j = 0; j < kOut; ++j) {
    const float u = t[b] - Y[b * kOut + j];
    const float ind = u < 0.f ? 1.f : 0.f;
    l += (double)u * (double)(kTau[j] - ind);
    dY[b * kOut + j] = -(kTau[j] - ind) / (float)B;
  }
  lossb[b] = l;
}

// dA_prev = dZ W^T, then dZ_prev = dA_prev * GELU'(Z_prev): row b per workgroup.
__global__ __launch_bounds__(128) void k_backprop(const float* dZ, int dout, const float* W,
                                                  int din, const float* Zprev, float* dZprev) {
  __shared__ float ds[128];
  const int b = blockIdx.x;
  for (int o = threadIdx.x; o < dout; o += blockDim.x) ds[o] = dZ[(size_t)b * dout + o];
  __syncthreads();
  const int i = threadIdx.x;
  if (i >= din) return;
  float a = 0.f;
  for (int o = 0; o < dout; ++o) a = fmaf(ds[o], W[i * dout + o], a);
  dZprev[(size_t)b * din + i] = a * gelu_grad(Zprev[(size_t)b * din + i]);
}

// gW[i][o] = sum_b X[b][i] dZ[b][o]; gb[o] = sum_b dZ[b][o] (row i = din of the
// grid); sums run over the batch in increasing order.
__global__ void k_weight_grad(const float* X, int din, const float* dZ, int dout, int B, float* gW,
                              float* gb) {
  const int o = threadIdx.x + blockIdx.y * blockDim.x;
  const int i = blockIdx.x;  // 0..din (din = bias row)
  if (o >= dout) return;
  float acc = 0.f;
  if (i < din) {
    for (int b = 0; b < B; ++b) acc = fmaf(X[(size_t)b * din + i], dZ[(size_t)b * dout + o], acc);
    gW[i * dout + o] = acc;
  } else {
    for (int b = 0; b < B; ++b) acc += dZ[(size_t)b * dout + o];
    gb[o] = acc;
  }
}

__global__ void k_adam(float* th, const float* g, float* m, float* v, int n, float lr, float b1,
                       float b2, float eps, float bc1, float bc2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

__global__ void k_sum_f64(const double* x, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += x[i];
  *out = s;
}

struct MlpBuffers {
  float *Z1, *A1, *Z2, *A2, *Y, *dY, *dZ2, *dZ1;
  double *lossb, *loss;
};

size_t mlp_ws(int B) {
  size_t b = 2 * align_up((size_t)B * kH * 4) * 2 + align_up((size_t)B * kOut * 4) * 2 +
             2 * align_up((size_t)B * kH * 4) + align_up((size_t)B * 8) + align_up(8);
  return b + 1024;
}

MlpBuffers carve_mlp(Arena& ar, int B) {
  MlpBuffers m;
  m.Z1 = ar.take<float>((size_t)B * kH);
  m.A1 = ar.take<float>((size_t)B * kH);
  m.Z2 = ar.take<float>((size_t)B * kH);
  m.A2 = ar.take<float>((size_t)B * kH);
  m.Y = ar.take<float>((size_t)B * kOut);
  m.dY = ar.take<float>((size_t)B * kOut);
  m.dZ2 = ar.take<float>((size_t)B * kH);
  m.dZ1 = ar.take<float>((size_t)B * kH);
  m.lossb = ar.take<double>(B);
  m.loss = ar.take<double>(1);
  return m;
}

csc_status forward(const float* th, const float* X, int B, const MlpBuffers& m, hipStream_t s) {
  hipLaunchKernelGGL(k_linear, dim3(B), dim3(128), 0, s, X, kIn, th + kOffW1, th + kOffB1, kH,
                     m.Z1, m.A1, 1);
  hipLaunchKernelGGL(k_linear, dim3(B), dim3(128), 0, s, m.A1, kH, th + kOffW2, th + kOffB2, kH,
                     m.Z2, m.A2, 1);
  hipLaunchKernelGGL(k_linear, dim3(B), dim3(128), 0, s, m.A2, kH, th + kOffW3, th + kOffB3, kOut,
                     m.Y, m.Y, 0);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// Jackson-Chebyshev damping factors (same formula as the filter coefficients).
void jackson_factors(int p, double* g) {
  const double pi = 3.14159265358979323846, al = pi / (p + 2);
  for (int m = 0; m <= p; ++m)
    g[m] = ((p + 2 - m) * std::cos(m * al) + std::sin(m * al) / std::tan(al)) / (p + 2);
}

void features(const double* mu, int N, int k, float* x) {
  double g[51];
  jackson_factors(50, g);
  for (int m = 1; m <= 50; ++m) x[m - 1] = (float)(g[m] * mu[m] / mu[0]);
  x[50] = (float)(std::log((double)N) / 10.0);
  x[51] = (float)((double)k / (double)N);
}

}  // namespace

void learned_features(const double* mu, int N, int k, float* x) { features(mu, N, k, x); }

void count_root(const double* mom, int p, int k, int n_signals, double* lam0, double* scale) {
  double lo = 0.0, hi = 2.0;
  for (int it = 0; it < 50; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_from_moments(mid, p, mom) < k)
      lo = mid;
    else
      hi = mid;
  }
  const double l0 = 0.5 * (lo + hi), h = 1e-3;
  const double a = std::max(0.0, l0 - h), b = std::min(2.0, l0 + h);
  const double slope = (count_from_moments(b, p, mom) - count_from_moments(a, p, mom)) / (b - a);
  const double s = std::sqrt(2.0 * k / n_signals) / std::max(slope, 1e-9);
  *lam0 = l0;
  *scale = std::min(std::max(s, 1e-4), 0.5);
}

void learned_begin(LearnedState& S, const double* mom, int p, int k, int n_signals, double c1,
                   const float y[2]) {
  S.half_lo = c1 < k ? 1.0 : 0.0;
  S.half_hi = c1 < k ? 2.0 : 1.0;
  double l0 = 0.0, sc = 0.0;
  count_root(mom, p, k, n_signals, &l0, &sc);
  double lo = l0 + sc * std::min(y[0], y[1]), hi = l0 + sc * std::max(y[0], y[1]);
  lo = std::max(lo, S.half_lo);
  hi = std::min(hi, S.half_hi);
  if (!(hi - lo >= 1.0 / 1024)) {  // empty or degenerate: a narrow bracket at lambda_0
    const double c = std::min(std::max(l0, S.half_lo), S.half_hi);
    lo = std::max(S.half_lo, c - std::max(sc, 1.0 / 1024));
    hi = std::min(S.half_hi, c + std::max(sc, 1.0 / 1024));
  }
  S.lo = S.lo0 = lo;
  S.hi = S.hi0 = hi;
  S.inside = 0;
  S.below = S.above = S.widened = false;
  S.status = CSC_OK;
}

bool learned_update(LearnedState& S, double mid, double cnt, int k) {
  if (std::floor(cnt + 0.5) == (double)k) return true;
  ++S.inside;
  if (cnt < k) {
    S.lo = mid;
    S.below = true;
  } else {
    S.hi = mid;
    S.above = true;
  }
  // four one-sided tests inside the bracket (the interval is then a
  // sixteenth of it): lambda_k is taken to lie outside, reopen once
  if (!S.widened && !(S.below && S.above) && S.inside >= 4) {
    S.widened = true;
    S.status = CSC_W_BRACKET_MISS;
    if (S.below && S.hi0 < S.half_hi) {
      S.lo = S.hi0;
      S.hi = S.half_hi;
    } else if (S.above && S.lo0 > S.half_lo) {
      S.hi = S.lo0;
      S.lo = S.half_lo;
    }
  }
  return false;
}

size_t mlp_workspace(int B) { return mlp_ws(B); }

}  // namespace csc

using namespace csc;

extern "C" int32_t csc_mlp_param_count(void) { return kParams; }

extern "C" size_t csc_mlp_workspace_bytes(int32_t B) { return B < 1 ? 0 : mlp_ws(B); }

extern "C" csc_status csc_mlp_features(const double* moments, int32_t p, int32_t N, int32_t k,
                                       float* x_out) {
  clear_error();
  CSC_REQUIRE(moments && x_out, "moments and x_out must be non-NULL");
  CSC_REQUIRE(p >= 50, "the features need moments up to order 50 (p >= 50)");
  CSC_REQUIRE(N >= 1 && k >= 1 && moments[0] > 0.0, "need N >= 1, k >= 1, moments[0] > 0");
  features(moments, N, k, x_out);
  return CSC_OK;
}

extern "C" csc_status csc_mlp_forward(const float* params, const float* X, int32_t B, float* Y,
                                      void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  CSC_REQUIRE(params && X && Y && B >= 1, "need params, X, Y and B >= 1");
  CSC_TRY(check_ws(ws, ws_bytes, mlp_ws(B)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  const MlpBuffers m = carve_mlp(ar, B);
  CSC_TRY(forward(params, X, B, m, s));
  CSC_HIP(hipMemcpyAsync(Y, m.Y, (size_t)B * kOut * sizeof(float), hipMemcpyDeviceToDevice, s));
  return CSC_OK;
}

extern "C" csc_status csc_mlp_loss_grad(const float* params, const float* X, const float* target,
                                        int32_t B, float* grad, double* loss_out, void* ws,
                                        size_t ws_bytes, void* stream) {
  clear_error();
  CSC_REQUIRE(params && X && target && grad && B >= 1, "need params, X, target, grad, B >= 1");
  CSC_TRY(check_ws(ws, ws_bytes, mlp_ws(B)));
  hipStream_t s = as_stream(stream);
  Arena ar(ws, ws_bytes);
  const MlpBuffers m = carve_mlp(ar, B);
  CSC_TRY(forward(params, X, B, m, s));
  hipLaunchKernelGGL(k_pinball, dim3((B + 255) / 256), dim3(256), 0, s, m.Y, target, B, m.dY,
                     m.lossb);
  // layer 3: gW3, gb3 from A2 and dY; dZ2 = (dY W3^T) * GELU'(Z2)
  hipLaunchKernelGGL(k_weight_grad, dim3(kH + 1, 1), dim3(kOut), 0, s, m.A2, kH, m.dY, kOut, B,
                     grad + kOffW3, grad + kOffB3);
  hipLaunchKernelGGL(k_backprop, dim3(B), dim3(128), 0, s, m.dY, kOut, params + kOffW3, kH, m.Z2,
                     m.dZ2);
  hipLaunchKernelGGL(k_weight_grad, dim3(kH + 1, 1), dim3(kH), 0, s, m.A1, kH, m.dZ2, kH, B,
                     grad + kOffW2, grad + kOffB2);
  hipLaunchKernelGGL(k_backprop, dim3(B), dim3(128), 0, s, m.dZ2, kH, params + kOffW2, kH, m.Z1,
                     m.dZ1);
  hipLaunchKernelGGL(k_weight_grad, dim3(kIn + 1, 1), dim3(kH), 0, s, X, kIn, m.dZ1, kH, B,
                     grad + kOffW1, grad + kOffB1);
  CSC_HIP(hipGetLastError());
  if (loss_out) {
    hipLaunchKernelGGL(k_sum_f64, dim3(1), dim3(64), 0, s, m.lossb, B, m.loss);
    CSC_HIP(hipGetLastError());
    double h = 0.0;
    CSC_HIP(hipMemcpyAsync(&h, m.loss, sizeof(double), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    *loss_out = h / B;
  }
  return CSC_OK;
}

extern "C" csc_status csc_mlp_adam_step(float* params, const float* grad, float* m, float* v,
                                        int32_t step, float lr, void* stream) {
  clear_error();
  CSC_REQUIRE(params && grad && m && v && step >= 1 && lr > 0.f, "bad Adam arguments");
  const float b1 = 0.9f, b2 = 0.999f;
  const float bc1 = (float)(1.0 - std::pow(0.9, step)), bc2 = (float)(1.0 - std::pow(0.999, step));
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, as_stream(stream), params,
                     grad, m, v, kParams, lr, b1, b2, 1e-8f, bc1, bc2);
  CSC_HIP(hipGetLastError());
  return CSC_OK;
}

// ----------------------------------------------------- learned dichotomy ---
extern "C" csc_status csc_count_root(const double* moments, int32_t p, int32_t k,
                                     int32_t n_signals, double* lambda0_out, double* scale_out) {
  clear_error();
  CSC_REQUIRE(moments && lambda0_out && scale_out, "moments and outputs must be non-NULL");
  CSC_REQUIRE(p >= 1 && k >= 1 && n_signals >= 1, "need p, k, n_signals >= 1");
  count_root(moments, p, k, n_signals, lambda0_out, scale_out);
  return CSC_OK;
}

extern "C" size_t csc_estimate_workspace_bytes_learned(int32_t n, int32_t n_signals, int32_t p) {
  return csc_estimate_workspace_bytes(n, n_signals, p) + mlp_ws(1) + 1024;
}

extern "C" csc_status csc_estimate_lambda_k_learned(const csc_graph* g, int32_t k, int32_t p,
                                                    int32_t n_signals, uint64_t seed,
                                                    int32_t max_steps, const float* params,
                                                    double* lambda_out, int32_t* steps_out,
                                                    double* trace_out, double* bracket_out,
                                                    void* ws, size_t ws_bytes, void* stream) {
  clear_error();
  CSC_TRY(check_graph(g));
  CSC_REQUIRE(params && lambda_out && steps_out, "params, lambda_out, steps_out must be non-NULL");
  CSC_REQUIRE(k >= 1 && k <= g->n && p >= 50 && n_signals >= 1 && max_steps >= 2,
              "need 1 <= k <= N, p >= 50, n_signals >= 1, max_steps >= 2");
  const size_t est_ws = csc_estimate_workspace_bytes(g->n, n_signals, p);
  CSC_TRY(check_ws(ws, ws_bytes, csc_estimate_workspace_bytes_learned(g->n, n_signals, p)));
  hipStream_t s = as_stream(stream);
  char* base = (char*)ws;
  void* est = base;
  Arena ar(base + align_up(est_ws), ws_bytes - align_up(est_ws));
  float* dx = ar.take<float>(kIn);
  float* dy = ar.take<float>(kOut);
  char* mws = ar.take<char>(mlp_ws(1));

  // Passes 1, 2, ... with fresh signals each: pass 1 is the first pass of the
  // plain dichotomy (lambda = 1) and its moments give the network's bracket;
  // the later ones bisect inside that bracket.
  LearnedState S;
  int used = 0;
  bool done = false;
  double lam = 0.0;
  csc_status st = CSC_OK;
  // the bracket from the network on the first pass's moments (count c1 at 1)
  auto network = [&](const double* mom, double c1) -> csc_status {
    float x[kIn], y[kOut];
    features(mom, g->n, k, x);
    CSC_HIP(hipMemcpyAsync(dx, x, sizeof(x), hipMemcpyHostToDevice, s));
    CSC_TRY(csc_mlp_forward(params, dx, 1, dy, mws, mlp_ws(1), stream));
    CSC_HIP(hipMemcpyAsync(y, dy, sizeof(y), hipMemcpyDeviceToHost, s));
    CSC_HIP(hipStreamSynchronize(s));
    learned_begin(S, mom, p, k, n_signals, c1, y);
    return CSC_OK;
  };
  auto more = [&](uint32_t, const double* mom) -> bool {
    const double mid = used == 0 ? 1.0 : 0.5 * (S.lo + S.hi);
    const double cnt = count_from_moments(mid, p, mom);
    if (trace_out) {
      trace_out[2 * used] = mid;
      trace_out[2 * used + 1] = cnt;
    }
    ++used;
    if (used == 1) {
      if (std::floor(cnt + 0.5) == (double)k) {
        done = true;
        lam = 1.0;
        if (bracket_out) bracket_out[0] = bracket_out[1] = 1.0;
        return false;
      }
      if ((st = network(mom, cnt)) != CSC_OK) return false;
      if (bracket_out) {
        bracket_out[0] = S.lo;
        bracket_out[1] = S.hi;
      }
      return used < max_steps;
    }
    if (learned_update(S, mid, cnt, k)) {
      done = true;
      lam = mid;
      return false;
    }
    return used < max_steps;
  };
  CSC_TRY(count_passes(*g, n_signals, p, seed, 1, est, est_ws, s, more));
  CSC_TRY(st);
  *steps_out = used;
  if (done) {
    *lambda_out = lam;
    return used == 1 ? CSC_OK : S.status;
  }
  *lambda_out = S.hi;
  return S.status == CSC_OK ? CSC_W_BISECT_EXHAUSTED : S.status;
}
