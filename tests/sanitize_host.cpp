// Host-only checks of the library's CPU code, built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_host.py: the host k-means
// (seeding, Lloyd, replicate threads, batched form), community cores and the
// block CG's dense float64 algebra, over random and degenerate inputs
// (n = 1, k = n, duplicate points, all points equal, zero columns,
// rank-deficient Gram matrices) and rejected arguments.  Exits non-zero on the
// first failed check; the sanitizers abort on the first memory or UB error.
#include <cmath>
#include <cstdio>
#include <random>
#include <string>
#include <vector>

#include "../include/csc.h"
#include "../paper_1602_02018_amd/csrc/dense.hpp"

namespace csc {
// the library's error hooks live in its GPU translation unit; this harness
// links only the host code
void set_error(const std::string&) {}
void clear_error() {}
}  // namespace csc

static int failures = 0;
#define CHECK(c)                                                  \
  do {                                                            \
    if (!(c)) {                                                   \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
      ++failures;                                                 \
    }                                                             \
  } while (0)

static void kmeans_case(int n, int d, int k, int reps, unsigned seed, int mode) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> N01;
  std::vector<double> F((size_t)n * d);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) {
      double v = N01(g);
      if (mode == 1) v = (double)((i % 3) == j % 3);  // many duplicate points
      if (mode == 2) v = 0.5;                          // every point equal: zero D^2 total
      F[(size_t)i * d + j] = v;
    }
  std::vector<int32_t> lab(n, -7), picks((size_t)reps * k, -7);
  double inertia = -1.0;
  CHECK(csc_kmeans_reduced_f64(F.data(), n, d, d, k, reps, 100, seed, lab.data(), &inertia) == CSC_OK);
  for (int i = 0; i < n; ++i) CHECK(lab[i] >= 0 && lab[i] < k);
  CHECK(std::isfinite(inertia) && inertia >= 0.0);
  CHECK(csc_kmeans_seeds(F.data(), n, d, d, k, reps, seed, picks.data()) == CSC_OK);
  for (int v : picks) CHECK(v >= 0 && v < n);
  // float32 input with a leading dimension above d
  std::vector<float> Ff((size_t)n * (d + 3), 9.0f);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) Ff[(size_t)i * (d + 3) + j] = (float)F[(size_t)i * d + j];
  std::vector<int32_t> lab2(n, -7);
  CHECK(csc_kmeans_reduced(Ff.data(), n, d, d + 3, k, reps, 100, seed, lab2.data(), nullptr) == CSC_OK);
  for (int i = 0; i < n; ++i) CHECK(lab2[i] >= 0 && lab2[i] < k);
}

static void kmeans_batched_case() {
  const int G = 3;
  int32_t n[G] = {40, 1, 17}, d[G] = {5, 3, 2}, k[G] = {7, 1, 17};
  uint64_t seeds[G] = {1, 2, 3};
  std::vector<std::vector<float>> F(G);
  std::vector<std::vector<int32_t>> L(G);
  std::vector<const float*> fp(G);
  std::vector<int32_t*> lp(G);
  std::mt19937 g(5);
  std::uniform_real_distribution<float> U(-1.f, 1.f);
  for (int i = 0; i < G; ++i) {
    F[i].resize((size_t)n[i] * d[i]);
    for (auto& v : F[i]) v = U(g);
    L[i].assign(n[i], -7);
    fp[i] = F[i].data();
    lp[i] = L[i].data();
  }
  double inertia[G];
  CHECK(csc_kmeans_reduced_batched(G, fp.data(), n, d, k, 4, 50, seeds, lp.data(), inertia) == CSC_OK);
  for (int i = 0; i < G; ++i)
    for (int v : L[i]) CHECK(v >= 0 && v < k[i]);
}

static void rejected_arguments() {
  std::vector<double> F(12, 1.0);
  std::vector<int32_t> lab(4);
  CHECK(csc_kmeans_reduced_f64(nullptr, 4, 3, 3, 2, 1, 10, 0, lab.data(), nullptr) == CSC_E_INVALID_ARG);
  CHECK(csc_kmeans_reduced_f64(F.data(), 4, 3, 2, 2, 1, 10, 0, lab.data(), nullptr) == CSC_E_INVALID_ARG);
  CHECK(csc_kmeans_reduced_f64(F.data(), 4, 3, 3, 5, 1, 10, 0, lab.data(), nullptr) == CSC_E_INVALID_ARG);
  CHECK(csc_kmeans_reduced_f64(F.data(), 4, 3, 3, 0, 1, 10, 0, lab.data(), nullptr) == CSC_E_INVALID_ARG);
  CHECK(csc_kmeans_reduced_f64(F.data(), 4, 3, 3, 2, 0, 10, 0, lab.data(), nullptr) == CSC_E_INVALID_ARG);
  CHECK(csc_community_cores(0, 1, 1, lab.data(), lab.data()) == CSC_E_INVALID_ARG);
}

static void cores_case(int n, int T, int k, unsigned seed) {
  std::mt19937 g(seed);
  std::uniform_int_distribution<int> U(0, 3);
  std::vector<int32_t> labels((size_t)n * T), out(n, -9);
  for (auto& v : labels) v = U(g);
  CHECK(csc_community_cores(n, T, k, labels.data(), out.data()) == CSC_OK);
  for (int v : out) CHECK(v >= -1 && v < k);
}

static void dense_case(int k, int rank, unsigned seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> N01;
  const int m = 3 * k + 5;
  std::vector<double> B((size_t)m * rank), Z((size_t)m * k, 0.0);
  for (auto& v : B) v = N01(g);
  std::vector<double> C((size_t)rank * k);
  for (auto& v : C) v = N01(g);
  for (int i = 0; i < m; ++i)
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
      for (int r = 0; r < rank; ++r) s += B[(size_t)i * rank + r] * C[(size_t)r * k + c];
      Z[(size_t)i * k + c] = s;
    }
  if (k > 2) {
    for (int i = 0; i < m; ++i) Z[(size_t)i * k + 1] = 0.0;  // a zero column
  }
  std::vector<double> G((size_t)k * k, 0.0), T;
  for (int a = 0; a < k; ++a)
    for (int b = 0; b < k; ++b) {
      double s = 0.0;
      for (int i = 0; i < m; ++i) s += Z[(size_t)i * k + a] * Z[(size_t)i * k + b];
      G[(size_t)a * k + b] = s;
    }
  const int s = csc::dense::orth_transform(G, k, 1e-10, T);
  CHECK(s >= 0 && s <= k);
  CHECK(T.size() >= (size_t)k * (size_t)(s > 0 ? s : 1) || s == 0);
  // an SPD system of size s solved in place
  if (s > 0) {
    std::vector<double> W((size_t)s * s, 0.0), R((size_t)s * k);
    for (int a = 0; a < s; ++a) W[(size_t)a * s + a] = 2.0 + a;
    for (int a = 0; a + 1 < s; ++a) W[(size_t)a * s + a + 1] = W[(size_t)(a + 1) * s + a] = 0.5;
    for (auto& v : R) v = N01(g);
    const std::vector<double> R0 = R;
    CHECK(csc::dense::cholesky(W, s, s));
    csc::dense::chol_solve(W, s, s, R, k, 1.0);
    for (auto v : R) CHECK(std::isfinite(v));
    (void)R0;
  }
  std::vector<double> bad(4, 0.0);  // not positive definite
  CHECK(!csc::dense::cholesky(bad, 2, 2));
}

// A solve large enough to split its right-hand sides over threads, against
// the one-thread solve (same operations per element: equal bit for bit).
static void threaded_solve_case(int s, int k, int threads, unsigned seed) {
  std::mt19937_64 g(seed);
  std::normal_distribution<double> N01;
  std::vector<double> W((size_t)s * s, 0.0), R((size_t)s * k);
  for (int a = 0; a < s; ++a) W[(size_t)a * s + a] = 2.0 + a;
  for (int a = 0; a + 1 < s; ++a) W[(size_t)a * s + a + 1] = W[(size_t)(a + 1) * s + a] = 0.5;
  for (auto& v : R) v = N01(g);
  CHECK(csc::dense::cholesky(W, s, s));
  std::vector<double> R1 = R;
  csc::dense::chol_solve(W, s, s, R1, k, -1.0, 1);
  csc::dense::chol_solve(W, s, s, R, k, -1.0, threads);
  for (size_t i = 0; i < R.size(); ++i) CHECK(R[i] == R1[i]);
}

int main() {
  unsigned seed = 11;
  for (int mode = 0; mode < 3; ++mode) {
    kmeans_case(1, 3, 1, 2, seed++, mode);
    kmeans_case(9, 4, 9, 3, seed++, mode);          // k = n
    kmeans_case(100, 7, 10, 4, seed++, mode);
    kmeans_case(333, 17, 33, 2, seed++, mode);       // n not a multiple of the seeding block
    kmeans_case(64, 2, 5, 20, seed++, mode);         // whole seeding blocks, 20 replicates
  }
  kmeans_batched_case();
  rejected_arguments();
  cores_case(1, 1, 1, 3);
  cores_case(50, 4, 6, 4);
  cores_case(200, 1, 300, 5);
  for (int k : {1, 2, 5, 16, 40})
    for (int rank : {1, k / 2 + 1, k}) dense_case(k, rank, (unsigned)(k * 31 + rank));
  threaded_solve_case(128, 256, 4, 5);
  threaded_solve_case(200, 257, 3, 6);
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("sanitized host checks passed\n");
  return 0;
}
