// k-means on the sampled features (Alg. 2 step 6), host float64.
//
// The paper runs Matlab's kmeans with 20 replicates and a 100-iteration cap
// (Sec. 5).  This implementation fixes every rounding so that it is
// reproducible: squared distances sum coordinates in increasing order,
// centroids sum member points in increasing index order, and ties go to the
// lowest index.  Replicates run on worker threads; the winner is chosen in
// replicate order, so the result does not depend on scheduling.  This file is
// compiled with floating-point contraction disabled.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "common.hpp"

namespace csc {
namespace {

double draw_uniform(uint64_t seed, uint64_t j, uint64_t r) {
  const Words4 x = philox4x64_10(j, r, (uint64_t)CSC_STREAM_KMEANS, 0ull, seed, 0ull);
  return (double)(x.x0 >> 11) * 0x1p-53;
}

inline double sqd(const double* x, const double* c, int d) {
  double acc = 0.0;
  for (int j = 0; j < d; ++j) {
    const double diff = x[j] - c[j];
    acc = acc + diff * diff;
  }
  return acc;
}

struct Run {
  std::vector<int> labels;
  double inertia = 0.0;
};

void seed_plusplus(const double* X, int n, int d, int k, uint64_t seed, int r, double* C) {
  std::vector<double> mind(n), cum(n);
  double u = draw_uniform(seed, 0, (uint64_t)r);
  int first = std::min((int)std::floor(u * n), n - 1);
  std::memcpy(C, X + (size_t)first * d, d * sizeof(double));
  for (int i = 0; i < n; ++i) mind[i] = sqd(X + (size_t)i * d, C, d);
  for (int c = 1; c < k; ++c) {
    u = draw_uniform(seed, (uint64_t)c, (uint64_t)r);
    double run = 0.0;
    for (int i = 0; i < n; ++i) {
      run = run + mind[i];
      cum[i] = run;
    }
    const double total = cum[n - 1];
    int pick;
    if (total == 0.0) {
      pick = std::min((int)std::floor(u * n), n - 1);
    } else {
      const double target = u * total;
      pick = n;
      for (int i = 0; i < n; ++i)
        if (cum[i] > target) {
          pick = i;
          break;
        }
      if (pick >= n)
        for (int i = n - 1; i >= 0; --i)
          if (mind[i] > 0.0) {
            pick = i;
            break;
          }
    }
    double* cc = C + (size_t)c * d;
    std::memcpy(cc, X + (size_t)pick * d, d * sizeof(double));
    for (int i = 0; i < n; ++i) {
      const double v = sqd(X + (size_t)i * d, cc, d);
      mind[i] = v < mind[i] ? v : mind[i];
    }
  }
}

void assign(const double* X, int n, int d, int k, const double* C, int* lab) {
  for (int i = 0; i < n; ++i) {
    const double* x = X + (size_t)i * d;
    double best = sqd(x, C, d);
    int arg = 0;
    for (int c = 1; c < k; ++c) {
      const double v = sqd(x, C + (size_t)c * d, d);
      if (v < best) {
        best = v;
        arg = c;
      }
    }
    lab[i] = arg;
  }
}

Run lloyd(const double* X, int n, int d, int k, std::vector<double>& C, int max_iter) {
  Run out;
  std::vector<int> labels, fresh(n), counts(k);
  std::vector<double> sum(d);
  bool have = false, reseeded = false;
  for (int it = 0; it < max_iter; ++it) {
    assign(X, n, d, k, C.data(), fresh.data());
    if (have && !reseeded && fresh == labels) break;
    labels = fresh;
    have = true;
    std::fill(counts.begin(), counts.end(), 0);
    for (int i = 0; i < n; ++i) ++counts[labels[i]];
    for (int c = 0; c < k; ++c) {
      if (counts[c] == 0) continue;
      std::fill(sum.begin(), sum.end(), 0.0);
      for (int i = 0; i < n; ++i)
        if (labels[i] == c)
          for (int j = 0; j < d; ++j) sum[j] = sum[j] + X[(size_t)i * d + j];
      for (int j = 0; j < d; ++j) C[(size_t)c * d + j] = sum[j] / (double)counts[c];
    }
    reseeded = false;
    for (int c = 0; c < k; ++c) reseeded = reseeded || counts[c] == 0;
    for (int c = 0; c < k; ++c) {
      if (counts[c] != 0) continue;
      int far = 0;
      double fd = -1.0;
      for (int i = 0; i < n; ++i) {
        const double v = sqd(X + (size_t)i * d, C.data() + (size_t)labels[i] * d, d);
        if (v > fd) {
          fd = v;
          far = i;
        }
      }
      std::memcpy(C.data() + (size_t)c * d, X + (size_t)far * d, d * sizeof(double));
      --counts[labels[far]];
      labels[far] = c;
      counts[c] = 1;
    }
  }
  double acc = 0.0;
  for (int i = 0; i < n; ++i)
    acc = acc + sqd(X + (size_t)i * d, C.data() + (size_t)labels[i] * d, d);
  out.labels = labels;
  out.inertia = acc;
  return out;
}

csc_status kmeans_f64(const double* X, int n, int d, int k, int replicates, int max_iter,
                      uint64_t seed, int32_t* labels, double* inertia_out) {
  std::vector<Run> runs(replicates);
  auto work = [&](int r) {
    std::vector<double> C((size_t)k * d);
    seed_plusplus(X, n, d, k, seed, r, C.data());
    runs[r] = lloyd(X, n, d, k, C, max_iter);
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nt = std::min<int>((int)hw, replicates);
  if (nt <= 1) {
    for (int r = 0; r < replicates; ++r) work(r);
  } else {
    std::vector<std::thread> pool;
    for (int t = 0; t < nt; ++t)
      pool.emplace_back([&, t] {
        for (int r = t; r < replicates; r += nt) work(r);
      });
    for (auto& th : pool) th.join();
  }
  int best = 0;
  for (int r = 1; r < replicates; ++r)
    if (runs[r].inertia < runs[best].inertia) best = r;
  std::memcpy(labels, runs[best].labels.data(), (size_t)n * sizeof(int32_t));
  if (inertia_out) *inertia_out = runs[best].inertia;
  return CSC_OK;
}

csc_status kmeans_batched(int G, const std::vector<std::vector<double>>& X, const int32_t* n,
                          const int32_t* d, const int32_t* k, int replicates, int max_iter,
                          const uint64_t* seeds, int32_t* const* labels, double* inertia_out) {
  std::vector<std::vector<Run>> runs(G, std::vector<Run>(replicates));
  const int total = G * replicates;
  auto work = [&](int job) {
    const int g = job / replicates, r = job - g * replicates;
    std::vector<double> C((size_t)k[g] * d[g]);
    seed_plusplus(X[g].data(), n[g], d[g], k[g], seeds[g], r, C.data());
    runs[g][r] = lloyd(X[g].data(), n[g], d[g], k[g], C, max_iter);
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  const int nt = std::min<int>((int)hw, total);
  std::vector<std::thread> pool;
  for (int t = 0; t < nt; ++t)
    pool.emplace_back([&, t] {
      for (int job = t; job < total; job += nt) work(job);
    });
  for (auto& th : pool) th.join();
  for (int g = 0; g < G; ++g) {
    int best = 0;
    for (int r = 1; r < replicates; ++r)
      if (runs[g][r].inertia < runs[g][best].inertia) best = r;
    std::memcpy(labels[g], runs[g][best].labels.data(), (size_t)n[g] * sizeof(int32_t));
    if (inertia_out) inertia_out[g] = runs[g][best].inertia;
  }
  return CSC_OK;
}

csc_status check_kmeans_args(const void* F, int n, int d, int ld, int k, int replicates,
                             int max_iter, const int32_t* labels) {
  CSC_REQUIRE(F && labels, "F and labels must be non-NULL");
  CSC_REQUIRE(n >= 1 && d >= 1 && ld >= d, "need n >= 1, d >= 1, ld >= d");
  CSC_REQUIRE(k >= 1 && k <= n, "k must lie in [1, n]");
  CSC_REQUIRE(replicates >= 1 && max_iter >= 1, "need replicates >= 1 and max_iter >= 1");
  return CSC_OK;
}

}  // namespace
}  // namespace csc

using namespace csc;

extern "C" csc_status csc_kmeans_reduced(const float* F, int32_t n, int32_t d, int32_t ld,
                                         int32_t k, int32_t replicates, int32_t max_iter,
                                         uint64_t seed, int32_t* labels, double* inertia_out) {
  clear_error();
  CSC_TRY(check_kmeans_args(F, n, d, ld, k, replicates, max_iter, labels));
  std::vector<double> X((size_t)n * d);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) X[(size_t)i * d + j] = (double)F[(size_t)i * ld + j];
  return kmeans_f64(X.data(), n, d, k, replicates, max_iter, seed, labels, inertia_out);
}

extern "C" csc_status csc_kmeans_reduced_f64(const double* F, int32_t n, int32_t d, int32_t ld,
                                             int32_t k, int32_t replicates, int32_t max_iter,
                                             uint64_t seed, int32_t* labels,
                                             double* inertia_out) {
  clear_error();
  CSC_TRY(check_kmeans_args(F, n, d, ld, k, replicates, max_iter, labels));
  std::vector<double> X((size_t)n * d);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) X[(size_t)i * d + j] = F[(size_t)i * ld + j];
  return kmeans_f64(X.data(), n, d, k, replicates, max_iter, seed, labels, inertia_out);
}

extern "C" csc_status csc_kmeans_reduced_batched(int32_t G, const float* const* F, const int32_t* n,
                                                 const int32_t* d, const int32_t* k,
                                                 int32_t replicates, int32_t max_iter,
                                                 const uint64_t* seeds, int32_t* const* labels,
                                                 double* inertia_out) {
  clear_error();
  CSC_REQUIRE(G >= 1 && F && n && d && k && seeds && labels, "bad batched k-means arguments");
  std::vector<std::vector<double>> X(G);
  for (int g = 0; g < G; ++g) {
    CSC_TRY(check_kmeans_args(F[g], n[g], d[g], d[g], k[g], replicates, max_iter, labels[g]));
    X[g].resize((size_t)n[g] * d[g]);
    for (size_t e = 0; e < X[g].size(); ++e) X[g][e] = (double)F[g][e];
  }
  return kmeans_batched(G, X, n, d, k, replicates, max_iter, seeds, labels, inertia_out);
}
