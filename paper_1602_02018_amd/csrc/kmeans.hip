// k-means on the sampled features (Alg. 2 step 6), host float64.
//
// The paper runs Matlab's kmeans with 20 replicates and a 100-iteration cap
// (Sec. 5).  This implementation fixes every rounding so that it is
// reproducible: squared distances sum coordinates in increasing order, the
// k-means++ weights are summed in blocks of kSeedBlock points (block offset
// plus in-block running sum, each in order), centroids sum member points in
// increasing index order, and ties go to the lowest index.  Replicates run on worker threads; the winner is chosen in
// replicate order, so the result does not depend on scheduling.  This file is
// compiled with floating-point contraction disabled.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "common.hpp"
#include "kmeans.hpp"

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

// Eight squared distances at once, each summed over coordinates in order
// exactly as sqd does (independent chains, so the loop pipelines and
// vectorises without changing any rounding).
constexpr int kB = 8;

// x (d coordinates) against the centroids c0 .. c0+7 stored transposed:
// coordinate j of centroid c at Ct[j * kp + c].
inline void sqd_centroids8(const double* x, const double* Ct, int kp, int c0, int d, double* out) {
  double acc[kB] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = 0; j < d; ++j) {
    const double xj = x[j];
    const double* cr = Ct + (size_t)j * kp + c0;
    for (int u = 0; u < kB; ++u) {
      const double diff = xj - cr[u];
      acc[u] = acc[u] + diff * diff;
    }
  }
  for (int u = 0; u < kB; ++u) out[u] = acc[u];
}

// points i0 .. i0+7 stored transposed (coordinate j of point i at Xt[j * np + i])
// against one centroid c.
inline void sqd_points8(const double* Xt, int np, int i0, const double* c, int d, double* out) {
  double acc[kB] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int j = 0; j < d; ++j) {
    const double cj = c[j];
    const double* xr = Xt + (size_t)j * np + i0;
    for (int u = 0; u < kB; ++u) {
      const double diff = xr[u] - cj;
      acc[u] = acc[u] + diff * diff;
    }
  }
  for (int u = 0; u < kB; ++u) out[u] = acc[u];
}

inline int round8(int v) { return (v + kB - 1) / kB * kB; }

// A point set in both layouts: X (n x d) and Xt (d x np, np = n rounded up to 8,
// padding points at the origin).
struct Points {
  const double* X;
  std::vector<double> Xt;
  int n, d, np;
  Points(const double* X_, int n_, int d_) : X(X_), n(n_), d(d_), np(round8(n_)) {
    Xt.assign((size_t)d * np, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < d; ++j) Xt[(size_t)j * np + i] = X[(size_t)i * d + j];
  }
};

// squared distances of every point to centroid c (n entries of out)
void dist_to(const Points& P, const double* c, double* out) {
  double v[kB];
  for (int i0 = 0; i0 < P.n; i0 += kB) {
    sqd_points8(P.Xt.data(), P.np, i0, c, P.d, v);
    for (int u = 0; u < kB && i0 + u < P.n; ++u) out[i0 + u] = v[u];
  }
}

struct Run {
  std::vector<int> labels;
  double inertia = 0.0;
};

void seed_plusplus(const Points& P, int k, uint64_t seed, int r, double* C, int32_t* picks = nullptr) {
  const int n = P.n, d = P.d;
  const double* X = P.X;
  std::vector<double> mind(n), cum(n), dist(n);
  double u = draw_uniform(seed, 0, (uint64_t)r);
  int first = std::min((int)std::floor(u * n), n - 1);
  if (picks) picks[0] = first;
  std::memcpy(C, X + (size_t)first * d, d * sizeof(double));
  dist_to(P, C, mind.data());
  for (int c = 1; c < k; ++c) {
    u = draw_uniform(seed, (uint64_t)c, (uint64_t)r);
    // running sums in blocks of kSeedBlock points: block offset plus the
    // running sum inside the block, both in index order
    double off = 0.0;
    for (int b0 = 0; b0 < n; b0 += kSeedBlock) {
      const int b1 = std::min(n, b0 + kSeedBlock);
      double in = 0.0;
      for (int i = b0; i < b1; ++i) {
        in = in + mind[i];
        cum[i] = off + in;
      }
      off = off + in;
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
    if (pick >= n) pick = n - 1;  // only with non-finite weights
    if (picks) picks[c] = pick;
    double* cc = C + (size_t)c * d;
    std::memcpy(cc, X + (size_t)pick * d, d * sizeof(double));
    dist_to(P, cc, dist.data());
    for (int i = 0; i < n; ++i) mind[i] = dist[i] < mind[i] ? dist[i] : mind[i];
  }
}

// nearest centroid of every point (ties to the lowest index); Ct is C transposed
void assign(const Points& P, int k, const double* Ct, int kp, int* lab) {
  double v[kB];
  for (int i = 0; i < P.n; ++i) {
    const double* x = P.X + (size_t)i * P.d;
    double best = 0.0;
    int arg = 0;
    for (int c0 = 0; c0 < k; c0 += kB) {
      sqd_centroids8(x, Ct, kp, c0, P.d, v);
      for (int u = 0; u < kB && c0 + u < k; ++u) {
        if (c0 + u == 0 || v[u] < best) {
          best = v[u];
          arg = c0 + u;
        }
      }
    }
    lab[i] = arg;
  }
}

void transpose_centroids(const std::vector<double>& C, int k, int d, int kp, std::vector<double>& Ct) {
  Ct.assign((size_t)d * kp, 0.0);
  for (int c = 0; c < k; ++c)
    for (int j = 0; j < d; ++j) Ct[(size_t)j * kp + c] = C[(size_t)c * d + j];
}

Run lloyd(const Points& P, int k, std::vector<double>& C, int max_iter) {
  const int n = P.n, d = P.d, kp = round8(k);
  const double* X = P.X;
  Run out;
  std::vector<int> labels, fresh(n), counts(k);
  std::vector<double> sum(d), Ct;
  bool have = false, reseeded = false;
  for (int it = 0; it < max_iter; ++it) {
    transpose_centroids(C, k, d, kp, Ct);
    assign(P, k, Ct.data(), kp, fresh.data());
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
  const Points P(X, n, d);
  auto work = [&](int r) {
    std::vector<double> C((size_t)k * d);
    seed_plusplus(P, k, seed, r, C.data());
    runs[r] = lloyd(P, k, C, max_iter);
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
  std::vector<Points> P;
  P.reserve(G);
  for (int g = 0; g < G; ++g) P.emplace_back(X[g].data(), n[g], d[g]);
  auto work = [&](int job) {
    const int g = job / replicates, r = job - g * replicates;
    std::vector<double> C((size_t)k[g] * d[g]);
    seed_plusplus(P[g], k[g], seeds[g], r, C.data());
    runs[g][r] = lloyd(P[g], k[g], C, max_iter);
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

extern "C" csc_status csc_kmeans_seeds(const double* F, int32_t n, int32_t d, int32_t ld, int32_t k,
                                       int32_t replicates, uint64_t seed, int32_t* picks) {
  clear_error();
  CSC_TRY(check_kmeans_args(F, n, d, ld, k, replicates, 1, picks));
  std::vector<double> X((size_t)n * d);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < d; ++j) X[(size_t)i * d + j] = F[(size_t)i * ld + j];
  const Points P(X.data(), n, d);
  std::vector<double> C((size_t)k * d);
  for (int r = 0; r < replicates; ++r) seed_plusplus(P, k, seed, r, C.data(), picks + (size_t)r * k);
  return CSC_OK;
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

// Community cores: the k largest classes of sampled nodes that share their
// label in every run (tuple of T labels), ranked by size and then by their
// first member's position; members of core c get label c, others -1.
extern "C" csc_status csc_community_cores(int32_t n, int32_t T, int32_t k, const int32_t* labels,
                                          int32_t* core_labels) {
  clear_error();
  CSC_REQUIRE(n >= 1 && T >= 1 && k >= 1, "need n >= 1, T >= 1 and k >= 1");
  CSC_REQUIRE(labels && core_labels, "labels and core_labels must be non-NULL");
  std::vector<int> idx(n);
  for (int s = 0; s < n; ++s) idx[s] = s;
  auto less = [&](int a, int b) {
    for (int t = 0; t < T; ++t) {
      const int la = labels[(size_t)t * n + a], lb = labels[(size_t)t * n + b];
      if (la != lb) return la < lb;
    }
    return false;
  };
  std::stable_sort(idx.begin(), idx.end(), less);  // equal tuples keep sample order
  struct Cls {
    int size, first, begin;
  };
  std::vector<Cls> cls;
  for (int i = 0; i < n;) {
    int j = i + 1;
    while (j < n && !less(idx[i], idx[j]) && !less(idx[j], idx[i])) ++j;
    cls.push_back(Cls{j - i, idx[i], i});
    i = j;
  }
  std::sort(cls.begin(), cls.end(), [](const Cls& a, const Cls& b) {
    return a.size != b.size ? a.size > b.size : a.first < b.first;
  });
  for (int s = 0; s < n; ++s) core_labels[s] = -1;
  for (int c = 0; c < (int)cls.size() && c < k; ++c)
    for (int q = cls[c].begin; q < cls[c].begin + cls[c].size; ++q) core_labels[idx[q]] = c;
  return CSC_OK;
}
