// C entry points over the host float64 algebra of the block CG, built by
// tests/test_dense_host.py with the system C++ compiler.
#include <cmath>
#include <cstring>
#include <vector>

#include "../paper_1602_02018_amd/csrc/dense.hpp"

extern "C" int dense_orth(const double* G, int k, double rtol, double* T) {
  std::vector<double> g(G, G + (size_t)k * k), t;
  const int s = csc::dense::orth_transform(g, k, rtol, t);
  std::memcpy(T, t.data(), (size_t)k * k * sizeof(double));
  return s;
}

extern "C" int dense_solve(const double* W, int s, double* C, int k, double scale, int threads) {
  std::vector<double> w(W, W + (size_t)s * s), c(C, C + (size_t)s * k);
  if (!csc::dense::cholesky(w, s, s)) return 0;
  csc::dense::chol_solve(w, s, s, c, k, scale, threads);
  std::memcpy(C, c.data(), (size_t)s * k * sizeof(double));
  return 1;
}

// The textbook forms of the same computations, for bit-for-bit comparison:
// the library's routines reorganise the loops (a left-looking factorisation,
// register tiles of several rows) but must take, for every entry, the same
// operations in the same order as these.

// Outer-product pivoted Cholesky of the unit-diagonal scaling of G (every
// row of the remaining matrix updated after each pivot), then the factor's
// inverse row by row and T from it.
extern "C" int dense_orth_plain(const double* G, int k, double rtol, double* T) {
  std::vector<double> d(k), A((size_t)k * k), F((size_t)k * k, 0.0), diag(k);
  for (int i = 0; i < k; ++i) {
    const double g = G[(size_t)i * k + i];
    d[i] = g > 0.0 ? std::sqrt(g) : 0.0;
  }
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j)
      A[(size_t)i * k + j] = (d[i] > 0.0 && d[j] > 0.0) ? G[(size_t)i * k + j] / (d[i] * d[j]) : 0.0;
  for (int i = 0; i < k; ++i) diag[i] = d[i] > 0.0 ? A[(size_t)i * k + i] : -1.0;
  std::vector<int> piv;
  for (int r = 0; r < k; ++r) {
    int j = 0;
    for (int i = 1; i < k; ++i)
      if (diag[i] > diag[j]) j = i;
    if (!(diag[j] > rtol)) break;
    const double ljj = std::sqrt(diag[j]);
    double* l = F.data() + (size_t)r * k;  // factor column r, by original index
    for (int i = 0; i < k; ++i)
      l[i] = i == j ? ljj : (diag[i] >= 0.0 ? A[(size_t)i * k + j] / ljj : 0.0);
    diag[j] = -1.0;
    for (int i = 0; i < k; ++i) {
      if (diag[i] < 0.0) continue;
      for (int c = 0; c < k; ++c) A[(size_t)i * k + c] -= l[i] * l[c];
      diag[i] -= l[i] * l[i];
    }
    piv.push_back(j);
  }
  const int s = (int)piv.size();
  std::vector<double> X((size_t)s * s, 0.0);
  for (int r = 0; r < s; ++r) {
    X[(size_t)r * s + r] = 1.0;
    for (int t = 0; t < r; ++t)
      for (int c = 0; c <= t; ++c) X[(size_t)r * s + c] -= F[(size_t)t * k + piv[r]] * X[(size_t)t * s + c];
    for (int c = 0; c <= r; ++c) X[(size_t)r * s + c] /= F[(size_t)r * k + piv[r]];
  }
  std::memset(T, 0, (size_t)k * k * sizeof(double));
  for (int r = 0; r < s; ++r)
    for (int c = r; c < s; ++c) T[(size_t)piv[r] * k + c] = X[(size_t)c * s + r] / d[piv[r]];
  return s;
}

// Given the factor L (lower triangle of W), C <- scale * (L L^T)^{-1} C by
// forward then back substitution, one row at a time.
extern "C" void dense_subst_plain(const double* L, int s, double* C, int k, double scale) {
  for (int i = 0; i < s; ++i) {
    for (int t = 0; t < i; ++t)
      for (int j = 0; j < k; ++j) C[(size_t)i * k + j] -= L[(size_t)i * s + t] * C[(size_t)t * k + j];
    for (int j = 0; j < k; ++j) C[(size_t)i * k + j] /= L[(size_t)i * s + i];
  }
  for (int i = s - 1; i >= 0; --i) {
    for (int t = i + 1; t < s; ++t)
      for (int j = 0; j < k; ++j) C[(size_t)i * k + j] -= L[(size_t)t * s + i] * C[(size_t)t * k + j];
    for (int j = 0; j < k; ++j) C[(size_t)i * k + j] /= L[(size_t)i * s + i];
  }
  if (scale != 1.0)
    for (size_t e = 0; e < (size_t)s * k; ++e) C[e] *= scale;
}

// The Cholesky factor alone (lower triangle of W in place); 0 if W is not
// positive definite.
extern "C" int dense_factor(double* W, int s) {
  std::vector<double> w(W, W + (size_t)s * s);
  if (!csc::dense::cholesky(w, s, s)) return 0;
  std::memcpy(W, w.data(), (size_t)s * s * sizeof(double));
  return 1;
}
