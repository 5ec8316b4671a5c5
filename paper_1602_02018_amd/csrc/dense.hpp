// Small dense float64 algebra of the block conjugate gradient, on the host.
// Plain loops; the matrices are at most k x k with k the number of clusters.
#pragma once

#include <cmath>
#include <cstddef>
#include <vector>

namespace csc {
namespace dense {

// Rank-revealing orthonormalisation for the block CG: with G = Z^T Z (k x k,
// row-major), returns s and T (k x s, row-major, leading dimension k) such
// that P = Z T has orthonormal columns spanning the columns of Z.  Columns are
// first scaled to unit norm (so a small residual column is not mistaken for
// a dependent one); pivoted Cholesky of the scaled Gram stops when the
// largest remaining pivot falls to rtol.
inline int orth_transform(const std::vector<double>& G, int k, double rtol, std::vector<double>& T) {
  std::vector<double> d(k), A((size_t)k * k), Lm((size_t)k * k, 0.0), diag(k);
  for (int i = 0; i < k; ++i) d[i] = G[(size_t)i * k + i] > 0.0 ? std::sqrt(G[(size_t)i * k + i]) : 0.0;
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
    for (int i = 0; i < k; ++i) {
      if (diag[i] < 0.0 && i != j) continue;  // pivoted already, or a zero column
      double v = A[(size_t)i * k + j];
      for (int t = 0; t < r; ++t) v -= Lm[(size_t)i * k + t] * Lm[(size_t)j * k + t];
      Lm[(size_t)i * k + r] = i == j ? ljj : v / ljj;
    }
    for (int i = 0; i < k; ++i)
      if (diag[i] >= 0.0 && i != j) diag[i] -= Lm[(size_t)i * k + r] * Lm[(size_t)i * k + r];
    diag[j] = -1.0;
    piv.push_back(j);
  }
  const int s = (int)piv.size();
  // Ls[r][c] = Lm[piv[r]][c], lower triangular; T[piv[r]][c] = inv(Ls)[c][r] / d[piv[r]]
  std::vector<double> inv((size_t)s * s, 0.0);
  for (int c = 0; c < s; ++c) {  // column c of inv(Ls) by forward substitution
    for (int r = 0; r < s; ++r) {
      double v = r == c ? 1.0 : 0.0;
      for (int t = c; t < r; ++t) v -= Lm[(size_t)piv[r] * k + t] * inv[(size_t)t * s + c];
      inv[(size_t)r * s + c] = r < c ? 0.0 : v / Lm[(size_t)piv[r] * k + r];
    }
  }
  T.assign((size_t)k * k, 0.0);
  for (int r = 0; r < s; ++r)
    for (int c = 0; c < s; ++c) T[(size_t)piv[r] * k + c] = inv[(size_t)c * s + r] / d[piv[r]];
  return s;
}

// Cholesky factor of the s x s SPD matrix W (row-major, leading dimension
// ldw) in place (lower triangle); false if a pivot is not positive.
inline bool cholesky(std::vector<double>& W, int s, int ldw) {
  for (int j = 0; j < s; ++j) {
    double v = W[(size_t)j * ldw + j];
    for (int t = 0; t < j; ++t) v -= W[(size_t)j * ldw + t] * W[(size_t)j * ldw + t];
    if (!(v > 0.0)) return false;
    const double ljj = std::sqrt(v);
    W[(size_t)j * ldw + j] = ljj;
    for (int i = j + 1; i < s; ++i) {
      double u = W[(size_t)i * ldw + j];
      for (int t = 0; t < j; ++t) u -= W[(size_t)i * ldw + t] * W[(size_t)j * ldw + t];
      W[(size_t)i * ldw + j] = u / ljj;
    }
  }
  return true;
}

// C (s x k, leading dimension k) <- scale * (L L^T)^{-1} C.
inline void chol_solve(const std::vector<double>& Lw, int s, int ldw, std::vector<double>& C, int k,
                double scale) {
  for (int i = 0; i < s; ++i) {  // L Y = C, row by row
    for (int t = 0; t < i; ++t) {
      const double l = Lw[(size_t)i * ldw + t];
      for (int j = 0; j < k; ++j) C[(size_t)i * k + j] -= l * C[(size_t)t * k + j];
    }
    const double l = Lw[(size_t)i * ldw + i];
    for (int j = 0; j < k; ++j) C[(size_t)i * k + j] /= l;
  }
  for (int i = s - 1; i >= 0; --i) {  // L^T X = Y
    for (int t = i + 1; t < s; ++t) {
      const double l = Lw[(size_t)t * ldw + i];
      for (int j = 0; j < k; ++j) C[(size_t)i * k + j] -= l * C[(size_t)t * k + j];
    }
    const double l = Lw[(size_t)i * ldw + i];
    for (int j = 0; j < k; ++j) C[(size_t)i * k + j] /= l;
  }
  if (scale != 1.0)
    for (auto& v : C) v *= scale;
}

}  // namespace dense
}  // namespace csc
