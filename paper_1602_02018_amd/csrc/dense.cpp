// Small dense float64 algebra of the block conjugate gradient (host code,
// built as plain C++ so that it can be compiled for several x86-64 vector
// extensions).  The matrices are at most k x k with k the number of clusters.
// Every routine uses row-major inner loops over contiguous, unaliased rows
// (no reductions), so the compiler vectorises them.
#include "dense.hpp"

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <thread>

namespace csc {
namespace dense {

// The routines below are built for the widest vector unit the host has
// (AVX-512, AVX2 or baseline x86-64, chosen when the library loads).  This
// file is compiled without floating-point contraction: a product and a
// difference are never fused, so every variant rounds the same.
#define CSC_DENSE_CLONES __attribute__((target_clones("avx512f", "avx2", "default")))

// y[0..n) -= a * x[0..n)
__attribute__((always_inline)) inline void sub_scaled(double* __restrict__ y,
                                                      const double* __restrict__ x, double a,
                                                      int n) {
  for (int j = 0; j < n; ++j) y[j] -= a * x[j];
}

// Rank-revealing orthonormalisation for the block CG: with G = Z^T Z (k x k,
// row-major), returns s and T (k x s, row-major, leading dimension k) such
// that P = Z T has orthonormal columns spanning the columns of Z.  Columns are
// first scaled to unit norm (so a small residual column is not mistaken for
// a dependent one); pivoted Cholesky of the scaled Gram (outer-product form:
// the trailing matrix is updated after each pivot) stops when the largest
// remaining pivot falls to rtol.
CSC_DENSE_CLONES int orth_transform(const std::vector<double>& G, int k, double rtol,
                                    std::vector<double>& T) {
  std::vector<double> d(k), A((size_t)k * k), Lc((size_t)k * k, 0.0), diag(k);
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
    // column r of the factor (row-indexed by the original column index), in Lc[r][.]
    double* lr = Lc.data() + (size_t)r * k;
    for (int i = 0; i < k; ++i) {
      const bool live = diag[i] >= 0.0 && i != j;
      lr[i] = i == j ? ljj : (live ? A[(size_t)i * k + j] / ljj : 0.0);
    }
    diag[j] = -1.0;
    for (int i = 0; i < k; ++i) {
      if (diag[i] < 0.0) continue;  // pivoted already, or a zero column
      sub_scaled(A.data() + (size_t)i * k, lr, lr[i], k);
      diag[i] -= lr[i] * lr[i];
    }
    piv.push_back(j);
  }
  const int s = (int)piv.size();
  // Ls[r][c] = Lc[c][piv[r]] (lower triangular); X = inv(Ls) row by row;
  // T[piv[r]][c] = X[c][r] / d[piv[r]]
  std::vector<double> X((size_t)s * s, 0.0);
  for (int r = 0; r < s; ++r) {
    double* xr = X.data() + (size_t)r * s;
    xr[r] = 1.0;
    for (int t = 0; t < r; ++t)
      sub_scaled(xr, X.data() + (size_t)t * s, Lc[(size_t)t * k + piv[r]], t + 1);
    const double l = Lc[(size_t)r * k + piv[r]];
    for (int c = 0; c <= r; ++c) xr[c] /= l;
  }
  T.assign((size_t)k * k, 0.0);
  for (int r = 0; r < s; ++r)
    for (int c = r; c < s; ++c) T[(size_t)piv[r] * k + c] = X[(size_t)c * s + r] / d[piv[r]];
  return s;
}

// Cholesky factor of the s x s SPD matrix W (row-major, leading dimension
// ldw) in place (lower triangle, outer-product form); false if a pivot is not
// positive.
CSC_DENSE_CLONES bool cholesky(std::vector<double>& W, int s, int ldw) {
  std::vector<double> col(s);
  for (int j = 0; j < s; ++j) {
    const double v = W[(size_t)j * ldw + j];
    if (!(v > 0.0)) return false;
    const double ljj = std::sqrt(v);
    W[(size_t)j * ldw + j] = ljj;
    for (int i = j + 1; i < s; ++i) col[i] = W[(size_t)i * ldw + j] /= ljj;
    // trailing update of the lower triangle: row i, columns j+1..i
    for (int i = j + 1; i < s; ++i)
      sub_scaled(W.data() + (size_t)i * ldw + j + 1, col.data() + j + 1, col[i], i - j);
  }
  return true;
}

// Columns [j0, j1) of C (s x k, leading dimension k) <- scale * (L L^T)^{-1} C.
CSC_DENSE_CLONES void solve_cols(const double* Lw, int s, int ldw, double* c, int k, int j0,
                                  int j1, double scale) {
  const int w = j1 - j0;
  for (int i = 0; i < s; ++i) {  // L Y = C, row by row
    double* ci = c + (size_t)i * k + j0;
    for (int t = 0; t < i; ++t) sub_scaled(ci, c + (size_t)t * k + j0, Lw[(size_t)i * ldw + t], w);
    const double l = Lw[(size_t)i * ldw + i];
    for (int j = 0; j < w; ++j) ci[j] /= l;
  }
  for (int i = s - 1; i >= 0; --i) {  // L^T X = Y
    double* ci = c + (size_t)i * k + j0;
    for (int t = i + 1; t < s; ++t) sub_scaled(ci, c + (size_t)t * k + j0, Lw[(size_t)t * ldw + i], w);
    const double l = Lw[(size_t)i * ldw + i];
    for (int j = 0; j < w; ++j) ci[j] /= l;
  }
  if (scale != 1.0)
    for (int i = 0; i < s; ++i)
      for (int j = 0; j < w; ++j) c[(size_t)i * k + j0 + j] *= scale;
}

void chol_solve(const std::vector<double>& Lw, int s, int ldw, std::vector<double>& C, int k,
                double scale, int threads) {
  int nt = 1;
  if (threads > 1 && (double)s * s * k >= (double)(1 << 22)) nt = std::min(threads, k / 32);
  if (nt <= 1) {
    solve_cols(Lw.data(), s, ldw, C.data(), k, 0, k, scale);
    return;
  }
  const int chunk = ((k + nt - 1) / nt + 7) / 8 * 8;  // slices of whole 64-byte lines
  std::vector<std::thread> pool;
  for (int j0 = chunk; j0 < k; j0 += chunk) {
    const int j1 = std::min(k, j0 + chunk);
    // a direct call from the lambda: the address of a multi-versioned
    // function is not a callable pointer in every compiler's shared objects
    try {
      pool.emplace_back([&Lw, &C, s, ldw, k, j0, j1, scale] {
        solve_cols(Lw.data(), s, ldw, C.data(), k, j0, j1, scale);
      });
    } catch (...) {  // no thread to be had: solve the slice here
      solve_cols(Lw.data(), s, ldw, C.data(), k, j0, j1, scale);
    }
  }
  solve_cols(Lw.data(), s, ldw, C.data(), k, 0, std::min(k, chunk), scale);
  for (auto& t : pool) t.join();
}

}  // namespace dense
}  // namespace csc
