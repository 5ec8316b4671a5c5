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

// Forward substitution, one register tile of RB rows x CB columns: rows
// i0 .. i0+RB-1, columns c0 .. c0+CB-1 of C (leading dimension ldc) become
//   (C[i] - sum_{t0 <= t < i} L[i][t] C[t]) / L[i][i],
// the subtractions taken one at a time in increasing t.  Rows t < i0 are
// final already; their products are shared by the tile's rows, which is what
// the tile saves (one load of C[t] per RB rows).
template <int RB, int CB>
__attribute__((always_inline)) inline void forward_tile(const double* __restrict__ L, int ldl,
                                                        double* __restrict__ c, int ldc, int i0,
                                                        int c0, int t0) {
  double acc[RB][CB];
  for (int r = 0; r < RB; ++r)
    for (int j = 0; j < CB; ++j) acc[r][j] = c[(size_t)(i0 + r) * ldc + c0 + j];
  for (int t = t0; t < i0; ++t) {
    const double* x = c + (size_t)t * ldc + c0;
    for (int r = 0; r < RB; ++r) {
      const double a = L[(size_t)(i0 + r) * ldl + t];
      for (int j = 0; j < CB; ++j) acc[r][j] -= a * x[j];
    }
  }
  for (int r = 0; r < RB; ++r) {
    for (int t = 0; t < r; ++t) {
      const double a = L[(size_t)(i0 + r) * ldl + i0 + t];
      for (int j = 0; j < CB; ++j) acc[r][j] -= a * acc[t][j];
    }
    const double l = L[(size_t)(i0 + r) * ldl + i0 + r];
    for (int j = 0; j < CB; ++j) acc[r][j] /= l;
  }
  for (int r = 0; r < RB; ++r)
    for (int j = 0; j < CB; ++j) c[(size_t)(i0 + r) * ldc + c0 + j] = acc[r][j];
}

constexpr int kRB = 6;  // forward tile rows: 6 x 16 columns keep 12 of the 32 AVX-512 registers

// Forward substitution of columns c0 .. c0+CB-1 over every row, in tiles of kRB rows.
template <int CB>
__attribute__((always_inline)) inline void forward_block(const double* L, int s, int ldl, double* c,
                                                         int ldc, int c0, bool unit_lower) {
  const int i_begin = unit_lower ? std::min(c0, s) : 0;
  int i0 = i_begin;
  for (; i0 + kRB <= s; i0 += kRB) forward_tile<kRB, CB>(L, ldl, c, ldc, i0, c0, i_begin);
  for (; i0 < s; ++i0) forward_tile<1, CB>(L, ldl, c, ldc, i0, c0, i_begin);
}

// C (s x w, leading dimension ldc) <- L^{-1} C for the lower-triangular L (s x s, leading
// dimension ldl): every element (i, c) is C[i][c] minus L[i][t] C[t][c] for t = 0, 1, ..., i-1
// in turn, then divided by L[i][i].  Columns go in blocks of 16, then 8, 4 and 1.
// unit_lower: C starts as the identity (s = w), so a column block starting at c0 is zero above
// row c0 and the rows t < c0 add nothing to it; the block then starts at row c0 (the zero
// entries it does subtract leave every value as it was: C holds no negative zeros).
CSC_DENSE_CLONES void forward_cols(const double* L, int s, int ldl, double* c, int ldc, int w,
                                   bool unit_lower) {
  int c0 = 0;
  for (; c0 + 16 <= w; c0 += 16) forward_block<16>(L, s, ldl, c, ldc, c0, unit_lower);
  if (c0 + 8 <= w) {
    forward_block<8>(L, s, ldl, c, ldc, c0, unit_lower);
    c0 += 8;
  }
  if (c0 + 4 <= w) {
    forward_block<4>(L, s, ldl, c, ldc, c0, unit_lower);
    c0 += 4;
  }
  for (; c0 < w; ++c0) forward_block<1>(L, s, ldl, c, ldc, c0, unit_lower);
}

constexpr int kGB = 32;  // orth_transform's column block (doubles)

// out[0..kGB) = y0[0..kGB) - sum_t a[t] x[t * ldx + 0..kGB), subtracted in increasing t
__attribute__((always_inline)) inline void block_gemv(double* out, const double* y0,
                                                      const double* __restrict__ x, size_t ldx,
                                                      const double* __restrict__ a, int nt) {
  double acc[kGB];
  for (int j = 0; j < kGB; ++j) acc[j] = y0[j];
  for (int t = 0; t < nt; ++t) {
    const double s = a[t];
    const double* xt = x + (size_t)t * ldx;
    for (int j = 0; j < kGB; ++j) acc[j] -= s * xt[j];
  }
  for (int j = 0; j < kGB; ++j) out[j] = acc[j];
}

// Rank-revealing orthonormalisation for the block CG: with G = Z^T Z (k x k,
// row-major), returns s and T (k x s, row-major, leading dimension k) such
// that P = Z T has orthonormal columns spanning the columns of Z.  Columns are
// first scaled to unit norm (so a small residual column is not mistaken for
// a dependent one); pivoted Cholesky of the scaled Gram A stops when the
// largest remaining pivot falls to rtol.  Each step pivots on the largest
// remaining diagonal entry (the lowest index among equals); a column whose
// remaining diagonal entry is negative is dependent and leaves the search.
// The factor is formed column by column (left-looking): step r needs only
// the pivot's column of the updated A, i.e. A[i][j] minus l_t[i] l_t[j] for
// the earlier factor columns t = 0 .. r-1 in turn, over the columns still in
// the search, which sit compacted in positions 0 .. m-1 (dependent ones are
// squeezed out once 16 have gathered).
CSC_DENSE_CLONES int orth_transform(const std::vector<double>& G, int k, double rtol,
                                    std::vector<double>& T) {
  const size_t ld = (size_t)(k + kGB - 1) / kGB * kGB;
  std::vector<double> d(k), diag(k);
  std::vector<int> perm, pos(k, -1), keep(k);
  for (int i = 0; i < k; ++i) {
    const double g = G[(size_t)i * k + i];
    d[i] = g > 0.0 ? std::sqrt(g) : 0.0;
    diag[i] = d[i] > 0.0 ? g / (d[i] * d[i]) : -1.0;
    if (diag[i] >= 0.0) {
      pos[i] = (int)perm.size();
      perm.push_back(i);
    }
  }
  int m = (int)perm.size(), ndead = 0;
  // Lp[t][p]: factor column t at position p; Ls: the factor's rows in pivot order
  std::vector<double> Lp((size_t)k * ld, 0.0), Ls((size_t)k * k, 0.0), a(k), col0(ld, 0.0),
      col(ld);
  // At[j][i] = A[i][j] = G[i][j] / (d[i] d[j]) (read for columns i, j both in the search):
  // the scaled rows, then their transpose in 16 x 16 blocks
  std::vector<double> A((size_t)k * k), At((size_t)k * k);
  for (int i = 0; i < k; ++i) {
    const double* g = G.data() + (size_t)i * k;
    double* a = A.data() + (size_t)i * k;
    const double di = d[i];
    for (int j = 0; j < k; ++j) a[j] = g[j] / (di * d[j]);
  }
  for (int i0 = 0; i0 < k; i0 += 16)
    for (int j0 = 0; j0 < k; j0 += 16)
      for (int j = j0; j < std::min(k, j0 + 16); ++j)
        for (int i = i0; i < std::min(k, i0 + 16); ++i) At[(size_t)j * k + i] = A[(size_t)i * k + j];
  std::vector<int> piv;
  for (int r = 0; r < k; ++r) {
    // pivot: the lowest index holding the largest diagonal entry (NaN entries never win;
    // nothing beats a NaN at index 0, which ends the factorisation)
    int j = 0;
    if (!std::isnan(diag[0])) {
      double mx[8];
      for (int l = 0; l < 8; ++l) mx[l] = diag[0];
      int i = 1;
      for (; i + 8 <= k; i += 8)
        for (int l = 0; l < 8; ++l) mx[l] = diag[i + l] > mx[l] ? diag[i + l] : mx[l];
      for (; i < k; ++i) mx[0] = diag[i] > mx[0] ? diag[i] : mx[0];
      double best = mx[0];
      for (int l = 1; l < 8; ++l) best = mx[l] > best ? mx[l] : best;
      while (!(diag[j] == best)) ++j;
    }
    if (!(diag[j] > rtol)) break;
    const double ljj = std::sqrt(diag[j]);
    const int pj = pos[j];
    for (int t = 0; t < r; ++t) a[t] = Lp[(size_t)t * ld + pj];
    std::copy(a.begin(), a.begin() + r, Ls.begin() + (size_t)r * k);
    Ls[(size_t)r * k + r] = ljj;
    const double* atj = At.data() + (size_t)j * k;
    for (int p = 0; p < m; ++p) col0[p] = atj[perm[p]];
    for (int p0 = 0; p0 < m; p0 += kGB)
      block_gemv(col.data() + p0, col0.data() + p0, Lp.data() + p0, ld, a.data(), r);
    double* lr = Lp.data() + (size_t)r * ld;
    diag[j] = -1.0;
    for (int p = 0; p < m; ++p) {
      const int i = perm[p];
      if (!(diag[i] >= 0.0)) {  // the pivot, or out of the search already
        lr[p] = p == pj ? ljj : 0.0;
        continue;
      }
      lr[p] = col[p] / ljj;
      diag[i] -= lr[p] * lr[p];
      if (!(diag[i] >= 0.0)) ++ndead;
    }
    piv.push_back(j);
    if (++ndead >= 16) {  // squeeze the columns out of the search out of the positions
      int q = 0;
      for (int p = 0; p < m; ++p) {
        const int i = perm[p];
        if (!(diag[i] >= 0.0)) {
          pos[i] = -1;
          continue;
        }
        keep[q] = p;
        perm[q] = i;
        pos[i] = q++;
      }
      for (int t = 0; t <= r; ++t) {  // keep[q] >= q, increasing: in place, row by row
        double* row = Lp.data() + (size_t)t * ld;
        for (int u = 0; u < q; ++u) row[u] = row[keep[u]];
      }
      m = q;
      ndead = 0;
    }
  }
  const int s = (int)piv.size();
  // X = Ls^{-1} (row r of Ls: Ls[r][t] = l_t[piv[r]]); T[piv[r]][c] = X[c][r] / d[piv[r]]
  const int lx = std::max(1, s);
  std::vector<double> X((size_t)s * lx, 0.0);
  for (int r = 0; r < s; ++r) X[(size_t)r * lx + r] = 1.0;
  forward_cols(Ls.data(), s, k, X.data(), lx, s, /*unit_lower=*/true);
  T.assign((size_t)k * k, 0.0);
  for (int r = 0; r < s; ++r)
    for (int c = r; c < s; ++c) T[(size_t)piv[r] * k + c] = X[(size_t)c * lx + r] / d[piv[r]];
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
  forward_cols(Lw, s, ldw, c + j0, k, w, false);  // L Y = C
  for (int i = s - 1; i >= 0; --i) {              // L^T X = Y, row by row
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
