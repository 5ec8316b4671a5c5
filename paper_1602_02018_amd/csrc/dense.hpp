// Small dense float64 algebra of the block conjugate gradient, on the host
// (definitions in dense.cpp).  Matrices are row-major std::vectors of at most
// k x k entries, k the number of clusters.
#pragma once

#include <vector>

namespace csc {
namespace dense {

// Rank-revealing orthonormalisation for the block CG: with G = Z^T Z (k x k),
// returns s and T (k x s, leading dimension k) such that P = Z T has
// orthonormal columns spanning the columns of Z.  Columns are first scaled to
// unit norm (so a small residual column is not mistaken for a dependent one);
// pivoted Cholesky of the scaled Gram stops when the largest remaining pivot
// falls to rtol.
int orth_transform(const std::vector<double>& G, int k, double rtol, std::vector<double>& T);

// Cholesky factor of the s x s SPD matrix W (leading dimension ldw) in place
// (lower triangle); false if a pivot is not positive.
bool cholesky(std::vector<double>& W, int s, int ldw);

// C (s x k, leading dimension k) <- scale * (L L^T)^{-1} C, L the factor
// cholesky() left in Lw.  threads > 1 splits the k right-hand sides into
// column slices solved on that many host threads when the solve is large
// (s^2 k >= 2^22); every element takes the same operations either way.
void chol_solve(const std::vector<double>& Lw, int s, int ldw, std::vector<double>& C, int k,
                double scale, int threads = 1);

}  // namespace dense
}  // namespace csc
