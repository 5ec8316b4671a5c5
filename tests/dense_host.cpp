// C entry points over the host float64 algebra of the block CG, built by
// tests/test_dense_host.py with the system C++ compiler.
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
