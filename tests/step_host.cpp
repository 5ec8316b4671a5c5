// Host build of the step kernels' indexing, run under AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_host.py:
// * the gather loop (spmm_row_t, the sparse row product of every Chebyshev
//   step) on rows of every length around its loop boundaries, with each
//   array allocated to its exact size, so any read outside a row's CSR
//   segment or outside the gathered block stops the run; every result must
//   equal a plain CSR-order loop of fused multiply-adds bit for bit, as a
//   panel of four columns (lanes q of lpr) and as a single column;
// * the XCD work orders (work_unit): each one a bijection of [0, U);
// * the row walk (step_row): rows past n and schedule entries outside [0, n)
//   give -1.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "../paper_1602_02018_amd/csrc/device.hpp"

using csc::StepArgs;
using csc::dev::v4f;

static int failures = 0;
#define CHECK(c)                                                            \
  do {                                                                      \
    if (!(c)) {                                                             \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

// exact-size heap arrays (ASan guards both ends)
template <class T>
static std::unique_ptr<T[]> exact(size_t n) {
  return std::unique_ptr<T[]>(new T[n > 0 ? n : 1]);
}

static void gather_rows(unsigned seed) {
  std::mt19937 g(seed);
  const std::vector<int> lens = {0,  1,  2,  3,  4,  5,  7,  8,  9,  15, 16,  17,  31,  32,  33,
                                 63, 64, 65, 71, 72, 73, 79, 80, 81, 127, 128, 129, 200, 1999};
  const int n = 2100;  // columns of the graph (rows of the gathered block)
  const int rows = (int)lens.size();
  std::vector<int> rp_v(rows + 1, 0);
  for (int r = 0; r < rows; ++r) rp_v[r + 1] = rp_v[r] + lens[r];
  const int nnz = rp_v[rows];
  auto rp = exact<int>(rows + 1);
  auto col = exact<int>(nnz);
  auto val = exact<float>(nnz);
  std::memcpy(rp.get(), rp_v.data(), (rows + 1) * sizeof(int));
  std::uniform_int_distribution<int> J(0, n - 1);
  std::normal_distribution<float> N01;
  for (int k = 0; k < nnz; ++k) {
    col[k] = J(g);
    val[k] = N01(g);
  }
  StepArgs a;
  a.row_ptr = rp.get();
  a.col = col.get();
  a.val = val.get();
  for (int lpr : {1, 2, 16, 64}) {  // lanes per row: panel widths 4, 8, 64, 256
    const size_t nv = (size_t)n * lpr;
    std::unique_ptr<v4f[]> T4(new v4f[nv]);
    for (size_t e = 0; e < nv; ++e) T4[e] = v4f{N01(g), N01(g), N01(g), N01(g)};
    for (int r = 0; r < rows; ++r)
      for (int q = 0; q < lpr; ++q) {
        const v4f got = csc::dev::spmm_row_t<v4f>(a, T4.get(), r, q, lpr, true);
        for (int c = 0; c < 4; ++c) {
          float ref = 0.f;
          for (int k = rp[r]; k < rp[r + 1]; ++k) ref = std::fmaf(val[k], T4[(size_t)col[k] * lpr + q][c], ref);
          const float gc = got[c];
          CHECK(std::memcmp(&ref, &gc, sizeof(float)) == 0);
        }
      }
    const v4f none = csc::dev::spmm_row_t<v4f>(a, T4.get(), 0, 0, lpr, false);
    for (int c = 0; c < 4; ++c) CHECK(none[c] == 0.f);
  }
  auto x = exact<float>(n);  // a single column as an n-vector
  for (int j = 0; j < n; ++j) x[j] = N01(g);
  for (int r = 0; r < rows; ++r) {
    const float got = csc::dev::spmm_row_t<float>(a, x.get(), r, 0, 1, true);
    float ref = 0.f;
    for (int k = rp[r]; k < rp[r + 1]; ++k) ref = std::fmaf(val[k], x[col[k]], ref);
    CHECK(std::memcmp(&ref, &got, sizeof(float)) == 0);
  }
}

static void work_orders() {
  for (int P : {1, 2, 3, 8})
    for (int T : {1, 2, 7, 8, 9, 15, 16, 17, 100, 1001})
      for (int xcd : {0, 1, 2}) {
        const int U = P * T;
        std::vector<int> seen(U, 0);
        for (int b = 0; b < U; ++b) {
          const int u = csc::dev::work_unit(b, U, T, xcd);
          CHECK(u >= 0 && u < U);
          if (u >= 0 && u < U) ++seen[u];
        }
        for (int u = 0; u < U; ++u) CHECK(seen[u] == 1);
      }
}

static void row_walk() {
  const int n = 10;
  auto sched = exact<int>(n);
  for (int r = 0; r < n; ++r) sched[r] = n - 1 - r;
  sched[3] = n;   // invalid entries
  sched[4] = -5;
  StepArgs a;
  a.L.n = n;
  a.sched = nullptr;
  for (int r = 0; r < n; ++r) CHECK(csc::dev::step_row(a, r) == r);
  CHECK(csc::dev::step_row(a, n) == -1);
  a.sched = sched.get();
  CHECK(csc::dev::step_row(a, 0) == n - 1);
  CHECK(csc::dev::step_row(a, 3) == -1);
  CHECK(csc::dev::step_row(a, 4) == -1);
  CHECK(csc::dev::step_row(a, n + 7) == -1);
}

int main() {
  for (unsigned seed = 1; seed <= 3; ++seed) gather_rows(seed);
  work_orders();
  row_walk();
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("step host checks passed\n");
  return 0;
}
