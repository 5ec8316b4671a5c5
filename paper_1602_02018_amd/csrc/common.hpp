// Internal declarations shared by the libcsc translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/csc.h"

namespace csc {

// ---------------------------------------------------------------- errors ---
void set_error(const std::string& msg);
void clear_error();

#define CSC_HIP(call)                                                               \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::csc::set_error(std::string(#call " failed: ") + hipGetErrorString(e_));     \
      return CSC_E_HIP;                                                             \
    }                                                                               \
  } while (0)

#define CSC_REQUIRE(cond, msg)                                                      \
  do {                                                                              \
    if (!(cond)) {                                                                  \
      ::csc::set_error(msg);                                                        \
      return CSC_E_INVALID_ARG;                                                     \
    }                                                                               \
  } while (0)

#define CSC_TRY(expr)                                                               \
  do {                                                                              \
    csc_status s_ = (expr);                                                         \
    if (s_ != CSC_OK) return s_;                                                    \
  } while (0)

// --------------------------------------------------- Philox4x64-10 -------
// Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3"
// (SC'11): ten rounds of two 64x64->128-bit products on a 4-word counter,
// with the 2-word key bumped by Weyl constants between rounds.
constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

struct Words4 {
  uint64_t x0, x1, x2, x3;
};

__host__ __device__ inline uint64_t mul_hi64(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __umul64hi(a, b);
#else
  return (uint64_t)(((unsigned __int128)a * (unsigned __int128)b) >> 64);
#endif
}

__host__ __device__ inline Words4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                                uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = mul_hi64(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = mul_hi64(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return Words4{c0, c1, c2, c3};
}

// ------------------------------------------------ internal block layout ---
// Dense blocks inside the library are stored panel-major: the w columns are
// padded to P panels of PW columns, panel q holds an N x PW node-major slab,
// element (i, c) lives at base[(c / PW) * N * PW + i * PW + c % PW].  A
// Chebyshev step gathers rows of one panel at a time, so the rows gathered by
// concurrently running workgroups come from a slab of N*PW*4 bytes, which is
// what the caches have to hold.  Padding columns are kept at zero.
struct Layout {
  int n = 0;   // rows
  int w = 0;   // logical columns
  int pw = 8;  // panel width (4, 8, 16, 32 or 64)
  int np = 0;  // number of panels
  __host__ __device__ size_t panel_elems() const { return (size_t)n * pw; }
  __host__ __device__ size_t elems() const { return panel_elems() * np; }
  __host__ __device__ size_t bytes() const { return elems() * sizeof(float); }
};

Layout make_layout(int n, int w, int pw);
int choose_panel_width(int n, int w, long long nnz);
size_t align_up(size_t x, size_t a = 256);

// Bump allocator over a caller workspace.
struct Arena {
  char* base;
  size_t cap;
  size_t off = 0;
  Arena(void* b, size_t c) : base((char*)b), cap(c) {}
  template <class T>
  T* take(size_t count) {
    off = align_up(off);
    T* p = (T*)(base + off);
    off += count * sizeof(T);
    return p;
  }
  bool ok() const { return off <= cap; }
};

}  // namespace csc
