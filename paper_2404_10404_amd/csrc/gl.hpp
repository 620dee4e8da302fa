// Goldilocks field arithmetic, p = 2^64 - 2^32 + 1 (Section 4.1, the field
// choice: the prover-fast alternative to BN254), for the device and the host.
//
// Elements are canonical 64-bit integers (< p); no Montgomery form. A product
// is a 64 x 64 -> 128-bit multiplication followed by the reduction that uses
// 2^64 = 2^32 - 1 and 2^96 = -1 (mod p): for x = hi * 2^64 + lo with
// hi = hh * 2^32 + hl, x = lo - hh + hl (2^32 - 1) (mod p).
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define GL_HD __host__ __device__ inline __attribute__((always_inline))
#else
#define GL_HD inline
#endif

namespace gkr {

constexpr uint64_t kGlP = 0xFFFFFFFF00000001ull;
constexpr uint64_t kGlEps = 0xFFFFFFFFull;          // 2^64 mod p = 2^32 - 1
constexpr uint64_t kGlHalf = 0x7FFFFFFF80000001ull;  // (p + 1) / 2, the inverse of 2

GL_HD uint64_t gl_add(uint64_t a, uint64_t b) {
  const uint64_t s = a + b;
  // a carry out of 64 bits means s + 2^64 = s + (2^32 - 1) (mod p), already below p
  const uint64_t r = (s < a) ? s + kGlEps : s;
  return r >= kGlP ? r - kGlP : r;
}

GL_HD uint64_t gl_sub(uint64_t a, uint64_t b) {
  const uint64_t d = a - b;
  // a borrow means d - 2^64 + p = d - (2^32 - 1), at least 1
  return (a < b) ? d - kGlEps : d;
}

GL_HD uint64_t gl_double(uint64_t a) { return gl_add(a, a); }

// a / 2: a >> 1 for even a, (a >> 1) + (p + 1) / 2 for odd a.
GL_HD uint64_t gl_half(uint64_t a) { return (a >> 1) + ((a & 1) ? kGlHalf : 0); }

// x = hi * 2^64 + lo reduced mod p.
GL_HD uint64_t gl_reduce128(uint64_t lo, uint64_t hi) {
  const uint64_t hh = hi >> 32, hl = hi & kGlEps;
  uint64_t t0 = lo - hh;
  if (lo < hh) t0 -= kGlEps;  // lo - hh + p
  const uint64_t t1 = (hl << 32) - hl;  // hl (2^32 - 1) < 2^64
  uint64_t r = t0 + t1;
  if (r < t1) r += kGlEps;  // carry: + 2^64 = + (2^32 - 1)
  return r >= kGlP ? r - kGlP : r;
}

GL_HD uint64_t gl_mul(uint64_t a, uint64_t b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return gl_reduce128(a * b, __umul64hi(a, b));
#else
  const unsigned __int128 x = (unsigned __int128)a * b;
  return gl_reduce128((uint64_t)x, (uint64_t)(x >> 64));
#endif
}

GL_HD uint64_t gl_one_minus(uint64_t a) { return gl_sub(1, a); }

// Value at r of the degree-2 polynomial with values e0, e1, e2 at t = 0, 1, 2:
// e0 + r (A + r B) with B = (e2 - 2 e1 + e0) / 2 and A = e1 - e0 - B.
GL_HD uint64_t gl_interp3(uint64_t e0, uint64_t e1, uint64_t e2, uint64_t r) {
  const uint64_t B = gl_half(gl_add(gl_sub(e2, gl_double(e1)), e0));
  const uint64_t A = gl_sub(gl_sub(e1, e0), B);
  return gl_add(e0, gl_mul(r, gl_add(A, gl_mul(r, B))));
}

}  // namespace gkr
