// BN254 scalar-field arithmetic for gfx950 and the host.
//
// The paper proves over BN254 (Section 4.1, choice of finite field). Elements
// live in Montgomery form x*R mod p with R = 2^256, as eight 32-bit limbs
// (little-endian). Products use coarsely integrated operand scanning (CIOS)
// Montgomery multiplication: 32x32->64 multiply-adds on the VALU (the work is
// a carry chain, not a dense float contraction, so MFMA does not apply).
// p < 2^254, so sums of two reduced values never overflow 256 bits and a
// CIOS result is below 2p before its final conditional subtraction.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define GKR_HD __host__ __device__ inline __attribute__((always_inline))
#else
#define GKR_HD inline
#endif

namespace gkr {

struct Fr {
  uint32_t v[8];
};

// p = 0x30644e72e131a029b85045b68181585d2833e84879b9709143e1f593f0000001
#define GKR_P0 0xf0000001u
#define GKR_P1 0x43e1f593u
#define GKR_P2 0x79b97091u
#define GKR_P3 0x2833e848u
#define GKR_P4 0x8181585du
#define GKR_P5 0xb85045b6u
#define GKR_P6 0xe131a029u
#define GKR_P7 0x30644e72u
#define GKR_NINV 0xefffffffu  // -p^{-1} mod 2^32

GKR_HD uint32_t p_limb(int k) {
  switch (k) {
    case 0: return GKR_P0;
    case 1: return GKR_P1;
    case 2: return GKR_P2;
    case 3: return GKR_P3;
    case 4: return GKR_P4;
    case 5: return GKR_P5;
    case 6: return GKR_P6;
    default: return GKR_P7;
  }
}

GKR_HD Fr fr_make(uint32_t a0, uint32_t a1, uint32_t a2, uint32_t a3, uint32_t a4, uint32_t a5,
                  uint32_t a6, uint32_t a7) {
  Fr r;
  r.v[0] = a0; r.v[1] = a1; r.v[2] = a2; r.v[3] = a3;
  r.v[4] = a4; r.v[5] = a5; r.v[6] = a6; r.v[7] = a7;
  return r;
}

GKR_HD Fr fr_zero() { return fr_make(0, 0, 0, 0, 0, 0, 0, 0); }
// R mod p: the Montgomery form of 1.
GKR_HD Fr fr_one() {
  return fr_make(0x4ffffffbu, 0xac96341cu, 0x9f60cd29u, 0x36fc7695u, 0x7879462eu, 0x666ea36fu,
                 0x9a07df2fu, 0x0e0a77c1u);
}
// R^2 mod p: multiplying a canonical value by it converts to Montgomery form.
GKR_HD Fr fr_r2() {
  return fr_make(0xae216da7u, 0x1bb8e645u, 0xe35c59e3u, 0x53fe3ab1u, 0x53bb8085u, 0x8c49833du,
                 0x7f4e44a5u, 0x0216d0b1u);
}
// Montgomery form of 1/2.
GKR_HD Fr fr_inv2() {
  return fr_make(0x1ffffffeu, 0x783c14d8u, 0x0c8d1eddu, 0xaf982f6fu, 0xfcfd4f45u, 0x8f5f7492u,
                 0x3d9cbfacu, 0x1f37631au);
}

// 32-bit add and subtract with carry. On the device these are the clang
// carry-chain builtins, one v_add_co/v_addc (v_sub_co/v_subb) per limb with
// the carry in VCC; on the host plain C.
GKR_HD uint32_t adc32(uint32_t a, uint32_t b, uint32_t cin, uint32_t& cout) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_addc(a, b, cin, &cout);
#else
  const uint64_t s = (uint64_t)a + b + cin;
  cout = (uint32_t)(s >> 32);
  return (uint32_t)s;
#endif
}
GKR_HD uint32_t sbb32(uint32_t a, uint32_t b, uint32_t bin, uint32_t& bout) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_subc(a, b, bin, &bout);
#else
  const uint64_t d = (uint64_t)a - b - bin;
  bout = (uint32_t)(d >> 63);
  return (uint32_t)d;
#endif
}

// a - p if a >= p, else a (a < 2p).
GKR_HD Fr fr_reduce_once(const Fr& a) {
  Fr t;
  uint32_t br = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) t.v[k] = sbb32(a.v[k], p_limb(k), br, br);
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = br ? a.v[k] : t.v[k];
  return r;
}

GKR_HD Fr fr_add(const Fr& a, const Fr& b) {
  Fr s;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s.v[k] = adc32(a.v[k], b.v[k], c, c);
  return fr_reduce_once(s);
}

// a - b; p is added back under a mask (no branch) when the difference borrows.
GKR_HD Fr fr_sub(const Fr& a, const Fr& b) {
  Fr d;
  uint32_t br = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) d.v[k] = sbb32(a.v[k], b.v[k], br, br);
  const uint32_t mask = 0u - br;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) d.v[k] = adc32(d.v[k], p_limb(k) & mask, c, c);
  return d;
}

// a / 2 (of a reduced value): a >> 1 when a is even, (a + p) >> 1 when odd
// (a + p < 2^255). Halving a Montgomery form halves the value it represents.
GKR_HD Fr fr_half(const Fr& a) {
  const uint32_t mask = 0u - (a.v[0] & 1u);
  Fr t;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) t.v[k] = adc32(a.v[k], p_limb(k) & mask, c, c);
  Fr r;
#pragma unroll
  for (int k = 0; k < 7; ++k) r.v[k] = (t.v[k] >> 1) | (t.v[k + 1] << 31);
  r.v[7] = t.v[7] >> 1;
  return r;
}

GKR_HD Fr fr_neg(const Fr& a) { return fr_sub(fr_zero(), a); }
GKR_HD Fr fr_double(const Fr& a) { return fr_add(a, a); }

#if defined(__HIP_DEVICE_COMPILE__)
// Column multiply-accumulate of product scanning: (ov:acc) += x * y, where the
// 64-bit add inside v_mad_u64_u32 reports its carry in VCC and v_addc folds it
// into the 32-bit overflow word. Two VALU instructions per 32x32 product.
__device__ __forceinline__ void fr_mac_vv(uint64_t& acc, uint32_t& ov, uint32_t x, uint32_t y) {
  asm volatile("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\tv_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
               : "+v"(acc), "+v"(ov)
               : "v"(x), "v"(y)
               : "vcc");
}
__device__ __forceinline__ void fr_mac_vs(uint64_t& acc, uint32_t& ov, uint32_t x, uint32_t y) {
  asm volatile("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\tv_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
               : "+v"(acc), "+v"(ov)
               : "v"(x), "s"(y)
               : "vcc");
}

// Montgomery product on the device: finely integrated product scanning (FIPS,
// Koc-Acar-Kaliski 1996). Column k of a*b and of m*p is summed into a 96-bit
// accumulator; m_k is chosen so the low word of column k vanishes.
__device__ __forceinline__ Fr fr_mul_device(const Fr& a, const Fr& b) {
  uint32_t m[8];
  Fr r;
  uint64_t acc = 0;
  uint32_t ov = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int j = 0; j < k; ++j) {
      fr_mac_vv(acc, ov, a.v[j], b.v[k - j]);
      fr_mac_vs(acc, ov, m[j], p_limb(k - j));
    }
    fr_mac_vv(acc, ov, a.v[k], b.v[0]);
    m[k] = (uint32_t)acc * GKR_NINV;
    fr_mac_vs(acc, ov, m[k], GKR_P0);
    acc = (acc >> 32) | ((uint64_t)ov << 32);
    ov = 0;
  }
#pragma unroll
  for (int k = 8; k < 15; ++k) {
#pragma unroll
    for (int j = k - 7; j < 8; ++j) {
      fr_mac_vv(acc, ov, a.v[j], b.v[k - j]);
      fr_mac_vs(acc, ov, m[j], p_limb(k - j));
    }
    r.v[k - 8] = (uint32_t)acc;
    acc = (acc >> 32) | ((uint64_t)ov << 32);
    ov = 0;
  }
  r.v[7] = (uint32_t)acc;
  return fr_reduce_once(r);
}
#else
// Host form of the column multiply-accumulate: (ov:acc) += x * y.
GKR_HD void fr_mac_vv(uint64_t& acc, uint32_t& ov, uint32_t x, uint32_t y) {
  const uint64_t s = acc + (uint64_t)x * y;
  ov += (s < acc) ? 1u : 0u;
  acc = s;
}
GKR_HD void fr_mac_vs(uint64_t& acc, uint32_t& ov, uint32_t x, uint32_t y) { fr_mac_vv(acc, ov, x, y); }
#endif

// Unreduced (lazy) products: a 512-bit accumulator of sums of products of
// reduced values, reduced once at the end. A product into the accumulator
// costs 64 multiply-adds instead of the 136 of a Montgomery product, so sums
// of products (dot products, a*b + c*d) pay for one reduction only.
struct FrWide {
  uint32_t w[16];
};

GKR_HD FrWide frw_zero() {
  FrWide A;
#pragma unroll
  for (int k = 0; k < 16; ++k) A.w[k] = 0;
  return A;
}

// A += a * b by product scanning. The carry between columns is below 2^35,
// so adding the accumulator's word to it cannot overflow 64 bits.
GKR_HD void frw_mac(FrWide& A, const Fr& a, const Fr& b) {
  uint64_t acc = 0;
  uint32_t ov = 0;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    acc += A.w[k];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = k - i;
      if (j >= 0 && j < 8) fr_mac_vv(acc, ov, a.v[i], b.v[j]);
    }
    A.w[k] = (uint32_t)acc;
    acc = (acc >> 32) | ((uint64_t)ov << 32);
    ov = 0;
  }
  A.w[15] += (uint32_t)acc;
}

// Column accumulator of a sum of products: column k (k < 15) holds
// sum_{i+j=k} a_i b_j over every product added, as a 64-bit sum with an
// overflow word. Adding a product costs exactly its 64 multiply-adds (no
// carry propagation between columns); carries are propagated once, when the
// accumulator becomes an FrWide. Up to 16 products of reduced values: a
// column then sums at most 128 terms below 2^64 (below 2^71).
struct FrCols {
  uint64_t c[15];
  uint32_t o[15];
};

GKR_HD FrCols frc_zero() {
  FrCols A;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    A.c[k] = 0;
    A.o[k] = 0;
  }
  return A;
}

GKR_HD void frc_mac(FrCols& A, const Fr& a, const Fr& b) {
#pragma unroll
  for (int i = 0; i < 8; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) fr_mac_vv(A.c[i + j], A.o[i + j], a.v[i], b.v[j]);
}

// The 512-bit value of the columns, carries propagated.
GKR_HD FrWide frc_wide(const FrCols& A) {
  FrWide W;
  uint64_t carry = 0;  // below 2^64 + 2^39 after every column: kept as carry + overflow
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    const uint64_t s = carry + A.c[k];
    const uint32_t top = A.o[k] + (s < carry ? 1u : 0u);
    W.w[k] = (uint32_t)s;
    carry = (s >> 32) | ((uint64_t)top << 32);
  }
  W.w[15] = (uint32_t)carry;
  return W;
}

// Montgomery reduction of an accumulator of at most `Terms` products of
// reduced values: returns A * R^{-1} mod p, reduced. With p/2^256 < 0.1895,
// A < Terms * p^2 gives a high half below 0.1895 * Terms * p; subtracting p
// from it until it is below p changes A by multiples of pR only, after which
// A < pR and the reduction of the low words leaves a value below 2p.
template <int Terms>
GKR_HD Fr frw_reduce(const FrWide& A) {
  static_assert(Terms >= 1 && Terms <= 16, "accumulator bound");
  constexpr int kSub = Terms <= 5 ? 0 : Terms <= 10 ? 1 : Terms <= 15 ? 2 : 3;
  Fr hi;
#pragma unroll
  for (int k = 0; k < 8; ++k) hi.v[k] = A.w[8 + k];
#pragma unroll
  for (int rep = 0; rep < kSub; ++rep) hi = fr_reduce_once(hi);
  uint32_t m[8];
  Fr r;
  uint64_t acc = 0;
  uint32_t ov = 0;
#pragma unroll
  for (int k = 0; k < 15; ++k) {
    acc += k < 8 ? A.w[k] : hi.v[k - 8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int i = k - j;
      if (j < k && i >= 1 && i < 8) fr_mac_vs(acc, ov, m[j], p_limb(i));
    }
    if (k < 8) {
      m[k] = (uint32_t)acc * GKR_NINV;
      fr_mac_vs(acc, ov, m[k], GKR_P0);
    } else {
      r.v[k - 8] = (uint32_t)acc;
    }
    acc = (acc >> 32) | ((uint64_t)ov << 32);
    ov = 0;
  }
  r.v[7] = (uint32_t)acc + hi.v[7];
  return fr_reduce_once(r);
}

// a*b + c*d with one reduction.
// Product scanning of both products and the Montgomery reduction in one
// pass (the FIPS schedule with two product terms per column): a*b + c*d <
// 2p^2 < pR, so the result is below 2p before the final subtraction; a
// column sums at most 24 terms below 2^64, well inside the 96-bit
// accumulator.
GKR_HD Fr fr_mul_add2(const Fr& a, const Fr& b, const Fr& c, const Fr& d) {
  uint32_t m[8];
  Fr r;
  uint64_t acc = 0;
  uint32_t ov = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
#pragma unroll
    for (int j = 0; j < k; ++j) {
      fr_mac_vv(acc, ov, a.v[j], b.v[k - j]);
      fr_mac_vv(acc, ov, c.v[j], d.v[k - j]);
      fr_mac_vs(acc, ov, m[j], p_limb(k - j));
    }
    fr_mac_vv(acc, ov, a.v[k], b.v[0]);
    fr_mac_vv(acc, ov, c.v[k], d.v[0]);
    m[k] = (uint32_t)acc * GKR_NINV;
    fr_mac_vs(acc, ov, m[k], GKR_P0);
    acc = (acc >> 32) | ((uint64_t)ov << 32);
    ov = 0;
  }
#pragma unroll
  for (int k = 8; k < 15; ++k) {
#pragma unroll
    for (int j = k - 7; j < 8; ++j) {
      fr_mac_vv(acc, ov, a.v[j], b.v[k - j]);
      fr_mac_vv(acc, ov, c.v[j], d.v[k - j]);
      fr_mac_vs(acc, ov, m[j], p_limb(k - j));
    }
    r.v[k - 8] = (uint32_t)acc;
    acc = (acc >> 32) | ((uint64_t)ov << 32);
    ov = 0;
  }
  r.v[7] = (uint32_t)acc;
  return fr_reduce_once(r);
}

// Montgomery product a*b*R^{-1} mod p. Host: coarsely integrated operand
// scanning (CIOS) in plain C; device: the product-scanning form above.
GKR_HD Fr fr_mul(const Fr& a, const Fr& b) {
#if defined(__HIP_DEVICE_COMPILE__)
  return fr_mul_device(a, b);
#else
  uint32_t t[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) t[k] = 0;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    uint64_t c = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint64_t s = (uint64_t)a.v[j] * b.v[i] + t[j] + c;
      t[j] = (uint32_t)s;
      c = s >> 32;
    }
    uint64_t s8 = (uint64_t)t[8] + c;
    t[8] = (uint32_t)s8;
    t[9] = (uint32_t)(s8 >> 32);
    uint32_t m = t[0] * GKR_NINV;
    uint64_t s = (uint64_t)m * GKR_P0 + t[0];
    c = s >> 32;
#pragma unroll
    for (int j = 1; j < 8; ++j) {
      s = (uint64_t)m * p_limb(j) + t[j] + c;
      t[j - 1] = (uint32_t)s;
      c = s >> 32;
    }
    s = (uint64_t)t[8] + c;
    t[7] = (uint32_t)s;
    t[8] = t[9] + (uint32_t)(s >> 32);
  }
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = t[k];
  return fr_reduce_once(r);
#endif
}

GKR_HD Fr fr_sqr(const Fr& a) { return fr_mul(a, a); }
GKR_HD Fr fr_to_mont(const Fr& a) { return fr_mul(a, fr_r2()); }
GKR_HD Fr fr_from_mont(const Fr& a) { return fr_mul(a, fr_make(1, 0, 0, 0, 0, 0, 0, 0)); }

GKR_HD bool fr_eq(const Fr& a, const Fr& b) {
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) d |= a.v[k] ^ b.v[k];
  return d == 0;
}

// True when the limbs hold a value below p.
GKR_HD bool fr_is_canonical(const Fr& a) {
  uint64_t br = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uint64_t d = (uint64_t)a.v[k] - p_limb(k) - br;
    br = d >> 63;
  }
  return br != 0;
}

// 1 - a (both Montgomery).
GKR_HD Fr fr_one_minus(const Fr& a) { return fr_sub(fr_one(), a); }

// Value at r of the degree-2 polynomial with values e0, e1, e2 at t = 0, 1, 2:
// g(r) = e0 + r (e1 - e0) + r (r - 1) / 2 * (e2 - 2 e1 + e0).
GKR_HD Fr fr_interp3(const Fr& e0, const Fr& e1, const Fr& e2, const Fr& r) {
  Fr d1 = fr_sub(e1, e0);
  Fr d2 = fr_add(fr_sub(e2, fr_double(e1)), e0);
  Fr rr = fr_mul(fr_mul(r, fr_sub(r, fr_one())), fr_inv2());
  return fr_add(fr_add(e0, fr_mul(r, d1)), fr_mul(rr, d2));
}

}  // namespace gkr
