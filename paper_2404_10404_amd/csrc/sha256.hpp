// SHA-256 (FIPS 180-4) compression for the device and the host.
//
// The Fiat-Shamir transcript hashes only word-aligned messages: a 32-byte
// state, a four-byte tag and whole 32-byte field elements, so every message is
// assembled directly as big-endian 32-bit words. A field element (eight
// little-endian limbs) contributes the byte-swapped limbs in order.
#pragma once

#include <stdint.h>

#include "fr.hpp"

namespace gkr {

GKR_HD uint32_t rotr32(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }
// a ^ b ^ c: one three-input bit operation on gfx950 (truth table 0x96).
GKR_HD uint32_t xor3_32(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
#else
  return a ^ b ^ c;
#endif
}
// Majority of a, b, c: one three-input bit operation on gfx950 (truth table
// 0xE8: set where at least two inputs are).
GKR_HD uint32_t maj32(uint32_t a, uint32_t b, uint32_t c) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0xE8);
#else
  return (a & b) ^ (a & c) ^ (b & c);
#endif
}
GKR_HD uint32_t bswap32(uint32_t x) {
  return (x >> 24) | ((x >> 8) & 0xff00u) | ((x << 8) & 0xff0000u) | (x << 24);
}

#if defined(__HIP_DEVICE_COMPILE__)
#define GKR_SHA_TABLE static __constant__
#else
#define GKR_SHA_TABLE static const
#endif

GKR_SHA_TABLE uint32_t kSha256K[64] = {
    0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u, 0xab1c5ed5u,
    0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u,
    0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
    0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u,
    0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u,
    0xa2bfe8a1u, 0xa81a664bu, 0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
    0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
    0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u};

struct Sha256State {
  uint32_t h[8];
};

struct Sha256Block {
  uint32_t w[16];
};

GKR_HD Sha256State sha256_iv() {
  Sha256State s;
  s.h[0] = 0x6a09e667u; s.h[1] = 0xbb67ae85u; s.h[2] = 0x3c6ef372u; s.h[3] = 0xa54ff53au;
  s.h[4] = 0x510e527fu; s.h[5] = 0x9b05688cu; s.h[6] = 0x1f83d9abu; s.h[7] = 0x5be0cd19u;
  return s;
}

// One compression of a 16-word (big-endian) block into the chaining value.
// The 64 rounds run as four passes of 16 unrolled rounds over a rolling
// 16-word schedule, so each inlined copy stays small.
// On the device the working variables are pinned to vector registers: with
// wave-uniform inputs the compiler would otherwise split the rounds between
// the scalar unit and the vector unit (rotations), paying a register
// transfer per rotation.
GKR_HD Sha256State sha256_compress_v(Sha256State st, Sha256Block blk) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
  for (int k = 0; k < 8; ++k) asm volatile("" : "+v"(st.h[k]));
#pragma unroll
  for (int k = 0; k < 16; ++k) asm volatile("" : "+v"(blk.w[k]));
#endif
  uint32_t a = st.h[0], b = st.h[1], c = st.h[2], d = st.h[3];
  uint32_t e = st.h[4], f = st.h[5], g = st.h[6], h = st.h[7];
  for (int j = 0; j < 64; j += 16) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      uint32_t wi = blk.w[i];
      if (j > 0) {
        const uint32_t w15 = blk.w[(i + 1) & 15], w2 = blk.w[(i + 14) & 15];
        const uint32_t s0 = xor3_32(rotr32(w15, 7), rotr32(w15, 18), w15 >> 3);
        const uint32_t s1 = xor3_32(rotr32(w2, 17), rotr32(w2, 19), w2 >> 10);
        wi = blk.w[i] + s0 + blk.w[(i + 9) & 15] + s1;
        blk.w[i] = wi;
      }
      const uint32_t S1 = xor3_32(rotr32(e, 6), rotr32(e, 11), rotr32(e, 25));
      const uint32_t ch = (e & f) ^ (~e & g);
      const uint32_t t1 = h + S1 + ch + kSha256K[j + i] + wi;
      const uint32_t S0 = xor3_32(rotr32(a, 2), rotr32(a, 13), rotr32(a, 22));
      const uint32_t maj = maj32(a, b, c);
      const uint32_t t2 = S0 + maj;
      h = g; g = f; f = e; e = d + t1;
      d = c; c = b; b = a; a = t1 + t2;
    }
  }
  st.h[0] += a; st.h[1] += b; st.h[2] += c; st.h[3] += d;
  st.h[4] += e; st.h[5] += f; st.h[6] += g; st.h[7] += h;
  return st;
}

GKR_HD void sha256_compress(Sha256State& st, const uint32_t blk[16]) {
  Sha256Block b;
#pragma unroll
  for (int i = 0; i < 16; ++i) b.w[i] = blk[i];
  st = sha256_compress_v(st, b);
}

// A digest's bytes (big-endian words h[0..7]) read as a little-endian integer,
// masked to 254 bits: the candidate of one squeeze attempt, as canonical limbs.
GKR_HD Fr sha256_to_candidate(const Sha256State& d) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = bswap32(d.h[k]);
  r.v[7] &= 0x3fffffffu;
  return r;
}

}  // namespace gkr
