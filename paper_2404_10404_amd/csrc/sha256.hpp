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
GKR_HD uint32_t bswap32(uint32_t x) {
  return (x >> 24) | ((x >> 8) & 0xff00u) | ((x << 8) & 0xff0000u) | (x << 24);
}

GKR_HD uint32_t sha256_k(int i) {
  switch (i) {
    case 0: return 0x428a2f98u; case 1: return 0x71374491u; case 2: return 0xb5c0fbcfu; case 3: return 0xe9b5dba5u;
    case 4: return 0x3956c25bu; case 5: return 0x59f111f1u; case 6: return 0x923f82a4u; case 7: return 0xab1c5ed5u;
    case 8: return 0xd807aa98u; case 9: return 0x12835b01u; case 10: return 0x243185beu; case 11: return 0x550c7dc3u;
    case 12: return 0x72be5d74u; case 13: return 0x80deb1feu; case 14: return 0x9bdc06a7u; case 15: return 0xc19bf174u;
    case 16: return 0xe49b69c1u; case 17: return 0xefbe4786u; case 18: return 0x0fc19dc6u; case 19: return 0x240ca1ccu;
    case 20: return 0x2de92c6fu; case 21: return 0x4a7484aau; case 22: return 0x5cb0a9dcu; case 23: return 0x76f988dau;
    case 24: return 0x983e5152u; case 25: return 0xa831c66du; case 26: return 0xb00327c8u; case 27: return 0xbf597fc7u;
    case 28: return 0xc6e00bf3u; case 29: return 0xd5a79147u; case 30: return 0x06ca6351u; case 31: return 0x14292967u;
    case 32: return 0x27b70a85u; case 33: return 0x2e1b2138u; case 34: return 0x4d2c6dfcu; case 35: return 0x53380d13u;
    case 36: return 0x650a7354u; case 37: return 0x766a0abbu; case 38: return 0x81c2c92eu; case 39: return 0x92722c85u;
    case 40: return 0xa2bfe8a1u; case 41: return 0xa81a664bu; case 42: return 0xc24b8b70u; case 43: return 0xc76c51a3u;
    case 44: return 0xd192e819u; case 45: return 0xd6990624u; case 46: return 0xf40e3585u; case 47: return 0x106aa070u;
    case 48: return 0x19a4c116u; case 49: return 0x1e376c08u; case 50: return 0x2748774cu; case 51: return 0x34b0bcb5u;
    case 52: return 0x391c0cb3u; case 53: return 0x4ed8aa4au; case 54: return 0x5b9cca4fu; case 55: return 0x682e6ff3u;
    case 56: return 0x748f82eeu; case 57: return 0x78a5636fu; case 58: return 0x84c87814u; case 59: return 0x8cc70208u;
    case 60: return 0x90befffau; case 61: return 0xa4506cebu; case 62: return 0xbef9a3f7u; default: return 0xc67178f2u;
  }
}

struct Sha256State {
  uint32_t h[8];
};

GKR_HD Sha256State sha256_iv() {
  Sha256State s;
  s.h[0] = 0x6a09e667u; s.h[1] = 0xbb67ae85u; s.h[2] = 0x3c6ef372u; s.h[3] = 0xa54ff53au;
  s.h[4] = 0x510e527fu; s.h[5] = 0x9b05688cu; s.h[6] = 0x1f83d9abu; s.h[7] = 0x5be0cd19u;
  return s;
}

// One compression of a 16-word (big-endian) block into the chaining value.
GKR_HD void sha256_compress(Sha256State& st, const uint32_t blk[16]) {
  uint32_t w[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) w[i] = blk[i];
  uint32_t a = st.h[0], b = st.h[1], c = st.h[2], d = st.h[3];
  uint32_t e = st.h[4], f = st.h[5], g = st.h[6], h = st.h[7];
#pragma unroll
  for (int i = 0; i < 64; ++i) {
    uint32_t wi;
    if (i < 16) {
      wi = w[i];
    } else {
      uint32_t w15 = w[(i - 15) & 15], w2 = w[(i - 2) & 15];
      uint32_t s0 = rotr32(w15, 7) ^ rotr32(w15, 18) ^ (w15 >> 3);
      uint32_t s1 = rotr32(w2, 17) ^ rotr32(w2, 19) ^ (w2 >> 10);
      wi = w[i & 15] + s0 + w[(i - 7) & 15] + s1;
      w[i & 15] = wi;
    }
    uint32_t S1 = rotr32(e, 6) ^ rotr32(e, 11) ^ rotr32(e, 25);
    uint32_t ch = (e & f) ^ (~e & g);
    uint32_t t1 = h + S1 + ch + sha256_k(i) + wi;
    uint32_t S0 = rotr32(a, 2) ^ rotr32(a, 13) ^ rotr32(a, 22);
    uint32_t maj = (a & b) ^ (a & c) ^ (b & c);
    uint32_t t2 = S0 + maj;
    h = g; g = f; f = e; e = d + t1;
    d = c; c = b; b = a; a = t1 + t2;
  }
  st.h[0] += a; st.h[1] += b; st.h[2] += c; st.h[3] += d;
  st.h[4] += e; st.h[5] += f; st.h[6] += g; st.h[7] += h;
}

// Streaming hasher over 32-bit big-endian words (messages are whole words).
struct Sha256Words {
  Sha256State st;
  uint32_t blk[16];
  uint32_t fill;    // words in blk
  uint64_t nwords;  // total words absorbed

  GKR_HD void init() {
    st = sha256_iv();
    fill = 0;
    nwords = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) blk[i] = 0;
  }
  GKR_HD void word(uint32_t w) {
    // Branch-free placement keeps blk in registers when fully unrolled by the caller.
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if ((uint32_t)i == fill) blk[i] = w;
    ++fill;
    ++nwords;
    if (fill == 16) {
      sha256_compress(st, blk);
      fill = 0;
    }
  }
  GKR_HD void element(const Fr& canonical) {
    for (int k = 0; k < 8; ++k) word(bswap32(canonical.v[k]));
  }
  GKR_HD void digest(const Sha256State& d) {
    for (int k = 0; k < 8; ++k) word(d.h[k]);
  }
  GKR_HD Sha256State finish() {
    uint64_t bits = nwords * 32;
    word(0x80000000u);
    while (fill != 14) word(0);
    word((uint32_t)(bits >> 32));
    word((uint32_t)bits);
    return st;
  }
};

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
