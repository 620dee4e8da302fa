// Step bodies of the GKR prover kernels (device code, included by the plain
// kernels and by the persistent batch kernel).
//
// Grid-wide bodies run with 256-thread workgroups (four 64-wide waves); the
// single-workgroup tails take any multiple of 64 threads from 128 to 1024
// (512 in the plain kernels, 256 in the batch kernel). Field
// elements are 32-byte records in Montgomery form, loaded and stored as two
// 16-byte vectors, so consecutive threads touch consecutive records and every
// access of a table sweep is coalesced. Gate g = z*2^n + c keeps the copy
// index in the low bits: a gather W[(y_z << n) | c] over consecutive c is
// contiguous.
//
// A body works over (tile, ntiles): tile plays the role of the workgroup index
// and ntiles of the grid size. The plain path launches one kernel per step
// with grid = ntiles; the persistent batch kernel hands tiles of many proofs'
// steps to resident workgroups.
//
// Reductions over a whole table (the round polynomials of the sumcheck) end in
// the last tile to finish: each tile writes its partial sums and publishes
// them with a device-scope release increment of an atomic counter; the tile
// that brings the counter to ntiles acquires, adds the partials and runs the
// round's Fiat-Shamir step: its first wave hashes the sums and takes the
// challenge, its second wave moves the claim through the previous round
// (the products by r stay off the chain of hashes).
// Challenges and claims never leave device memory, so a proof is a plain
// sequence of launches on one stream.
#pragma once

#include "gkr_device.hpp"
#include "gkr_kernels.hpp"

namespace gkr {


// ---------------------------------------------------------- transcript

// SHA-256 of a fixed-length word message (big-endian words).
template <int L>
__device__ __forceinline__ Sha256State sha256_fixed(const uint32_t* w) {
  constexpr int B = (L + 3 + 15) / 16;
  Sha256State st = sha256_iv();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    Sha256Block blk;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int idx = b * 16 + i;
      uint32_t v;
      if (idx < L) v = w[idx];
      else if (idx == L) v = 0x80000000u;
      else if (idx == B * 16 - 1) v = (uint32_t)(L * 32);
      else v = 0u;
      blk.w[i] = v;
    }
    st = sha256_compress_v(st, blk);
  }
  return st;
}

__device__ __forceinline__ Sha256State load_state(const DevState* S) {
  Sha256State s;
#pragma unroll
  for (int k = 0; k < 8; ++k) s.h[k] = S->st[k];
  return s;
}

__device__ __forceinline__ void save_state(DevState* S, const Sha256State& s) {
#pragma unroll
  for (int k = 0; k < 8; ++k) S->st[k] = s.h[k];
}

// The current state as a challenge: rehash with "GKRC" until the 254-bit
// little-endian value v is below p. The challenge is v * 2^-256 mod p, so v
// itself is its Montgomery form: the limbs returned are used as is. Each
// attempt is accepted with probability p / 2^254 > 3/4; the bound on
// attempts only guarantees termination.
__device__ Fr accept(Sha256State& st) {
  Fr c = sha256_to_candidate(st);
  for (int attempt = 0; attempt < 4096 && !fr_is_canonical(c); ++attempt) {
    uint32_t w[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = st.h[k];
    w[8] = kTagChallenge;
    st = sha256_fixed<9>(w);
    c = sha256_to_candidate(st);
  }
  return c;
}

__device__ Fr squeeze(Sha256State& st) {
  uint32_t w[9];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = kTagChallenge;
  st = sha256_fixed<9>(w);
  return accept(st);
}

__device__ void absorb_element(Sha256State& st, uint32_t tag, const Fr& canonical) {
  uint32_t w[17];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = tag;
#pragma unroll
  for (int k = 0; k < 8; ++k) w[9 + k] = bswap32(canonical.v[k]);
  st = sha256_fixed<17>(w);
}

__device__ void absorb_digest(Sha256State& st, const uint32_t* d) {
  uint32_t w[17];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = kTagDigest;
#pragma unroll
  for (int k = 0; k < 8; ++k) w[9 + k] = d[k];
  st = sha256_fixed<17>(w);
}

__device__ __forceinline__ Fr fr_one_canonical() { return fr_make(1, 0, 0, 0, 0, 0, 0, 0); }

// The value of lane `src` (a constant) in every lane of the wave.
__device__ __forceinline__ Fr lane_fr(const Fr& a, int src) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = (uint32_t)__builtin_amdgcn_readlane((int)a.v[k], src);
  return r;
}

// The transcript half of a round, on a transcript state held in registers
// (the same in every lane of the wave): one SHA-256 compression absorbs the
// Montgomery forms of the round's sums e0 and e2, and the accepted hash value
// is the challenge r in Montgomery form. No product precedes the hash, and
// the running claim is not needed (e1 enters only the message).
__device__ __forceinline__ Fr round_hash_wave(Sha256State& state, const Fr& e0, const Fr& e2) {
  Sha256Block blk;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    blk.w[k] = bswap32(e0.v[k]);
    blk.w[8 + k] = bswap32(k == 7 ? (e2.v[k] | kRoundMark) : e2.v[k]);
  }
  state = sha256_compress_v(state, blk);
  return accept(state);
}

// The product half: the next claim g(r) = e0 + r (e1 - e0) + r (r - 1)
// (e2 - 2 e1 + e0) / 2, evaluated as e0 + r (A + r B) with B = (e2 - 2 e1 +
// e0) / 2 and A = e1 - e0 - B, and the message (e0, e1, e2, canonical) stored
// by lanes 1..3 (one element each) to msg_out. The products run in different
// lanes: two rounds of products, both in every lane of the wave.
__device__ __forceinline__ Fr round_claim_wave(const Fr& r, const Fr& e0, const Fr& e1, const Fr& e2,
                                               uint32_t* msg_out) {
  const int lane = threadIdx.x & 63;
  const Fr B = fr_half(fr_add(fr_sub(e2, fr_double(e1)), e0));
  const Fr A = fr_sub(fr_sub(e1, e0), B);
  // lane 0: r B; lanes 1..3: canonical e0, e1, e2 (register selects over
  // opaque candidates: no private array for the optimizer to index)
  Fr c1 = e0, c2 = e1, c3 = e2, one = fr_one_canonical();
#pragma unroll
  for (int k = 0; k < 8; ++k) asm volatile("" : "+v"(c1.v[k]), "+v"(c2.v[k]), "+v"(c3.v[k]), "+v"(one.v[k]));
  Fr a = r, b = B;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    a.v[k] = lane == 1 ? c1.v[k] : (lane == 2 ? c2.v[k] : (lane == 3 ? c3.v[k] : a.v[k]));
    b.v[k] = lane == 0 ? b.v[k] : one.v[k];
  }
  const Fr prod = fr_mul(a, b);
  if (lane >= 1 && lane <= 3) stf(reinterpret_cast<Fr*>(msg_out), lane - 1, prod);
  const Fr t = fr_mul(r, fr_add(A, lane_fr(prod, 0)));
  return fr_add(e0, t);
}

// A phase's final value (one thread): store it, write it to the proof and absorb it.
__device__ __forceinline__ void finish_value(DevState* S, const Fr& v, Fr* v_out, uint32_t* proof_out) {
  const Fr c = fr_from_mont(v);
  Sha256State st = load_state(S);
  absorb_element(st, kTagValue, c);
  save_state(S, st);
  *v_out = v;
#pragma unroll
  for (int k = 0; k < 8; ++k) proof_out[k] = c.v[k];
}

// ---------------------------------------------------------------- bodies

#define GTID ((uint64_t)tile * kBlock + threadIdx.x)
#define GSTRIDE ((uint64_t)ntiles * kBlock)

// ST_TO_MONT: p0 canonical in, p1 out, q0 count.
__device__ __forceinline__ void body_to_mont(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* in = P<const Fr*>(st, 0);
  Fr* out = P<Fr*>(st, 1);
  for (uint64_t i = GTID; i < st.q[0]; i += GSTRIDE) stf(out, i, fr_to_mont(ldf(in, i)));
}

// ST_FROM_MONT: p0 in, p1 canonical out, q0 count.
__device__ __forceinline__ void body_from_mont(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* in = P<const Fr*>(st, 0);
  Fr* out = P<Fr*>(st, 1);
  for (uint64_t i = GTID; i < st.q[0]; i += GSTRIDE) stf(out, i, fr_from_mont(ldf(in, i)));
}

// ST_FORWARD: V_i[z*2^n + c] = W[x_z*2^n + c] (+ or *) W[y_z*2^n + c].
// p0 W, p1 V, p2 gate records, u0 n, q0 count.
__device__ __forceinline__ void body_forward(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ W = P<const Fr*>(st, 0);
  Fr* __restrict__ V = P<Fr*>(st, 1);
  const uint2* __restrict__ gates = P<const uint2*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t g = GTID; g < st.q[0]; g += GSTRIDE) {
    const uint64_t z = g >> n, c = g & mask;
    const uint2 gate = gates[z];
    const uint64_t x = gate.x & 0x7fffffffu, y = gate.y;
    const Fr a = ldf(W, (x << n) | c), b = ldf(W, (y << n) | c);
    stf(V, g, (gate.x >> 31) ? fr_mul(a, b) : fr_add(a, b));
  }
}

// ST_DIGEST: one level of a tree digest; chunk t of q0 words (256 words, 1 KiB,
// per chunk) is hashed by thread t; element words are byte-swapped (limbs are
// little-endian). p0 in, p1 out, q0 nwords, q1 nchunks, u0 swap.
__device__ __forceinline__ void body_digest(const Step& st, uint32_t tile, uint32_t ntiles) {
  const uint32_t* __restrict__ in = P<const uint32_t*>(st, 0);
  uint32_t* __restrict__ out = P<uint32_t*>(st, 1);
  const uint64_t nwords = st.q[0];
  const int swap = st.u[0];
  for (uint64_t t = GTID; t < st.q[1]; t += GSTRIDE) {
    const uint64_t begin = t * kChunkWords;
    const uint64_t end = (begin + kChunkWords < nwords) ? begin + kChunkWords : nwords;
    const uint64_t len = end - begin;  // a multiple of 8 words
    Sha256State sh = sha256_iv();
    const uint4* src = reinterpret_cast<const uint4*>(in + begin);
    const uint64_t full = len / 16;
    for (uint64_t b = 0; b < full; ++b) {
      Sha256Block blk;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const uint4 v = src[b * 4 + q];
        blk.w[4 * q + 0] = swap ? bswap32(v.x) : v.x;
        blk.w[4 * q + 1] = swap ? bswap32(v.y) : v.y;
        blk.w[4 * q + 2] = swap ? bswap32(v.z) : v.z;
        blk.w[4 * q + 3] = swap ? bswap32(v.w) : v.w;
      }
      sh = sha256_compress_v(sh, blk);
    }
    Sha256Block blk;
#pragma unroll
    for (int i = 0; i < 16; ++i) blk.w[i] = 0;
    if (len - full * 16 == 8) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const uint4 v = src[full * 4 + q];
        blk.w[4 * q + 0] = swap ? bswap32(v.x) : v.x;
        blk.w[4 * q + 1] = swap ? bswap32(v.y) : v.y;
        blk.w[4 * q + 2] = swap ? bswap32(v.z) : v.z;
        blk.w[4 * q + 3] = swap ? bswap32(v.w) : v.w;
      }
      blk.w[8] = 0x80000000u;
    } else {
      blk.w[0] = 0x80000000u;
    }
    const uint64_t bits = len * 32;
    blk.w[14] = (uint32_t)(bits >> 32);
    blk.w[15] = (uint32_t)bits;
    sh = sha256_compress_v(sh, blk);
#pragma unroll
    for (int k = 0; k < 8; ++k) out[t * 8 + k] = sh.h[k];
  }
}

// ST_TRANSCRIPT_BEGIN: st = seed state (w0..7), then absorb the circuit digest
// (w8..15) and the two vector digests; also zeroes the reduction counter and
// clears the pending round.
// p0 S, p1 dig_in, p2 dig_out.
__device__ __forceinline__ void body_transcript_begin(const Step& st, uint32_t, uint32_t) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  Sha256State sh;
#pragma unroll
  for (int k = 0; k < 8; ++k) sh.h[k] = st.w[k];
  absorb_digest(sh, st.w + 8);
  absorb_digest(sh, P<const uint32_t*>(st, 1));
  absorb_digest(sh, P<const uint32_t*>(st, 2));
  save_state(S, sh);
  S->counter = 0;
  S->pending = 0;
}

// ST_SQUEEZE: u0 challenges into p1 (Montgomery form). p0 S.
__device__ __forceinline__ void body_squeeze(const Step& st, uint32_t, uint32_t) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  Fr* out = P<Fr*>(st, 1);
  Sha256State sh = load_state(S);
  for (uint32_t k = 0; k < st.u[0]; ++k) stf(out, k, squeeze(sh));
  save_state(S, sh);
}

// ST_LAYER_BEGIN: draw alpha, beta (layer > 0) and set the claim to
// alpha * vu + beta * vv; on layer 0 (u0 = 1) alpha = 1, beta = 0 and claim = vu.
// p0 S, p1 vu, p2 vv.
__device__ __forceinline__ void body_layer_begin(const Step& st, uint32_t, uint32_t) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  const Fr vu = *P<const Fr*>(st, 1), vv = *P<const Fr*>(st, 2);
  if (st.u[0]) {
    S->alpha = fr_one();
    S->beta = fr_zero();
    S->claim = vu;
    return;
  }
  Sha256State sh = load_state(S);
  const Fr a = squeeze(sh);
  const Fr b = squeeze(sh);
  save_state(S, sh);
  S->alpha = a;
  S->beta = b;
  S->claim = fr_mul_add2(a, vu, b, vv);
}

// ST_EQ: up to four tables out_j[b] = scale_j * prod_k (bit_k(b) ? r_k : 1 - r_k),
// bit 1 = MSB. u0..3 bits, u4 count; p0..3 points, p4..7 scales (null = 1), p8..11 outs.
__device__ __forceinline__ void body_eq(const Step& st, uint32_t tile, uint32_t ntiles) {
  uint64_t total = 0;
  for (uint32_t j = 0; j < st.u[4]; ++j) total += 1ull << st.u[j];
  for (uint64_t g = GTID; g < total; g += GSTRIDE) {
    uint64_t t = g;
    uint32_t j = 0;
    while (t >= (1ull << st.u[j])) {
      t -= 1ull << st.u[j];
      ++j;
    }
    const Fr* r = P<const Fr*>(st, j);
    const int k = st.u[j];
    const Fr* scale = P<const Fr*>(st, 4 + j);
    // the k factors in four independent chains (variable i in chain i mod 4),
    // multiplied together at the end: a dependent chain of about k/4 + 2 products
    Fr acc[4] = {scale ? *scale : fr_one(), fr_one(), fr_one(), fr_one()};
    for (int i0 = 0; i0 < k; i0 += 4) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = i0 + q;
        if (i < k) {
          const Fr ri = ldf(r, i);
          const bool bit = (t >> (k - 1 - i)) & 1;
          acc[q] = fr_mul(acc[q], bit ? ri : fr_one_minus(ri));
        }
      }
    }
    stf(P<Fr*>(st, 8 + j), t, fr_mul(fr_mul(acc[0], acc[1]), fr_mul(acc[2], acc[3])));
  }
}

// ST_WSUM: sum_e V[e] A[e >> n] B[e & mask] into *p5.
// p0 V, p1 A, p2 B, p3 partials, p4 S, p5 dst, u0 n, q0 count.
__device__ __forceinline__ void body_wsum(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* V = P<const Fr*>(st, 0);
  const Fr* A = P<const Fr*>(st, 1);
  const Fr* B = P<const Fr*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  Fr acc[1] = {fr_zero()};
  for (uint64_t e = GTID; e < st.q[0]; e += GSTRIDE)
    acc[0] = fr_add(acc[0], fr_mul(fr_mul(ldf(V, e), ldf(A, e >> n)), ldf(B, e & mask)));
  write_partial<1>(acc, P<Fr*>(st, 3), tile);
}
__device__ __forceinline__ void finish_wsum(const Step& st, uint32_t ntiles) {
  Fr tot[1];
  sum_partials<1>(P<const Fr*>(st, 3), ntiles, tot);
  if (threadIdx.x == 0) *P<Fr*>(st, 5) = tot[0];
}

// Phase-1 bookkeeping tables over (x, c):
//   G[x,c] = sum_{MUL z: x_z=x} T[z,c] W[y_z,c] + sum_{ADD z: x_z=x} T[z,c]
//   H[x,c] = sum_{ADD z: x_z=x} T[z,c] W[y_z,c]
// with T[z,c] = aU[z] Cu[c] + bV[z] Cv[c] (the factored eq of both claims).
// p0 W, p1 G, p2 H, p3 xrow, p4 xent, p5 aU, p6 bV, p7 Cu, p8 Cv, u0 n.
__device__ __forceinline__ void phase1_entry(const Step& st, uint64_t e, Fr& g, Fr& h) {
  const Fr* __restrict__ W = P<const Fr*>(st, 0);
  const uint32_t* __restrict__ xrow = P<const uint32_t*>(st, 3);
  const uint2* __restrict__ xent = P<const uint2*>(st, 4);
  const Fr* __restrict__ aU = P<const Fr*>(st, 5);
  const Fr* __restrict__ bV = P<const Fr*>(st, 6);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  const uint64_t x = e >> n, c = e & mask;
  const Fr cu = ldf(P<const Fr*>(st, 7), c), cv = ldf(P<const Fr*>(st, 8), c);
  g = fr_zero();
  h = fr_zero();
  // The first gate's terms are assigned, not added to zero: with 2^n >= 64
  // copies every lane of a wave walks the same gate list (the entries of one
  // x), so these branches do not diverge and an entry with one gate costs no
  // additions.
  const uint32_t k0 = xrow[x], k1 = xrow[x + 1];
  for (uint32_t k = k0; k < k1; ++k) {
    const uint2 ent = xent[k];
    const uint64_t z = ent.x, y = ent.y & 0x7fffffffu;
    const Fr T = fr_mul_add2(ldf(aU, z), cu, ldf(bV, z), cv);
    const Fr tw = fr_mul(T, ldf(W, (y << n) | c));
    if (k == k0) {
      if (ent.y >> 31) {
        g = tw;
      } else {
        g = T;
        h = tw;
      }
    } else if (ent.y >> 31) {
      g = fr_add(g, tw);
    } else {
      g = fr_add(g, T);
      h = fr_add(h, tw);
    }
  }
}

// ST_P1_INIT: the tables alone; q0 count.
__device__ __forceinline__ void body_p1_init(const Step& st, uint32_t tile, uint32_t ntiles) {
  Fr* G = P<Fr*>(st, 1);
  Fr* H = P<Fr*>(st, 2);
  for (uint64_t e = GTID; e < st.q[0]; e += GSTRIDE) {
    Fr g, h;
    phase1_entry(st, e, g, h);
    stf(G, e, g);
    stf(H, e, h);
  }
}

// ST_P1_INIT_ROUND: the tables and the first round together: b builds entries
// b and b + half and evaluates the round-1 pair at t = 0, 2. With Lazy the
// t = 0 products of a thread's pairs are summed unreduced (a 512-bit
// accumulator, one reduction per 16 pairs; a thread takes many pairs here; a
// second accumulator for t = 2 would not fit the registers of three
// workgroups per CU); the batch kernel, which holds every body, takes the
// reduced form (Lazy = false) to stay within its registers.
// q0 half; p9 S, p10 partials, p11 r_out, p12 msg.
template <bool Lazy>
__device__ __forceinline__ void body_p1_init_round(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* W = P<const Fr*>(st, 0);
  Fr* G = P<Fr*>(st, 1);
  Fr* H = P<Fr*>(st, 2);
  const uint64_t half = st.q[0];
  Fr acc[2] = {fr_zero(), fr_zero()};
  FrWide e0 = frw_zero();
  uint32_t lazy = 0;
  // Lazy: the running sums wait in shared memory (a slot per thread), out of
  // the registers the gate walks need
  __shared__ Fr sacc[Lazy ? 2 : 1][Lazy ? kBlock : 1];
  __shared__ FrWide swide[Lazy ? kBlock : 1];
  if constexpr (Lazy) {
    sacc[0][threadIdx.x] = fr_zero();
    sacc[1][threadIdx.x] = fr_zero();
    swide[threadIdx.x] = frw_zero();
  }
  for (uint64_t b = GTID; b < half; b += GSTRIDE) {
    Fr g0, h0, g1, h1;
    phase1_entry(st, b, g0, h0);
    phase1_entry(st, b + half, g1, h1);
    stf(G, b, g0);
    stf(H, b, h0);
    stf(G, b + half, g1);
    stf(H, b + half, h1);
    const Fr w0 = ldf(W, b), w1 = ldf(W, b + half);
    const Fr w2 = fr_sub(fr_double(w1), w0), g2 = fr_sub(fr_double(g1), g0), h2 = fr_sub(fr_double(h1), h0);
    if constexpr (!Lazy) {
      acc[0] = fr_add(acc[0], fr_add(fr_mul(w0, g0), h0));
      acc[1] = fr_add(acc[1], fr_add(fr_mul(w2, g2), h2));
      continue;
    }
    FrWide ew = swide[threadIdx.x];
    frw_mac(ew, w0, g0);
    Fr a0 = fr_add(sacc[0][threadIdx.x], h0);
    sacc[1][threadIdx.x] = fr_add(sacc[1][threadIdx.x], fr_add(fr_mul(w2, g2), h2));
    if (++lazy == 16) {
      a0 = fr_add(a0, frw_reduce<16>(ew));
      ew = frw_zero();
      lazy = 0;
    }
    swide[threadIdx.x] = ew;
    sacc[0][threadIdx.x] = a0;
  }
  if constexpr (Lazy) {
    acc[0] = sacc[0][threadIdx.x];
    acc[1] = sacc[1][threadIdx.x];
    if (lazy) acc[0] = fr_add(acc[0], frw_reduce<16>(swide[threadIdx.x]));
  }
  write_partial<2>(acc, P<Fr*>(st, 10), tile);
}

// Sum of the partials, then the round's transcript step in wave 0: the hash
// of (e0, e2) gives r, and the round becomes the pending one. Meanwhile wave 1
// moves the claim through the previous pending round (if any) and writes that
// round's message, so the products by r stay off the chain of hashes.
__device__ __forceinline__ void finish_reduced_round(const Fr* partials, uint32_t ntiles, DevState* S, Fr* r_out,
                                     uint32_t* msg) {
  const uint32_t wid = threadIdx.x >> 6;
  // wave 0 fetches the transcript state while the partials are summed
  Sha256State st;
  if (wid == 0) st = load_state(S);
  Fr tot[2];
  if (ntiles <= 64) {
    // every partial fits in wave 0: a wave sum, no LDS round trip
    tot[0] = fr_zero();
    tot[1] = fr_zero();
    if (wid == 0) {
      if (threadIdx.x < ntiles) {
        tot[0] = ldf(partials, 2ull * threadIdx.x);
        tot[1] = ldf(partials, 2ull * threadIdx.x + 1);
      }
      tot[0] = lane_fr(wave_sum_to_lane63(tot[0]), 63);
      tot[1] = lane_fr(wave_sum_to_lane63(tot[1]), 63);
    }
  } else {
    sum_partials<2>(partials, ntiles, tot);
  }
  bool pend = false;
  Fr claim, pe0, pe2, pr;
  uint32_t* pmsg = nullptr;
  if (wid == 1) {
    pend = S->pending != 0;
    if (pend) {
      claim = S->claim;
      pe0 = S->pend_e0;
      pe2 = S->pend_e2;
      pr = S->pend_r;
      pmsg = S->pend_msg;
    }
  }
  // wave 1 has read the pending round before wave 0 overwrites it
  __syncthreads();
  if (wid == 0) {
    const Fr r = round_hash_wave(st, tot[0], tot[1]);
    if (threadIdx.x == 0) {
      save_state(S, st);
      stf(r_out, 0, r);
      S->pend_e0 = tot[0];
      S->pend_e2 = tot[1];
      S->pend_r = r;
      S->pend_msg = msg;
      S->pending = 1;
    }
  } else if (wid == 1 && pend) {
    claim = round_claim_wave(pr, pe0, fr_sub(claim, pe0), pe2, pmsg);
    if (threadIdx.x == 64) S->claim = claim;
  }
}

__device__ __forceinline__ void finish_p1_init_round(const Step& st, uint32_t ntiles) {
  finish_reduced_round(P<const Fr*>(st, 10), ntiles, P<DevState*>(st, 9), P<Fr*>(st, 11), P<uint32_t*>(st, 12));
}

// Entries b and b + half of one table of a round. With Fold the source has
// 4*half entries and is first folded by r (entry i of the folded table is
// src[i] + r (src[i + 2 half] - src[i])); the folded entries are stored to dst.
template <bool Fold>
__device__ __forceinline__ void pair_entries(const Fr* src, Fr* dst, uint64_t b, uint64_t half, const Fr& r,
                                             Fr& lo, Fr& hi) {
  if constexpr (Fold) {
    const uint64_t m = 2 * half;
    const Fr a0 = ldf(src, b), a1 = ldf(src, b + m);
    const Fr b0 = ldf(src, b + half), b1 = ldf(src, b + half + m);
    lo = fr_add(a0, fr_mul(r, fr_sub(a1, a0)));
    hi = fr_add(b0, fr_mul(r, fr_sub(b1, b0)));
    stf(dst, b, lo);
    stf(dst, b + half, hi);
  } else {
    lo = ldf(src, b);
    hi = ldf(src, b + half);
  }
}

// One pair b of a round: the round polynomial's terms at t = 0 (the entry b)
// and t = 2 (2 * entry(b + half) - entry(b)). The last table of a form is
// additive, the others multiply in pairs (0,1), (2,3). Tables are visited one
// group at a time (scheduling barriers between groups) so that only one
// group's operands are live.
template <class Form, bool Fold>
__device__ __forceinline__ void round_pair(const Fr* const* src, Fr* const* dst, uint64_t b,
                                           uint64_t half, const Fr& r, Fr& acc0, Fr& acc2) {
  constexpr int NT = Form::NT;
  {
    Fr lo, hi;
    pair_entries<Fold>(src[NT - 1], dst[NT - 1], b, half, r, lo, hi);
    acc0 = fr_add(acc0, lo);
    acc2 = fr_add(acc2, fr_sub(fr_double(hi), lo));
  }
  if constexpr (NT == 3) {
    __builtin_amdgcn_sched_barrier(0);
    Fr xl, xh, yl, yh;
    pair_entries<Fold>(src[0], dst[0], b, half, r, xl, xh);
    pair_entries<Fold>(src[1], dst[1], b, half, r, yl, yh);
    acc0 = fr_add(acc0, fr_mul(xl, yl));
    acc2 = fr_add(acc2, fr_mul(fr_sub(fr_double(xh), xl), fr_sub(fr_double(yh), yl)));
  } else {
    // both product pairs of a FormB pair at once: one reduction per point
    __builtin_amdgcn_sched_barrier(0);
    Fr pl, ph, fl, fh;
    pair_entries<Fold>(src[0], dst[0], b, half, r, pl, ph);
    pair_entries<Fold>(src[1], dst[1], b, half, r, fl, fh);
    __builtin_amdgcn_sched_barrier(0);
    Fr ql, qh, gl, gh;
    pair_entries<Fold>(src[2], dst[2], b, half, r, ql, qh);
    pair_entries<Fold>(src[3], dst[3], b, half, r, gl, gh);
    acc0 = fr_add(acc0, fr_mul_add2(pl, fl, ql, gl));
    acc2 = fr_add(acc2, fr_mul_add2(fr_sub(fr_double(ph), pl), fr_sub(fr_double(fh), fl),
                                    fr_sub(fr_double(qh), ql), fr_sub(fr_double(gh), gl)));
  }
  __builtin_amdgcn_sched_barrier(0);
}

// The pairs [b0, half) with stride `stride` of one round, accumulated.
template <class Form>
__device__ __forceinline__ void round_range(const Fr* const* src, Fr* const* dst, uint64_t b0, uint64_t stride,
                                            uint64_t half, bool fold, const Fr& r, Fr& acc0, Fr& acc2) {
  if (fold) {
    for (uint64_t b = b0; b < half; b += stride) round_pair<Form, true>(src, dst, b, half, r, acc0, acc2);
  } else {
    for (uint64_t b = b0; b < half; b += stride) round_pair<Form, false>(src, dst, b, half, r, acc0, acc2);
  }
}

// ST_ROUND_A / ST_ROUND_B: one sumcheck round (optional fold by the previous
// challenge, evaluation at t = 0, 2); q0 half. Pointers: src[0..NT),
// dst[NT..2NT), then rprev, S, partials, r_out, msg (RoundPtrs).
template <class Form>
__device__ __forceinline__ void body_round(const Step& st, uint32_t tile, uint32_t ntiles) {
  using R = RoundPtrs<Form::NT>;
  const Fr* src[Form::NT];
  Fr* dst[Form::NT];
#pragma unroll
  for (int k = 0; k < Form::NT; ++k) {
    src[k] = P<const Fr*>(st, k);
    dst[k] = P<Fr*>(st, Form::NT + k);
  }
  const Fr* rprev = P<const Fr*>(st, R::kR);
  const bool fold = rprev != nullptr;
  const Fr r = fold ? ldf(rprev, 0) : fr_zero();
  const uint64_t half = st.q[0];
  Fr acc[2] = {fr_zero(), fr_zero()};
  round_range<Form>(src, dst, GTID, GSTRIDE, half, fold, r, acc[0], acc[1]);
  write_partial<2>(acc, P<Fr*>(st, R::kPart), tile);
}
template <class Form>
__device__ __forceinline__ void finish_round_step(const Step& st, uint32_t ntiles) {
  using R = RoundPtrs<Form::NT>;
  finish_reduced_round(P<const Fr*>(st, R::kPart), ntiles, P<DevState*>(st, R::kS), P<Fr*>(st, R::kROut),
                       P<uint32_t*>(st, R::kMsg));
}

// Table k of NT pointers, for a k that varies across lanes: a chain of
// register selects. Each candidate passes through an empty asm statement, so
// the optimizer cannot turn the chain back into an indexed load from a
// private array (which would put the pointers in scratch memory and add a
// dependent load to every task).
template <int NT, class T>
__device__ __forceinline__ T pick(T const (&a)[NT], uint32_t k) {
  uint64_t p = reinterpret_cast<uint64_t>(a[0]);
#pragma unroll
  for (int q = 1; q < NT; ++q) {
    uint64_t c = reinterpret_cast<uint64_t>(a[q]);
    asm volatile("" : "+v"(c));
    p = k == (uint32_t)q ? c : p;
  }
  return reinterpret_cast<T>(p);
}

// ST_TAIL_A / ST_TAIL_B: the remaining u0 rounds of a phase in one workgroup
// (at least 128 threads), then the final fold. q0 = table size before the
// pending fold (if any). Pointers: src, dst, rpending, S, r_out, msg,
// final_out, proof_value. The final value of table 0 is stored in *final_out
// and, if proof_value is not null, written to the proof and absorbed.
// The transcript chain of the rounds needs only the sums e0 and e2 of each
// round (the hash absorbs them; the challenge is the hash value), not the
// running claim, so the two chains run in different waves:
//  - wave 0 holds the transcript state and hashes each round's e0, e2 as soon
//    as the sums are in, then publishes r;
//  - wave 1 holds the claim: while wave 0 hashes round j, it moves the claim
//    through round j - 1 (e1 = claim - e0, products by r) and writes that
//    round's message (in round 0, through the round a grid finisher left
//    pending, if any); the last round's claim moves after the final fold, and
//    nothing is left pending;
//  - waves 1.. (the workers) fold the tables by the previous challenge (one
//    task per entry, in place after the first round) and evaluate them at
//    t = 0 and t = 2 (one task per pair and t).
template <class Form>
__device__ __forceinline__ void body_tail(const Step& st, uint32_t, uint32_t) {
  constexpr int NT = Form::NT;
  const Fr* src[NT];
  Fr* dst[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    src[k] = P<const Fr*>(st, k);
    dst[k] = P<Fr*>(st, NT + k);
  }
  const Fr* rpending = P<const Fr*>(st, 2 * NT);
  DevState* S = P<DevState*>(st, 2 * NT + 1);
  Fr* r_out = P<Fr*>(st, 2 * NT + 2);
  uint32_t* msg = P<uint32_t*>(st, 2 * NT + 3);
  Fr* final_out = P<Fr*>(st, 2 * NT + 4);
  uint32_t* proof_value = P<uint32_t*>(st, 2 * NT + 5);
  const uint32_t wid = threadIdx.x >> 6;
  const uint32_t w = threadIdx.x - 64, nw = blockDim.x - 64;  // worker index and count
  uint64_t size = st.q[0];
  const uint32_t rounds = st.u[0];
  __shared__ Fr r_sh, e_sh[2];  // the last round's challenge and sums (e0, e2)
  __shared__ Fr red1[2];
  bool fold = rpending != nullptr;
  Sha256State state;  // wave 0
  // wave 1: the claim and the pending round it has not moved through yet
  Fr claim = fr_zero(), pe0 = fr_zero(), pe2 = fr_zero(), pr = fr_zero();
  uint32_t* pmsg = nullptr;
  bool pend = false;
  if (wid == 0) state = load_state(S);
  if (wid == 1) {
    claim = S->claim;
    pend = S->pending != 0;
    if (pend) {
      pe0 = S->pend_e0;
      pe2 = S->pend_e2;
      pr = S->pend_r;
      pmsg = S->pend_msg;
    }
  }
  if (threadIdx.x == 0) r_sh = fold ? ldf(rpending, 0) : fr_zero();
  __syncthreads();
  for (uint32_t j = 0;; ++j) {
    if (fold) {
      const uint64_t m = size / 2;
      if (wid > 0) {
        // entry i of table k becomes src[i] + r (src[i + m] - src[i])
        const uint32_t lg = 63 - __clzll(m);
        const Fr rf = r_sh;
        for (uint64_t t = w; t < NT * m; t += nw) {
          const uint32_t k = (uint32_t)(t >> lg);
          const uint64_t i = t & (m - 1);
          const Fr* sp = pick<NT>(src, k);
          const Fr a0 = ldf(sp, i), a1 = ldf(sp, i + m);
          stf(pick<NT>(dst, k), i, fr_add(a0, fr_mul(rf, fr_sub(a1, a0))));
        }
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NT; ++k) src[k] = dst[k];
      size = m;
    }
    if (j == rounds) break;
    // evaluate: task u < size is the pair b = u mod half at t = 0 (u < half) or t = 2
    const uint64_t half = size / 2;
    Fr acc[2] = {fr_zero(), fr_zero()};
    if (wid > 0) {
      for (uint64_t u = w; u < size; u += nw) {
        const bool t2 = u >= half;
        const uint64_t b = t2 ? u - half : u;
        Fr x[NT];
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          const Fr lo = ldf(src[k], b), hi = ldf(src[k], b + half);
          x[k] = t2 ? fr_sub(fr_double(hi), lo) : lo;
        }
        Fr v;
        if constexpr (NT == 3) v = fr_add(fr_mul(x[0], x[1]), x[2]);
        else v = fr_add(fr_mul_add2(x[0], x[1], x[2], x[3]), x[4]);
        if (t2) acc[1] = fr_add(acc[1], v);
        else acc[0] = fr_add(acc[0], v);
      }
    }
    // the claim wave takes the previous round's sums and challenge
    if (wid == 1 && j > 0) {
      pe0 = e_sh[0];
      pe2 = e_sh[1];
      pr = r_sh;
      pmsg = msg + 24 * (j - 1);
      pend = true;
    }
    if (size <= 64) {
      // Every task is in the first worker wave, one per lane: lanes [0, half)
      // hold the t = 0 terms and lanes [half, size) the t = 2 terms, so one
      // segmented sum over aligned blocks of `half` lanes (log2(half) DPP
      // steps) leaves e0 in lane half - 1 and e2 in lane size - 1.
      if (wid == 1) {
        Fr v = fr_add(acc[0], acc[1]);
        if (half >= 2) v = fr_add(v, dpp_fr<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
        if (half >= 4) v = fr_add(v, dpp_fr<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
        if (half >= 8) v = fr_add(v, dpp_fr<0x141, 0xF>(v));  // row_half_mirror
        if (half >= 16) v = fr_add(v, dpp_fr<0x140, 0xF>(v)); // row_mirror
        if (half >= 32) v = fr_add(v, dpp_fr<0x142, 0xA>(v)); // row_bcast15 into rows 1 and 3
        const uint32_t lane = threadIdx.x & 63;
        if (lane == half - 1) red1[0] = v;
        if (lane == size - 1) red1[1] = v;
      }
      __syncthreads();
      if (wid == 0) {
        acc[0] = red1[0];
        acc[1] = red1[1];
      }
    } else {
      block_sum_to_wave0<2>(acc);
    }
    if (wid == 0) {
      const Fr r = round_hash_wave(state, acc[0], acc[1]);
      if (threadIdx.x == 0) {
        r_sh = r;
        e_sh[0] = acc[0];
        e_sh[1] = acc[1];
        stf(r_out, j, r);
      }
    } else if (wid == 1 && pend) {
      claim = round_claim_wave(pr, pe0, fr_sub(claim, pe0), pe2, pmsg);
      pend = false;
    }
    __syncthreads();
    fold = true;
  }
  // the last round's claim move (the final fold has run)
  if (wid == 1) {
    if (rounds > 0) {
      pe0 = e_sh[0];
      pe2 = e_sh[1];
      pr = r_sh;
      pmsg = msg + 24 * (rounds - 1);
      pend = true;
    }
    if (pend) claim = round_claim_wave(pr, pe0, fr_sub(claim, pe0), pe2, pmsg);
    if (threadIdx.x == 64) {
      S->claim = claim;
      S->pending = 0;
    }
  }
  if (threadIdx.x == 0) {
    if (rounds > 0) save_state(S, state);
    const Fr v = ldf(src[0], 0);
    if (proof_value) finish_value(S, v, final_out, proof_value);
    else *final_out = v;
  }
}

// ---- pipelined tail
// The round sums of round j + 1 are quadratics in the challenge r_j that folds
// level j (the tables after j folds) into level j + 1: for pair b of level
// j + 1 (2Q entries, pairs (b, b + Q)) and point t, each table's value is
// linear in r_j, equal at r_j = 0 and r_j = 1 to entries of level j (4Q
// entries): t = 0: L[b] and L[b + 2Q]; t = 2: 2 L[b + Q] - L[b] and
// 2 L[b + 3Q] - L[b + 2Q]. The term (products of pairs of tables plus the
// additive table) is then a quadratic q(r) fixed by q(0), q(1) and its leading
// coefficient (the product of the slopes), three products per task and form
// product; the sums over tasks give e_t(r) = V0 + r (V1 - V0 - C2) + r^2 C2.

// One task of the coefficient sums: pair b of the next level at t = 0 or 2
// (t2), from level L (4Q entries); adds q(0), q(1) and the leading coefficient.
template <class Form>
__device__ __forceinline__ void tail_task(const Fr* const* L, uint64_t b, uint64_t Q, bool t2, Fr (&acc)[3]) {
  constexpr int NT = Form::NT;
  Fr p0[NT], p1[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const Fr a = ldf(L[k], b), c = ldf(L[k], b + 2 * Q);
    if (t2) {
      const Fr a1 = ldf(L[k], b + Q), c1 = ldf(L[k], b + 3 * Q);
      p0[k] = fr_sub(fr_double(a1), a);
      p1[k] = fr_sub(fr_double(c1), c);
    } else {
      p0[k] = a;
      p1[k] = c;
    }
  }
  Fr v0, v1, c2;
  if constexpr (NT == 3) {
    v0 = fr_add(fr_mul(p0[0], p0[1]), p0[2]);
    v1 = fr_add(fr_mul(p1[0], p1[1]), p1[2]);
    c2 = fr_mul(fr_sub(p1[0], p0[0]), fr_sub(p1[1], p0[1]));
  } else {
    v0 = fr_add(fr_mul_add2(p0[0], p0[1], p0[2], p0[3]), p0[4]);
    v1 = fr_add(fr_mul_add2(p1[0], p1[1], p1[2], p1[3]), p1[4]);
    c2 = fr_mul_add2(fr_sub(p1[0], p0[0]), fr_sub(p1[1], p0[1]), fr_sub(p1[2], p0[2]), fr_sub(p1[3], p0[3]));
  }
  acc[0] = fr_add(acc[0], v0);
  acc[1] = fr_add(acc[1], v1);
  acc[2] = fr_add(acc[2], c2);
}

// The same for a round whose level needs no fold (the tail's first round when
// no challenge is pending): pair b of L (2 half entries) at t; a constant
// quadratic (q(0) = q(1), no leading coefficient).
template <class Form>
__device__ __forceinline__ void tail_task_direct(const Fr* const* L, uint64_t b, uint64_t half, bool t2,
                                                 Fr (&acc)[3]) {
  constexpr int NT = Form::NT;
  Fr x[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    const Fr lo = ldf(L[k], b);
    x[k] = t2 ? fr_sub(fr_double(ldf(L[k], b + half)), lo) : lo;
  }
  Fr v;
  if constexpr (NT == 3) v = fr_add(fr_mul(x[0], x[1]), x[2]);
  else v = fr_add(fr_mul_add2(x[0], x[1], x[2], x[3]), x[4]);
  acc[0] = fr_add(acc[0], v);
  acc[1] = fr_add(acc[1], v);
}

// Worker waves whose tasks are nonempty for `tasks` tasks per half.
__device__ __forceinline__ uint32_t tail_active_waves(uint64_t tasks, uint32_t hw) {
  const uint64_t w = (tasks + 63) / 64;
  return w < hw ? (uint32_t)w : hw;
}

// The coefficient sums of one point over one half of the worker waves: each
// thread takes tasks th, th + nth, ..; each wave with tasks sums its lanes and
// stores (V0, V1, C2) in part[wave of the half].
template <class Form>
__device__ __forceinline__ void tail_coefficients(const Fr* const* L, uint64_t tasks, bool direct, bool t2,
                                                  uint32_t th, uint32_t nth, uint32_t wih, uint32_t nact,
                                                  Fr (*part)[3]) {
  if (wih >= nact) return;  // the wave has no task
  Fr acc[3] = {fr_zero(), fr_zero(), fr_zero()};
  if (direct) {
    for (uint64_t b = th; b < tasks; b += nth) tail_task_direct<Form>(L, b, tasks, t2, acc);
  } else {
    for (uint64_t b = th; b < tasks; b += nth) tail_task<Form>(L, b, tasks, t2, acc);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[k] = wave_sum_to_lane63(acc[k]);
  if ((threadIdx.x & 63) == 63) {
#pragma unroll
    for (int k = 0; k < 3; ++k) part[wih][k] = acc[k];
  }
}

// Round j + 1's coefficient sums for at most 32 pairs: coefficient s (q(0),
// q(1) or the leading one) of every task in one wave, lanes 0..31 at t = 0 and
// lanes 32..63 at t = 2, one pair per lane (one product, or one pair of
// products for Form B); a segmented sum leaves the totals in lanes 31 and 63.
template <class Form>
__device__ __forceinline__ void tail_coefficient_stream(const Fr* const* L, uint64_t Q, uint32_t s,
                                                        Fr (*part)[8][3]) {
  constexpr int NT = Form::NT;
  const uint32_t lane = threadIdx.x & 63;
  const bool t2 = lane >= 32;
  const uint64_t b = lane & 31;
  Fr v = fr_zero();
  if (b < Q) {
    Fr p[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) {
      if (s == 2 && k == NT - 1) {  // the additive table has no slope product
        p[k] = fr_zero();
        continue;
      }
      Fr x0 = fr_zero(), x1 = fr_zero();
      if (s != 1) {
        const Fr a = ldf(L[k], b);
        x0 = t2 ? fr_sub(fr_double(ldf(L[k], b + Q)), a) : a;
      }
      if (s != 0) {
        const Fr c = ldf(L[k], b + 2 * Q);
        x1 = t2 ? fr_sub(fr_double(ldf(L[k], b + 3 * Q)), c) : c;
      }
      p[k] = s == 0 ? x0 : (s == 1 ? x1 : fr_sub(x1, x0));
    }
    if constexpr (NT == 3) v = fr_add(fr_mul(p[0], p[1]), p[2]);
    else v = fr_add(fr_mul_add2(p[0], p[1], p[2], p[3]), p[4]);
  }
  v = fr_add(v, dpp_fr<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
  v = fr_add(v, dpp_fr<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
  v = fr_add(v, dpp_fr<0x141, 0xF>(v));  // row_half_mirror
  v = fr_add(v, dpp_fr<0x140, 0xF>(v));  // row_mirror
  v = fr_add(v, dpp_fr<0x142, 0xA>(v));  // row_bcast15 into rows 1 and 3
  if (lane == 31) part[0][0][s] = v;
  if (lane == 63) part[1][0][s] = v;
}

// The claim through a round with sums e0, e2 (e1 = claim - e0) and challenge
// r: g(r) = e0 + r (A + r B) with B = (e2 - 2 e1 + e0) / 2, A = e1 - e0 - B.
__device__ __forceinline__ Fr tail_claim_next(const Fr& claim, const Fr& e0, const Fr& e2, const Fr& r) {
  const Fr e1 = fr_sub(claim, e0);
  const Fr B = fr_half(fr_add(fr_sub(e2, fr_double(e1)), e0));
  const Fr A = fr_sub(fr_sub(e1, e0), B);
  return fr_add(e0, fr_mul(r, fr_add(A, fr_mul(r, B))));
}

// A round's message (e0, e1 = claim - e0, e2 in canonical form), lane k
// converting and storing element k.
__device__ __forceinline__ void tail_message(const Fr& claim, const Fr& e0, const Fr& e2, uint32_t* msg) {
  const uint32_t lane = threadIdx.x & 63;
  const Fr e1 = fr_sub(claim, e0);
  Fr x = e0;
#pragma unroll
  for (int k = 0; k < 8; ++k) x.v[k] = lane == 1 ? e1.v[k] : (lane == 2 ? e2.v[k] : x.v[k]);
  const Fr c = fr_from_mont(x);
  if (lane < 3) stf(reinterpret_cast<Fr*>(msg), lane, c);
}

// ST_TAIL_A / ST_TAIL_B, pipelined: the same rounds, messages, challenges and
// final values as body_tail, with the table work off the hash chain. Eight
// waves (two per SIMD, wave w on SIMD w mod 4), by role:
//  - wave 0 holds the transcript: in round j it sums the workers' coefficient
//    partials of round j, evaluates them at r_{j-1} (two products) and hashes
//    (e0, e2) into r_j;
//  - in the first half of round j, wave 1 moves the claim through round
//    j - 1 (two products) and wave 7 writes round j - 1's message (e0, e1 =
//    claim - e0, e2 in canonical form) from the claim before it;
//  - waves 2-7 fold level j - 1 into level j by r_{j-1} (first half of round
//    j, before a workgroup barrier); then, while wave 0 hashes, waves 1-7
//    compute round j + 1's coefficients from level j: for more than 32
//    pairs, one task (three products) per thread; for at most 32, one product
//    per lane, waves 2, 3 and 5 taking q(0), q(1) and the leading coefficient.
// Two workgroup barriers per round; the previous round's values sit in
// alternating shared slots.
template <class Form>
__device__ __forceinline__ void body_tail_pipe(const Step& st, uint32_t, uint32_t) {
  constexpr int NT = Form::NT;
  const Fr* src[NT];
  Fr* dst[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    src[k] = P<const Fr*>(st, k);
    dst[k] = P<Fr*>(st, NT + k);
  }
  const Fr* rpending = P<const Fr*>(st, 2 * NT);
  DevState* S = P<DevState*>(st, 2 * NT + 1);
  Fr* r_out = P<Fr*>(st, 2 * NT + 2);
  uint32_t* msg = P<uint32_t*>(st, 2 * NT + 3);
  Fr* final_out = P<Fr*>(st, 2 * NT + 4);
  uint32_t* proof_value = P<uint32_t*>(st, 2 * NT + 5);
  const uint32_t wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // Per-thread coefficient tasks: waves 2, 3, 1 at t = 0 and 5, 6, 7, 4 at
  // t = 2 (the first waves of each group on different SIMDs, for few tasks).
  // Folds: waves 2, 3, 5, 6, 4, 7 in that order. Wave 4 shares SIMD 0 with
  // wave 0 and wave 5 SIMD 1 with wave 1: the older wave of a SIMD issues
  // first, so the transcript, claim and message chains keep their speed.
  constexpr uint32_t kHw0 = 3, kHw2 = 4;  // coefficient waves for t = 0 and t = 2
  const bool worker = wid != 0;
  const bool t2 = wid >= 4;
  const uint32_t wih = t2 ? (wid == 4 ? 3 : wid - 5) : (wid == 1 ? 2 : wid - 2);  // index in its group
  const uint32_t th = wih * 64 + lane, nth = (t2 ? kHw2 : kHw0) * 64;
  const uint32_t ford = wid == 4 ? 4 : (wid == 7 ? 5 : wid - 2 - (wid > 4));
  const uint32_t fw = ford * 64 + lane, nfw = 6 * 64;  // index among the folders
  const uint64_t size = st.q[0];
  const uint32_t rounds = st.u[0];
  const bool pending = rpending != nullptr;
  __shared__ Fr part[2][8][3];    // coefficient partials (half, wave, V0 V1 C2)
  __shared__ Fr r_sh[2], e_sh[2][2], claim_sh[2];
  // Values that cross a barrier live in the shared slots (r_sh, e_sh) rather
  // than in registers: every wave holds the registers of every role.
  Sha256State state;  // wave 0
  Fr claim;           // waves 1 and 7: the claim before the first round (wave 1 moves it)
  bool grid_pend = false;  // waves 1 and 7: a grid round whose claim move is pending
  if (wid == 0) {
    state = load_state(S);
    if (lane == 0) r_sh[1] = pending ? ldf(rpending, 0) : fr_zero();  // r_{-1}
  } else if (wid == 1 || wid == 7) {
    claim = S->claim;
    grid_pend = S->pending != 0;
  }
  const Fr* cur[NT];  // the current level
#pragma unroll
  for (int k = 0; k < NT; ++k) cur[k] = src[k];
  // round 0's coefficients: from the unfolded tables (a pending fold) or directly
  uint64_t tasks = 0;
  if (rounds > 0) tasks = pending ? size / 4 : size / 2;
  uint32_t nact0 = tail_active_waves(tasks, kHw0), nact2 = tail_active_waves(tasks, kHw2);
  if (worker && rounds > 0)
    tail_coefficients<Form>(cur, tasks, !pending, t2, th, nth, wih, t2 ? nact2 : nact0, part[t2 ? 1 : 0]);
  __syncthreads();
  for (uint32_t j = 0; j < rounds; ++j) {
    const bool fold = pending || j > 0;
    const uint64_t m = 1ull << (rounds - j);  // entries of level j
    if (wid == 0) {
      // round j's sums at r_{j-1}: lane 0 for t = 0, lane 1 for t = 2
      const uint32_t h = lane & 1, nact = h ? nact2 : nact0;
      const Fr r_prev = opaque(r_sh[(j - 1) & 1]);
      Fr v0 = fr_zero(), v1 = fr_zero(), c2 = fr_zero();
      for (uint32_t a = 0; a < nact; ++a) {
        v0 = fr_add(v0, part[h][a][0]);
        v1 = fr_add(v1, part[h][a][1]);
        c2 = fr_add(c2, part[h][a][2]);
      }
      const Fr c1 = fr_sub(fr_sub(v1, v0), c2);
      const Fr e = fr_add(v0, fr_mul(r_prev, fr_add(c1, fr_mul(r_prev, c2))));
      if (lane < 2) e_sh[j & 1][lane] = e;
    } else if (wid == 1) {
      // the claim through round j - 1 (or the pending grid round)
      if (j > 0) {
        const uint32_t q = (j - 1) & 1;
        claim = tail_claim_next(claim, opaque(e_sh[q][0]), opaque(e_sh[q][1]), opaque(r_sh[q]));
      }
      else if (grid_pend) claim = tail_claim_next(claim, opaque(S->pend_e0), opaque(S->pend_e2), opaque(S->pend_r));
      if (lane == 0) claim_sh[j & 1] = claim;
    } else {  // waves 2-7: the folders
      if (wid == 7) {
        // round j - 1's message (or the pending grid round's), from the claim before it
        if (j > 0) {
          const uint32_t q = (j - 1) & 1;
          tail_message(opaque(claim_sh[q]), opaque(e_sh[q][0]), opaque(e_sh[q][1]), msg + 24 * (j - 1));
        } else if (grid_pend) {
          tail_message(claim, opaque(S->pend_e0), opaque(S->pend_e2), S->pend_msg);
        }
      }
      if (fold) {
        // level j - 1 into level j by r_{j-1} (in place after the first fold)
        const Fr rf = opaque(r_sh[(j - 1) & 1]);
        const uint32_t lg = rounds - j;
        for (uint64_t t = fw; t < NT * m; t += nfw) {
          const uint32_t k = (uint32_t)(t >> lg);
          const uint64_t i = t & (m - 1);
          const Fr* sp = pick<NT>(cur, k);
          const Fr a0 = ldf(sp, i), a1 = ldf(sp, i + m);
          stf(pick<NT>(dst, k), i, fr_add(a0, fr_mul(rf, fr_sub(a1, a0))));
        }
      }
    }
    if (fold) {
#pragma unroll
      for (int k = 0; k < NT; ++k) cur[k] = dst[k];
    }
    __syncthreads();
    const uint64_t next = j + 1 < rounds ? m / 4 : 0;  // tasks of round j + 1
    if (wid == 0) {
      const Fr r = round_hash_wave(state, opaque(e_sh[j & 1][0]), opaque(e_sh[j & 1][1]));
      if (lane == 0) {
        r_sh[j & 1] = r;
        stf(r_out, j, r);
      }
    } else if (next > 32) {
      if (worker)
        tail_coefficients<Form>(cur, next, false, t2, th, nth, wih,
                                t2 ? tail_active_waves(next, kHw2) : tail_active_waves(next, kHw0), part[t2 ? 1 : 0]);
    } else if (next && (wid == 2 || wid == 3 || wid == 5)) {
      tail_coefficient_stream<Form>(cur, next, wid == 2 ? 0 : (wid == 3 ? 1 : 2), part);
    }
    nact0 = next > 32 ? tail_active_waves(next, kHw0) : 1;
    nact2 = next > 32 ? tail_active_waves(next, kHw2) : 1;
    __syncthreads();
  }
  // the final fold (by r_{rounds-1}, or by the pending challenge when no
  // round is left) and the last claim move
  const bool any_fold = pending || rounds > 0;
  if (wid == 0) {
    const Fr r_prev = opaque(r_sh[(rounds - 1) & 1]);  // r_{rounds-1}, or r_{-1}
    Fr v = fr_zero();  // lane k: the final value of table k
    if (any_fold && lane < NT) {
      const Fr* sp = pick<NT>(cur, lane);
      const Fr a0 = ldf(sp, 0), a1 = ldf(sp, 1);
      v = fr_add(a0, fr_mul(r_prev, fr_sub(a1, a0)));
      stf(pick<NT>(dst, lane), 0, v);
    }
    if (lane == 0) {
      if (rounds > 0) save_state(S, state);
      if (!any_fold) v = ldf(src[0], 0);
      if (proof_value) finish_value(S, v, final_out, proof_value);
      else *final_out = v;
    }
  } else if (wid == 1) {
    if (rounds > 0) {
      const uint32_t q = (rounds - 1) & 1;
      claim = tail_claim_next(claim, opaque(e_sh[q][0]), opaque(e_sh[q][1]), opaque(r_sh[q]));
    } else if (grid_pend) {
      claim = tail_claim_next(claim, opaque(S->pend_e0), opaque(S->pend_e2), opaque(S->pend_r));
    }
    if (lane == 0) {
      S->claim = claim;
      S->pending = 0;
    }
  } else if (wid == 7) {
    if (rounds > 0) {
      const uint32_t q = (rounds - 1) & 1;
      tail_message(opaque(claim_sh[q]), opaque(e_sh[q][0]), opaque(e_sh[q][1]), msg + 24 * (rounds - 1));
    } else if (grid_pend) {
      tail_message(claim, opaque(S->pend_e0), opaque(S->pend_e2), S->pend_msg);
    }
  }
}

// ST_COPY_WEIGHTS: U[c] = Cu[c] EC[c], V[c] = Cv[c] EC[c]; SU, SV their sums
// (one workgroup). p0 Cu, p1 Cv, p2 EC, p3 U, p4 V, p5 S, q0 ncop.
__device__ __forceinline__ void body_copy_weights(const Step& st, uint32_t, uint32_t) {
  const Fr* Cu = P<const Fr*>(st, 0);
  const Fr* Cv = P<const Fr*>(st, 1);
  const Fr* EC = P<const Fr*>(st, 2);
  Fr* U = P<Fr*>(st, 3);
  Fr* V = P<Fr*>(st, 4);
  DevState* S = P<DevState*>(st, 5);
  Fr acc[2] = {fr_zero(), fr_zero()};
  for (uint64_t c = threadIdx.x; c < st.q[0]; c += kBlock) {
    const Fr ec = ldf(EC, c);
    const Fr u = fr_mul(ldf(Cu, c), ec), v = fr_mul(ldf(Cv, c), ec);
    stf(U, c, u);
    stf(V, c, v);
    acc[0] = fr_add(acc[0], u);
    acc[1] = fr_add(acc[1], v);
  }
  block_reduce<2>(acc);
  if (threadIdx.x == 0) {
    S->su = acc[0];
    S->sv = acc[1];
  }
}

// ST_P2_TABLES: phase-2 sub-circuit tables over y, the copy factors kept apart:
//   M[y,c] = U[c] Ma[y] + V[c] Mb[y],  A[y,c] = U[c] Aa[y] + V[c] Ab[y]
//   Ma[y] = sum_{MUL z: y_z=y} aU[z] EL[x_z] (Mb with bV; Aa, Ab over ADD gates)
//   Fa = vx Ma + Aa, Fb = vx Mb + Ab, Ka = vx Aa, Kb = vx Ab, Ks = SU Ka + SV Kb.
// p0 yrow, p1 yent, p2 aU, p3 bV, p4 EL, p5 S, p6 Fa, p7 Fb, p8 Ka, p9 Kb, p10 Ks, q0 count.
__device__ __forceinline__ void body_p2_tables(const Step& st, uint32_t tile, uint32_t ntiles) {
  const uint32_t* __restrict__ yrow = P<const uint32_t*>(st, 0);
  const uint2* __restrict__ yent = P<const uint2*>(st, 1);
  const Fr* __restrict__ aU = P<const Fr*>(st, 2);
  const Fr* __restrict__ bV = P<const Fr*>(st, 3);
  const Fr* __restrict__ EL = P<const Fr*>(st, 4);
  const DevState* S = P<const DevState*>(st, 5);
  const Fr vx = S->vx, su = S->su, sv = S->sv;
  for (uint64_t y = GTID; y < st.q[0]; y += GSTRIDE) {
    Fr ma = fr_zero(), mb = fr_zero(), aa = fr_zero(), ab = fr_zero();
    const uint32_t k1 = yrow[y + 1];
    for (uint32_t k = yrow[y]; k < k1; ++k) {
      const uint2 ent = yent[k];
      const uint64_t z = ent.x, x = ent.y & 0x7fffffffu;
      const Fr el = ldf(EL, x);
      const Fr a = fr_mul(ldf(aU, z), el), b = fr_mul(ldf(bV, z), el);
      if (ent.y >> 31) {
        ma = fr_add(ma, a);
        mb = fr_add(mb, b);
      } else {
        aa = fr_add(aa, a);
        ab = fr_add(ab, b);
      }
    }
    const Fr ka = fr_mul(vx, aa), kb = fr_mul(vx, ab);
    stf(P<Fr*>(st, 6), y, fr_add(fr_mul(vx, ma), aa));
    stf(P<Fr*>(st, 7), y, fr_add(fr_mul(vx, mb), ab));
    stf(P<Fr*>(st, 8), y, ka);
    stf(P<Fr*>(st, 9), y, kb);
    stf(P<Fr*>(st, 10), y, fr_mul_add2(su, ka, sv, kb));
  }
}

// ST_COPY_CONTRACT: row sums over the copies, P[y] = sum_c U[c] W[y,c],
// Q[y] = sum_c V[c] W[y,c]. A row of 2^n entries is handled by
// tpr = min(256, 2^n) threads; tile t covers rows t * (256 / tpr) onwards.
// p0 W, p1 U, p2 V, p3 P, p4 Q, u0 n, q0 rows.
__device__ __forceinline__ void body_copy_contract(const Step& st, uint32_t tile, uint32_t ntiles) {
  __shared__ Fr sp[kBlock], sq[kBlock];
  const Fr* __restrict__ W = P<const Fr*>(st, 0);
  const Fr* __restrict__ U = P<const Fr*>(st, 1);
  const Fr* __restrict__ V = P<const Fr*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t rows = st.q[0];
  const uint32_t tpr_log = n < 8 ? n : 8;
  const uint32_t tpr = 1u << tpr_log;
  const uint32_t lane = threadIdx.x & (tpr - 1);
  const uint64_t rows_per_tile = kBlock >> tpr_log;
  for (uint64_t base = (uint64_t)tile * rows_per_tile; base < rows; base += (uint64_t)ntiles * rows_per_tile) {
    const uint64_t row = base + (threadIdx.x >> tpr_log);
    Fr p = fr_zero(), q = fr_zero();
    if (row < rows) {
      // at most 16 unreduced products per accumulator between reductions
      const uint64_t ncop = 1ull << n;
      for (uint64_t c0 = lane; c0 < ncop; c0 += 16 * (uint64_t)tpr) {
        FrCols pw = frc_zero(), qw = frc_zero();
        const uint64_t c1 = c0 + 16 * (uint64_t)tpr < ncop ? c0 + 16 * (uint64_t)tpr : ncop;
        for (uint64_t c = c0; c < c1; c += tpr) {
          const Fr w = ldf(W, (row << n) | c);
          frc_mac(pw, ldf(U, c), w);
          frc_mac(qw, ldf(V, c), w);
        }
        p = fr_add(p, frw_reduce<16>(frc_wide(pw)));
        q = fr_add(q, frw_reduce<16>(frc_wide(qw)));
      }
    }
    __syncthreads();
    sp[threadIdx.x] = p;
    sq[threadIdx.x] = q;
    __syncthreads();
    for (uint32_t s = tpr / 2; s >= 1; s >>= 1) {
      if (lane < s) {
        sp[threadIdx.x] = fr_add(sp[threadIdx.x], sp[threadIdx.x + s]);
        sq[threadIdx.x] = fr_add(sq[threadIdx.x], sq[threadIdx.x + s]);
      }
      __syncthreads();
    }
    if (lane == 0 && row < rows) {
      stf(P<Fr*>(st, 3), row, sp[threadIdx.x]);
      stf(P<Fr*>(st, 4), row, sq[threadIdx.x]);
    }
  }
}

// ST_LOCAL_CONTRACT: column sums over the sub-circuit variables, first stage:
// part[c * R + k] = sum_{y in chunk k} EqR[y] W[y,c] for R = u1 chunks of rows;
// one thread per (column, chunk), tile t = column block (t % xb) and chunk (t / xb).
// p0 W, p1 EqR, p2 part, u0 n, u1 R, q0 rows.
__device__ __forceinline__ void body_local_contract(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ W = P<const Fr*>(st, 0);
  const Fr* __restrict__ EqR = P<const Fr*>(st, 1);
  Fr* __restrict__ part = P<Fr*>(st, 2);
  const uint32_t n = st.u[0], R = st.u[1];
  const uint64_t rows = st.q[0], ncop = 1ull << n;
  const uint64_t xb = (ncop + kBlock - 1) / kBlock;
  for (uint64_t t = tile; t < xb * R; t += ntiles) {
    const uint64_t c = (t % xb) * kBlock + threadIdx.x;
    const uint64_t k = t / xb;
    if (c >= ncop) continue;
    const uint64_t per = (rows + R - 1) / R;
    const uint64_t y0 = k * per, y1 = (y0 + per < rows) ? y0 + per : rows;
    Fr acc = fr_zero();
    for (uint64_t ya = y0; ya < y1; ya += 16) {
      const uint64_t yb = ya + 16 < y1 ? ya + 16 : y1;
      FrCols aw = frc_zero();
      for (uint64_t y = ya; y < yb; ++y) frc_mac(aw, ldf(EqR, y), ldf(W, (y << n) | c));
      acc = fr_add(acc, frw_reduce<16>(frc_wide(aw)));
    }
    stf(part, c * R + k, acc);
  }
}

// ST_COPY_TABLES: the copy tables of phase 2. A column's R partials are summed
// by tpc = min(64, R) lanes of one wave:
// Wc[c] = sum_k part[c*R + k], Fc[c] = U[c] Fa~ + V[c] Fb~, Kc[c] = U[c] Ka~ + V[c] Kb~.
// p0 part, p1 U, p2 V, p3 fa_f, p4 fb_f, p5 S, p6 Wc, p7 Fc, p8 Kc, u0 R, q0 ncop.
__device__ __forceinline__ void body_copy_tables(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ part = P<const Fr*>(st, 0);
  const uint32_t R = st.u[0];
  const uint64_t ncop = st.q[0];
  // tpc lanes (at most a wave) per column, reduced with shuffles inside aligned lane groups
  const uint32_t rlog = 31 - __clz(R);
  const uint32_t tpc_log = rlog < 6 ? rlog : 6;
  const uint32_t tpc = 1u << tpc_log;
  const uint32_t lane = threadIdx.x & (tpc - 1);
  const uint64_t cols_per_tile = kBlock >> tpc_log;
  const DevState* S = P<const DevState*>(st, 5);
  const Fr fa = opaque(*P<const Fr*>(st, 3)), fb = opaque(*P<const Fr*>(st, 4));
  const Fr ka = opaque(S->ka_f), kb = opaque(S->kb_f);
  for (uint64_t base = (uint64_t)tile * cols_per_tile; base < ncop; base += (uint64_t)ntiles * cols_per_tile) {
    const uint64_t c = base + (threadIdx.x >> tpc_log);
    Fr w = fr_zero();
    if (c < ncop)
      for (uint32_t k = lane; k < R; k += tpc) w = fr_add(w, ldf(part, c * R + k));
    for (uint32_t off = tpc / 2; off >= 1; off >>= 1) w = fr_add(w, shfl_xor_fr(w, off));
    if (lane == 0 && c < ncop) {
      const Fr u = ldf(P<const Fr*>(st, 1), c), v = ldf(P<const Fr*>(st, 2), c);
      stf(P<Fr*>(st, 6), c, w);
      stf(P<Fr*>(st, 7), c, fr_mul_add2(u, fa, v, fb));
      stf(P<Fr*>(st, 8), c, fr_mul_add2(u, ka, v, kb));
    }
  }
}

// ST_LOCAL_VALUES: Ka~, Kb~ at the phase-2 sub-circuit point: dot products with
// EqR (one workgroup). p0 EqR, p1 Ka, p2 Kb, p3 S, q0 rows.
__device__ __forceinline__ void body_local_values(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* EqR = P<const Fr*>(st, 0);
  const Fr* Ka = P<const Fr*>(st, 1);
  const Fr* Kb = P<const Fr*>(st, 2);
  Fr acc[2] = {fr_zero(), fr_zero()};
  // lazy sums: at most 16 unreduced products per column accumulator
  const uint64_t stride = (uint64_t)ntiles * kBlock;
  for (uint64_t y0 = (uint64_t)tile * kBlock + threadIdx.x; y0 < st.q[0]; y0 += 16 * stride) {
    FrCols a = frc_zero(), b = frc_zero();
    const uint64_t y1 = y0 + 16 * stride < st.q[0] ? y0 + 16 * stride : st.q[0];
    for (uint64_t y = y0; y < y1; y += stride) {
      const Fr e = ldf(EqR, y);
      frc_mac(a, e, ldf(Ka, y));
      frc_mac(b, e, ldf(Kb, y));
    }
    acc[0] = fr_add(acc[0], frw_reduce<16>(frc_wide(a)));
    acc[1] = fr_add(acc[1], frw_reduce<16>(frc_wide(b)));
  }
  write_partial<2>(acc, P<Fr*>(st, 4), tile);
}
__device__ __forceinline__ void finish_local_values(const Step& st, uint32_t ntiles) {
  Fr tot[2];
  sum_partials<2>(P<const Fr*>(st, 4), ntiles, tot);
  if (threadIdx.x == 0) {
    DevState* S = P<DevState*>(st, 3);
    S->ka_f = tot[0];
    S->kb_f = tot[1];
  }
}

// ST_STATE_EXPORT / ST_STATE_IMPORT: transcript state bytes <-> device state.
// p0 S, p1 32-byte buffer.
__device__ __forceinline__ void body_state_export(const Step& st, uint32_t, uint32_t) {
  const DevState* S = P<const DevState*>(st, 0);
  uint8_t* out = P<uint8_t*>(st, 1);
  if (threadIdx.x < 8) {
    const uint32_t h = S->st[threadIdx.x];
    out[4 * threadIdx.x + 0] = (uint8_t)(h >> 24);
    out[4 * threadIdx.x + 1] = (uint8_t)(h >> 16);
    out[4 * threadIdx.x + 2] = (uint8_t)(h >> 8);
    out[4 * threadIdx.x + 3] = (uint8_t)h;
  }
}
__device__ __forceinline__ void body_state_import(const Step& st, uint32_t, uint32_t) {
  DevState* S = P<DevState*>(st, 0);
  const uint8_t* in = P<const uint8_t*>(st, 1);
  if (threadIdx.x < 8) {
    const uint8_t* b = in + 4 * threadIdx.x;
    S->st[threadIdx.x] = ((uint32_t)b[0] << 24) | ((uint32_t)b[1] << 16) | ((uint32_t)b[2] << 8) | b[3];
  }
  if (threadIdx.x == 0) {
    S->counter = 0;
    S->pending = 0;
  }
}

#undef GTID
#undef GSTRIDE

// Runs tile `tile` of a step; for reduction steps the last tile (by the
// counter in the proof's state) also runs the finisher. Used by the batch kernel.
__device__ __forceinline__ void run_step_tile(const Step& st, uint32_t tile, uint32_t ntiles) {
  uint32_t* counter = nullptr;
  switch (st.type) {
    case ST_WSUM: counter = &P<DevState*>(st, 4)->counter; break;
    case ST_P1_INIT_ROUND: counter = &P<DevState*>(st, 9)->counter; break;
    case ST_ROUND_A: counter = &P<DevState*>(st, RoundPtrs<3>::kS)->counter; break;
    case ST_ROUND_B: counter = &P<DevState*>(st, RoundPtrs<5>::kS)->counter; break;
    case ST_LOCAL_VALUES: counter = &P<DevState*>(st, 3)->counter; break;
    default: break;
  }
  switch (st.type) {
    case ST_TO_MONT: body_to_mont(st, tile, ntiles); break;
    case ST_FROM_MONT: body_from_mont(st, tile, ntiles); break;
    case ST_FORWARD: body_forward(st, tile, ntiles); break;
    case ST_DIGEST: body_digest(st, tile, ntiles); break;
    case ST_TRANSCRIPT_BEGIN: body_transcript_begin(st, tile, ntiles); break;
    case ST_SQUEEZE: body_squeeze(st, tile, ntiles); break;
    case ST_LAYER_BEGIN: body_layer_begin(st, tile, ntiles); break;
    case ST_EQ: body_eq(st, tile, ntiles); break;
    case ST_WSUM:
      body_wsum(st, tile, ntiles);
      if (last_tile(counter, ntiles)) finish_wsum(st, ntiles);
      break;
    case ST_P1_INIT: body_p1_init(st, tile, ntiles); break;
    case ST_P1_INIT_ROUND:
      body_p1_init_round<false>(st, tile, ntiles);
      if (last_tile(counter, ntiles)) finish_p1_init_round(st, ntiles);
      break;
    case ST_ROUND_A:
      body_round<FormA>(st, tile, ntiles);
      if (last_tile(counter, ntiles)) finish_round_step<FormA>(st, ntiles);
      break;
    case ST_ROUND_B:
      body_round<FormB>(st, tile, ntiles);
      if (last_tile(counter, ntiles)) finish_round_step<FormB>(st, ntiles);
      break;
    case ST_TAIL_A: body_tail<FormA>(st, tile, ntiles); break;
    case ST_TAIL_B: body_tail<FormB>(st, tile, ntiles); break;
    case ST_COPY_WEIGHTS: body_copy_weights(st, tile, ntiles); break;
    case ST_P2_TABLES: body_p2_tables(st, tile, ntiles); break;
    case ST_COPY_CONTRACT: body_copy_contract(st, tile, ntiles); break;
    case ST_LOCAL_CONTRACT: body_local_contract(st, tile, ntiles); break;
    case ST_COPY_TABLES: body_copy_tables(st, tile, ntiles); break;
    case ST_LOCAL_VALUES:
      body_local_values(st, tile, ntiles);
      if (last_tile(counter, ntiles)) finish_local_values(st, ntiles);
      break;
    case ST_STATE_EXPORT: body_state_export(st, tile, ntiles); break;
    case ST_STATE_IMPORT: body_state_import(st, tile, ntiles); break;
    default: break;
  }
}

}  // namespace gkr
