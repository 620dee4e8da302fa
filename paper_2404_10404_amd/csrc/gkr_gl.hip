// The layered data-parallel prover over the Goldilocks field (Section 4.1,
// the field choice), for gfx950: kernels, the proof program and the C ABI.
//
// The protocol is the BN254 prover's (GKR layer relation, Libra's two-phase
// product sumcheck, claims combined with squeezed alpha and beta, bits bound
// from the most significant, copies in the low bits) with 8-byte canonical
// elements and this field's transcript rules:
//   accept         v = LE64(digest bytes 0..7); rehash with "GKRC" while v >= p
//   round(e0, e2)  one compression of LE64(e0) || LE64(e2) || 47 zero bytes || 0x01
//   values         vx, vy absorbed with "GKRV" as 8 bytes
// Elements are 8 bytes, so a wave's load of 64 consecutive entries is 512
// bytes; a product is four 32 x 32 multiplies and the reduction of gl.hpp.
// The kernels are written plainly (one kernel per step type, serial round
// finishers, phase-2 tables materialised over the whole layer): the BN254
// prover's factored phase 2 and two-chain finishers are not repeated here.
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gkr_bodies.hpp"
#include "gkr_gl.hpp"
#include "gkr_profile.hpp"
#include "gkr_program.hpp"
#include "gkr_tuning.hpp"
#include "gl.hpp"

namespace gkr {

// ---------------------------------------------------------------- device helpers

typedef __attribute__((address_space(1))) uint64_t GlobalU64;

__device__ __forceinline__ uint64_t gld(const uint64_t* p, uint64_t i) { return ((const GlobalU64*)p)[i]; }
__device__ __forceinline__ void gst(uint64_t* p, uint64_t i, uint64_t v) { ((GlobalU64*)p)[i] = v; }

// Two adjacent elements (i even) as one 16-byte access.
typedef uint64_t U64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) U64x2 GlobalU64x2;
__device__ __forceinline__ U64x2 gld2(const uint64_t* p, uint64_t i) { return *(const GlobalU64x2*)(p + i); }
__device__ __forceinline__ void gst2(uint64_t* p, uint64_t i, U64x2 v) { *(GlobalU64x2*)(p + i) = v; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask) {
  const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)v, mask, 64);
  const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(v >> 32), mask, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Sum of NV values over the workgroup (blockDim.x a multiple of 64); valid in thread 0.
template <int NV>
__device__ void gl_block_sum(uint64_t (&v)[NV]) {
  __shared__ uint64_t red[NV][16];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = gl_add(v[k], shfl_xor_u64(v[k], off));
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      uint64_t a = red[k][0];
      for (uint32_t w = 1; w < nw; ++w) a = gl_add(a, red[k][w]);
      v[k] = a;
    }
  __syncthreads();
}

// ---------------------------------------------------------------- transcript (device)

__device__ __forceinline__ uint64_t gl_candidate(const Sha256State& s) {
  return (uint64_t)bswap32(s.h[0]) | ((uint64_t)bswap32(s.h[1]) << 32);
}

__device__ uint64_t gl_accept(Sha256State& st) {
  uint64_t v = gl_candidate(st);
  for (int attempt = 0; attempt < 4096 && v >= kGlP; ++attempt) {
    uint32_t w[9];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = st.h[k];
    w[8] = kTagChallenge;
    st = sha256_fixed<9>(w);
    v = gl_candidate(st);
  }
  return v;
}

__device__ uint64_t gl_squeeze(Sha256State& st) {
  uint32_t w[9];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = kTagChallenge;
  st = sha256_fixed<9>(w);
  return gl_accept(st);
}

__device__ void gl_absorb_value(Sha256State& st, uint64_t v) {
  uint32_t w[11];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = kTagValue;
  w[9] = bswap32((uint32_t)v);
  w[10] = bswap32((uint32_t)(v >> 32));
  st = sha256_fixed<11>(w);
}

__device__ uint64_t gl_round_hash(Sha256State& st, uint64_t e0, uint64_t e2) {
  Sha256Block blk;
#pragma unroll
  for (int k = 0; k < 16; ++k) blk.w[k] = 0;
  blk.w[0] = bswap32((uint32_t)e0);
  blk.w[1] = bswap32((uint32_t)(e0 >> 32));
  blk.w[2] = bswap32((uint32_t)e2);
  blk.w[3] = bswap32((uint32_t)(e2 >> 32));
  blk.w[15] = 1u;
  st = sha256_compress_v(st, blk);
  return gl_accept(st);
}

__device__ __forceinline__ Sha256State gl_load_state(const GlState* S) {
  Sha256State s;
#pragma unroll
  for (int k = 0; k < 8; ++k) s.h[k] = S->st[k];
  return s;
}
__device__ __forceinline__ void gl_save_state(GlState* S, const Sha256State& s) {
#pragma unroll
  for (int k = 0; k < 8; ++k) S->st[k] = s.h[k];
}

// SHA-256 of `len` 32-bit words (byte-swapped when swap: element words are
// little-endian) with the standard padding.
__device__ void sha256_words(const uint32_t* in, uint64_t len, int swap, uint32_t* out) {
  Sha256State sh = sha256_iv();
  const uint64_t full = len / 16;
  for (uint64_t b = 0; b < full; ++b) {
    Sha256Block blk;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const uint32_t v = in[b * 16 + i];
      blk.w[i] = swap ? bswap32(v) : v;
    }
    sh = sha256_compress_v(sh, blk);
  }
  const uint32_t rem = (uint32_t)(len - full * 16);
  Sha256Block blk;
#pragma unroll
  for (int i = 0; i < 16; ++i) blk.w[i] = 0;
  for (uint32_t i = 0; i < rem; ++i) {
    const uint32_t v = in[full * 16 + i];
    blk.w[i] = swap ? bswap32(v) : v;
  }
  blk.w[rem] = 0x80000000u;
  const uint64_t bits = len * 32;
  if (rem <= 13) {
    blk.w[14] = (uint32_t)(bits >> 32);
    blk.w[15] = (uint32_t)bits;
    sh = sha256_compress_v(sh, blk);
  } else {
    sh = sha256_compress_v(sh, blk);
#pragma unroll
    for (int i = 0; i < 16; ++i) blk.w[i] = 0;
    blk.w[14] = (uint32_t)(bits >> 32);
    blk.w[15] = (uint32_t)bits;
    sh = sha256_compress_v(sh, blk);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) out[k] = sh.h[k];
}

// ---------------------------------------------------------------- bodies

#define GTID ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x)
#define GSTRIDE ((uint64_t)gridDim.x * blockDim.x)

// ST_GL_FORWARD: V[z*2^n + c] = W[x_z*2^n + c] (+ or *) W[y_z*2^n + c].
// p0 W, p1 V, p2 gate records (x | type << 31, y), u0 n, q0 count.
__global__ void __launch_bounds__(kBlock) k_gl_forward(Step st) {
  const uint64_t* __restrict__ W = P<const uint64_t*>(st, 0);
  uint64_t* __restrict__ V = P<uint64_t*>(st, 1);
  const uint2* __restrict__ gates = P<const uint2*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t g = GTID; g < st.q[0]; g += GSTRIDE) {
    const uint2 gate = gates[g >> n];
    const uint64_t c = g & mask;
    const uint64_t a = gld(W, ((uint64_t)(gate.x & 0x7fffffffu) << n) | c), b = gld(W, ((uint64_t)gate.y << n) | c);
    gst(V, g, (gate.x >> 31) ? gl_mul(a, b) : gl_add(a, b));
  }
}

// ST_GL_DIGEST: one level of a tree digest; chunk t (256 words) hashed by thread t.
// p0 in, p1 out, q0 nwords, q1 nchunks, u0 swap.
__global__ void __launch_bounds__(kBlock) k_gl_digest(Step st) {
  const uint32_t* in = P<const uint32_t*>(st, 0);
  uint32_t* out = P<uint32_t*>(st, 1);
  const uint64_t nwords = st.q[0];
  for (uint64_t t = GTID; t < st.q[1]; t += GSTRIDE) {
    const uint64_t begin = t * kChunkWords;
    const uint64_t end = (begin + kChunkWords < nwords) ? begin + kChunkWords : nwords;
    sha256_words(in + begin, end - begin, st.u[0], out + 8 * t);
  }
}

// ST_GL_BEGIN: st = seed state (w0..7), absorb the circuit digest (w8..15) and
// the two vector digests; the reduction counter starts at zero.
// p0 S, p1 dig_in, p2 dig_out.
__global__ void __launch_bounds__(kBlock) k_gl_begin(Step st) {
  if (threadIdx.x != 0) return;
  GlState* S = P<GlState*>(st, 0);
  Sha256State sh;
#pragma unroll
  for (int k = 0; k < 8; ++k) sh.h[k] = st.w[k];
  absorb_digest(sh, st.w + 8);
  absorb_digest(sh, P<const uint32_t*>(st, 1));
  absorb_digest(sh, P<const uint32_t*>(st, 2));
  gl_save_state(S, sh);
  S->counter = 0;
}

// ST_GL_SQUEEZE: u0 challenges into p1. p0 S.
__global__ void __launch_bounds__(kBlock) k_gl_squeeze(Step st) {
  if (threadIdx.x != 0) return;
  GlState* S = P<GlState*>(st, 0);
  uint64_t* out = P<uint64_t*>(st, 1);
  Sha256State sh = gl_load_state(S);
  for (uint32_t k = 0; k < st.u[0]; ++k) out[k] = gl_squeeze(sh);
  gl_save_state(S, sh);
}

// ST_GL_LAYER_BEGIN: alpha, beta squeezed (u0 = 0) and claim = alpha vu + beta vv;
// on layer 0 (u0 = 1) alpha = 1, beta = 0, claim = vu. p0 S, p1 vu, p2 vv.
__global__ void __launch_bounds__(kBlock) k_gl_layer_begin(Step st) {
  if (threadIdx.x != 0) return;
  GlState* S = P<GlState*>(st, 0);
  const uint64_t vu = *P<const uint64_t*>(st, 1), vv = *P<const uint64_t*>(st, 2);
  if (st.u[0]) {
    S->alpha = 1;
    S->beta = 0;
    S->claim = vu;
    return;
  }
  Sha256State sh = gl_load_state(S);
  const uint64_t a = gl_squeeze(sh), b = gl_squeeze(sh);
  gl_save_state(S, sh);
  S->alpha = a;
  S->beta = b;
  S->claim = gl_add(gl_mul(a, vu), gl_mul(b, vv));
}

// ST_GL_EQ: up to four tables out_j[b] = scale_j prod_k (bit_k(b) ? r_k : 1 - r_k),
// bit 1 the most significant. u0..3 bits, u4 count; p0..3 points, p4..7 scales
// (null = 1), p8..11 outs.
__global__ void __launch_bounds__(kBlock) k_gl_eq(Step st) {
  uint64_t total = 0;
  for (uint32_t j = 0; j < st.u[4]; ++j) total += 1ull << st.u[j];
  for (uint64_t g = GTID; g < total; g += GSTRIDE) {
    uint64_t t = g;
    uint32_t j = 0;
    while (t >= (1ull << st.u[j])) {
      t -= 1ull << st.u[j];
      ++j;
    }
    const uint64_t* r = P<const uint64_t*>(st, j);
    const int k = st.u[j];
    const uint64_t* scale = P<const uint64_t*>(st, 4 + j);
    uint64_t acc = scale ? *scale : 1;
    for (int i = 0; i < k; ++i) {
      const uint64_t ri = r[i];
      acc = gl_mul(acc, ((t >> (k - 1 - i)) & 1) ? ri : gl_one_minus(ri));
    }
    gst(P<uint64_t*>(st, 8 + j), t, acc);
  }
}

// Publishes this tile's partials and counts it; true in every thread of the last tile.
__device__ __forceinline__ bool gl_last_tile(uint32_t* counter, uint32_t ntiles) { return last_tile(counter, ntiles); }

// ST_GL_WSUM: sum_e V[e] A[e >> n] B[e & mask] into *p5.
// p0 V, p1 A, p2 B, p3 partials, p4 S, p5 dst, u0 n, q0 count.
__global__ void __launch_bounds__(kBlock) k_gl_wsum(Step st) {
  const uint64_t* V = P<const uint64_t*>(st, 0);
  const uint64_t* A = P<const uint64_t*>(st, 1);
  const uint64_t* B = P<const uint64_t*>(st, 2);
  uint64_t* partials = P<uint64_t*>(st, 3);
  GlState* S = P<GlState*>(st, 4);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  uint64_t acc[1] = {0};
  for (uint64_t e = GTID; e < st.q[0]; e += GSTRIDE)
    acc[0] = gl_add(acc[0], gl_mul(gl_mul(gld(V, e), gld(A, e >> n)), gld(B, e & mask)));
  gl_block_sum<1>(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc[0];
  if (gl_last_tile(&S->counter, gridDim.x)) {
    uint64_t tot[1] = {0};
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += blockDim.x) tot[0] = gl_add(tot[0], partials[b]);
    gl_block_sum<1>(tot);
    if (threadIdx.x == 0) *P<uint64_t*>(st, 5) = tot[0];
  }
}

// ST_GL_P1: phase-1 tables over (x, c), T[z,c] = aU[z] Cu[c] + bV[z] Cv[c]:
//   G[x,c] = sum_{MUL z: x_z=x} T W[y_z,c] + sum_{ADD z: x_z=x} T,  H[x,c] = sum_{ADD} T W[y_z,c].
// p0 W, p1 G, p2 H, p3 xrow, p4 xent (z, y | type << 31), p5 aU, p6 bV, p7 Cu, p8 Cv, u0 n, q0 count.
__global__ void __launch_bounds__(kBlock) k_gl_p1(Step st) {
  const uint64_t* __restrict__ W = P<const uint64_t*>(st, 0);
  uint64_t* __restrict__ G = P<uint64_t*>(st, 1);
  uint64_t* __restrict__ H = P<uint64_t*>(st, 2);
  const uint32_t* __restrict__ xrow = P<const uint32_t*>(st, 3);
  const uint2* __restrict__ xent = P<const uint2*>(st, 4);
  const uint64_t *aU = P<const uint64_t*>(st, 5), *bV = P<const uint64_t*>(st, 6);
  const uint64_t *Cu = P<const uint64_t*>(st, 7), *Cv = P<const uint64_t*>(st, 8);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t e = GTID; e < st.q[0]; e += GSTRIDE) {
    const uint64_t x = e >> n, c = e & mask;
    const uint64_t cu = gld(Cu, c), cv = gld(Cv, c);
    uint64_t g = 0, h = 0;
    const uint32_t k1 = xrow[x + 1];
    for (uint32_t k = xrow[x]; k < k1; ++k) {
      const uint2 r = xent[k];
      const uint64_t T = gl_add(gl_mul(gld(aU, r.x), cu), gl_mul(gld(bV, r.x), cv));
      const uint64_t tw = gl_mul(T, gld(W, ((uint64_t)(r.y & 0x7fffffffu) << n) | c));
      if (r.y >> 31) {
        g = gl_add(g, tw);
      } else {
        g = gl_add(g, T);
        h = gl_add(h, tw);
      }
    }
    gst(G, e, g);
    gst(H, e, h);
  }
}

// ---------------------------------------------------------------- phase 2
//
// Phase 2 sums W[y,c] F[y,c] + K[y,c] over (y, c). With the copy weights
// U[c] = EC[c] Cu[c], V[c] = EC[c] Cv[c] both tables have rank 2 per copy:
//   F[y,c] = U[c] Fa[y] + V[c] Fb[y],  K[y,c] = U[c] Ka[y] + V[c] Kb[y],
//   Fa = vx Mu + Au, Fb = vx Mv + Av, Ka = vx Au, Kb = vx Av, where
//   Mu[y] = sum_{MUL z: y_z = y} aU[z] EL[x_z] (Mv with bV; Au, Av over ADD gates).
// The sub-circuit rounds therefore run on the 2^sigma tables
//   sum_y P[y] Fa[y] + Q[y] Fb[y] + Ks[y],  P = sum_c U[c] W[., c], Q = sum_c V[c] W[., c],
//   Ks = su Ka + sv Kb (su = sum_c U[c], sv = sum_c V[c]),
// and the copy rounds on Wc[c] = W(ry_local, c), Fc[c] = U[c] Fa~ + V[c] Fb~,
// Kc[c] = U[c] Ka~ + V[c] Kb~: the same round polynomials as over the whole
// layer, with two passes over W instead of a pass per round.

// ST_GL_COPY_WEIGHTS (one workgroup): U = EC Cu, V = EC Cv for c < q0, and
// their sums into S->su, S->sv. p0 EC, p1 Cu, p2 Cv, p3 U, p4 V, p5 S.
__global__ void __launch_bounds__(kBlock) k_gl_copy_weights(Step st) {
  const uint64_t *EC = P<const uint64_t*>(st, 0), *Cu = P<const uint64_t*>(st, 1), *Cv = P<const uint64_t*>(st, 2);
  uint64_t *U = P<uint64_t*>(st, 3), *V = P<uint64_t*>(st, 4);
  GlState* S = P<GlState*>(st, 5);
  uint64_t acc[2] = {0, 0};
  for (uint64_t c = threadIdx.x; c < st.q[0]; c += blockDim.x) {
    const uint64_t e = gld(EC, c);
    const uint64_t u = gl_mul(e, gld(Cu, c)), v = gl_mul(e, gld(Cv, c));
    gst(U, c, u);
    gst(V, c, v);
    acc[0] = gl_add(acc[0], u);
    acc[1] = gl_add(acc[1], v);
  }
  gl_block_sum<2>(acc);
  if (threadIdx.x == 0) {
    S->su = acc[0];
    S->sv = acc[1];
  }
}

// ST_GL_P2T: the 2^sigma phase-2 tables for y < q0 from the wiring by y.
// p0 yrow, p1 yent (z, x | type << 31), p2 aU, p3 bV, p4 EL, p5 S,
// p6 Fa, p7 Fb, p8 Ka, p9 Kb, p10 Ks.
__global__ void __launch_bounds__(kBlock) k_gl_p2t(Step st) {
  const uint32_t* __restrict__ yrow = P<const uint32_t*>(st, 0);
  const uint2* __restrict__ yent = P<const uint2*>(st, 1);
  const uint64_t *aU = P<const uint64_t*>(st, 2), *bV = P<const uint64_t*>(st, 3), *EL = P<const uint64_t*>(st, 4);
  const GlState* S = P<const GlState*>(st, 5);
  const uint64_t vx = S->vx, su = S->su, sv = S->sv;
  for (uint64_t y = GTID; y < st.q[0]; y += GSTRIDE) {
    uint64_t mu = 0, mv = 0, au = 0, av = 0;
    const uint32_t k1 = yrow[y + 1];
    for (uint32_t k = yrow[y]; k < k1; ++k) {
      const uint2 r = yent[k];
      const uint64_t e = gld(EL, r.y & 0x7fffffffu);
      const uint64_t tu = gl_mul(gld(aU, r.x), e), tv = gl_mul(gld(bV, r.x), e);
      if (r.y >> 31) {
        mu = gl_add(mu, tu);
        mv = gl_add(mv, tv);
      } else {
        au = gl_add(au, tu);
        av = gl_add(av, tv);
      }
    }
    const uint64_t ka = gl_mul(vx, au), kb = gl_mul(vx, av);
    gst(P<uint64_t*>(st, 6), y, gl_add(gl_mul(vx, mu), au));
    gst(P<uint64_t*>(st, 7), y, gl_add(gl_mul(vx, mv), av));
    gst(P<uint64_t*>(st, 8), y, ka);
    gst(P<uint64_t*>(st, 9), y, kb);
    gst(P<uint64_t*>(st, 10), y, gl_add(gl_mul(su, ka), gl_mul(sv, kb)));
  }
}

// Sum over the wave; valid in every lane.
__device__ __forceinline__ uint64_t gl_wave_sum(uint64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = gl_add(v, shfl_xor_u64(v, off));
  return v;
}

// ST_GL_COPY_CONTRACT: P[y] = sum_c U[c] W[y 2^n + c], Q[y] likewise with V,
// one wave per row y < q0. p0 W, p1 U, p2 V, p3 P, p4 Q, u0 n.
__global__ void __launch_bounds__(kBlock) k_gl_copy_contract(Step st) {
  const uint64_t *W = P<const uint64_t*>(st, 0), *U = P<const uint64_t*>(st, 1), *V = P<const uint64_t*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t ncop = 1ull << n;
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t wave = GTID >> 6, nwaves = GSTRIDE >> 6;
  for (uint64_t y = wave; y < st.q[0]; y += nwaves) {
    uint64_t p = 0, q = 0;
    for (uint64_t c = lane; c < ncop; c += 64) {
      const uint64_t w = gld(W, (y << n) | c);
      p = gl_add(p, gl_mul(gld(U, c), w));
      q = gl_add(q, gl_mul(gld(V, c), w));
    }
    p = gl_wave_sum(p);
    q = gl_wave_sum(q);
    if (lane == 0) {
      gst(P<uint64_t*>(st, 3), y, p);
      gst(P<uint64_t*>(st, 4), y, q);
    }
  }
}

// ST_GL_LOCAL_VALUES (one workgroup): Ka~ = sum_y EqR[y] Ka[y], Kb~ likewise,
// y < q0, into S->ka_f, S->kb_f. p0 EqR, p1 Ka, p2 Kb, p3 S.
__global__ void __launch_bounds__(kBlock) k_gl_local_values(Step st) {
  const uint64_t *E = P<const uint64_t*>(st, 0), *Ka = P<const uint64_t*>(st, 1), *Kb = P<const uint64_t*>(st, 2);
  GlState* S = P<GlState*>(st, 3);
  uint64_t acc[2] = {0, 0};
  for (uint64_t y = threadIdx.x; y < st.q[0]; y += blockDim.x) {
    const uint64_t e = gld(E, y);
    acc[0] = gl_add(acc[0], gl_mul(e, gld(Ka, y)));
    acc[1] = gl_add(acc[1], gl_mul(e, gld(Kb, y)));
  }
  gl_block_sum<2>(acc);
  if (threadIdx.x == 0) {
    S->ka_f = acc[0];
    S->kb_f = acc[1];
  }
}

// ST_GL_LOCAL_CONTRACT: part[ch 2^n + c] = sum over the 2^u1 rows y of chunk
// ch of EqR[y] W[y 2^n + c], for ch 2^n + c < q0. p0 W, p1 EqR, p2 part, u0 n.
__global__ void __launch_bounds__(kBlock) k_gl_local_contract(Step st) {
  const uint64_t *W = P<const uint64_t*>(st, 0), *E = P<const uint64_t*>(st, 1);
  uint64_t* part = P<uint64_t*>(st, 2);
  const uint32_t n = st.u[0], lr = st.u[1];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t g = GTID; g < st.q[0]; g += GSTRIDE) {
    const uint64_t ch = g >> n, c = g & mask;
    const uint64_t y0 = ch << lr, y1 = y0 + (1ull << lr);
    uint64_t acc = 0;
    for (uint64_t y = y0; y < y1; ++y) acc = gl_add(acc, gl_mul(gld(E, y), gld(W, (y << n) | c)));
    gst(part, g, acc);
  }
}

// ST_GL_COPY_TABLES: for c < q0, Wc[c] = sum of the u0 chunk partials,
// Fc = U Fa~ + V Fb~, Kc = U Ka~ + V Kb~ (Fa~, Fb~ the first entries of the
// folded Fa, Fb tables). p0 part, p1 U, p2 V, p3 Fa, p4 Fb, p5 S, p6 Wc, p7 Fc, p8 Kc.
// tpc lanes (up to a wave) per column, summed with shuffles inside aligned
// lane groups: few copies come with many chunks.
__global__ void __launch_bounds__(kBlock) k_gl_copy_tables(Step st) {
  const uint64_t* part = P<const uint64_t*>(st, 0);
  const uint64_t *U = P<const uint64_t*>(st, 1), *V = P<const uint64_t*>(st, 2);
  const uint64_t fa = *P<const uint64_t*>(st, 3), fb = *P<const uint64_t*>(st, 4);
  const GlState* S = P<const GlState*>(st, 5);
  const uint64_t ka = S->ka_f, kb = S->kb_f, ncop = st.q[0];
  const uint32_t R = st.u[0];
  const uint32_t rlog = 31 - __clz(R);
  const uint32_t tpc_log = rlog < 6 ? rlog : 6;
  const uint32_t tpc = 1u << tpc_log, lane = threadIdx.x & (tpc - 1);
  const uint64_t cols_per_tile = kBlock >> tpc_log;
  const uint32_t tile = blockIdx.x, ntiles = gridDim.x;
  for (uint64_t base = (uint64_t)tile * cols_per_tile; base < ncop; base += (uint64_t)ntiles * cols_per_tile) {
    const uint64_t c = base + (threadIdx.x >> tpc_log);
    uint64_t w = 0;
    if (c < ncop)
      for (uint32_t ch = lane; ch < R; ch += tpc) w = gl_add(w, gld(part, (uint64_t)ch * ncop + c));
    for (uint32_t off = tpc / 2; off >= 1; off >>= 1) {
      const uint64_t o = ((uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)(w >> 32), off, 64) << 32) |
                         (uint32_t)__shfl_xor((int)(uint32_t)w, off, 64);
      w = gl_add(w, o);
    }
    if (lane == 0 && c < ncop) {
      const uint64_t u = gld(U, c), v = gld(V, c);
      gst(P<uint64_t*>(st, 6), c, w);
      gst(P<uint64_t*>(st, 7), c, gl_add(gl_mul(u, fa), gl_mul(v, fb)));
      gst(P<uint64_t*>(st, 8), c, gl_add(gl_mul(u, ka), gl_mul(v, kb)));
    }
  }
}

// ---------------------------------------------------------------- rounds

// The transcript step of a round (one thread): message (e0, e1 = claim - e0,
// e2) to the proof, the hash gives r, the claim moves to the round polynomial at r.
__device__ __forceinline__ uint64_t gl_round_step(GlState* S, uint64_t e0, uint64_t e2, uint64_t* msg) {
  const uint64_t e1 = gl_sub(S->claim, e0);
  msg[0] = e0;
  msg[1] = e1;
  msg[2] = e2;
  Sha256State sh = gl_load_state(S);
  const uint64_t r = gl_round_hash(sh, e0, e2);
  gl_save_state(S, sh);
  S->claim = gl_interp3(e0, e1, e2, r);
  return r;
}

// The summand of a round over NT tables at one point: T0 T1 + T2 (NT = 3) or
// T0 T1 + T2 T3 + T4 (NT = 5).
template <int NT>
__device__ __forceinline__ uint64_t gl_form(const uint64_t (&v)[NT]) {
  if constexpr (NT == 3) return gl_add(gl_mul(v[0], v[1]), v[2]);
  else return gl_add(gl_add(gl_mul(v[0], v[1]), gl_mul(v[2], v[3])), v[4]);
}

// Evaluation of pair b of NT tables at t = 0 and t = 2, after an optional
// fold of the source by r (entry i of the folded table is
// src[i] + r (src[i + 2 half] - src[i])).
template <int NT>
__device__ __forceinline__ void gl_pair(const uint64_t* const* src, uint64_t* const* dst, bool fold, uint64_t r,
                                        uint64_t b, uint64_t half, uint64_t& acc0, uint64_t& acc2) {
  uint64_t lo[NT], hi[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    if (fold) {
      const uint64_t m = 2 * half;
      const uint64_t a0 = gld(src[k], b), a1 = gld(src[k], b + m);
      const uint64_t b0 = gld(src[k], b + half), b1 = gld(src[k], b + half + m);
      lo[k] = gl_add(a0, gl_mul(r, gl_sub(a1, a0)));
      hi[k] = gl_add(b0, gl_mul(r, gl_sub(b1, b0)));
      gst(dst[k], b, lo[k]);
      gst(dst[k], b + half, hi[k]);
    } else {
      lo[k] = gld(src[k], b);
      hi[k] = gld(src[k], b + half);
    }
  }
  acc0 = gl_add(acc0, gl_form<NT>(lo));
  uint64_t t2[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) t2[k] = gl_sub(gl_double(hi[k]), lo[k]);
  acc2 = gl_add(acc2, gl_form<NT>(t2));
}

// Pairs b and b + 1 (b even, half even) of NT tables: gl_pair for both, with
// 16-byte loads and stores.
template <int NT>
__device__ __forceinline__ void gl_pair2(const uint64_t* const* src, uint64_t* const* dst, bool fold, uint64_t r,
                                         uint64_t b, uint64_t half, uint64_t& acc0, uint64_t& acc2) {
  uint64_t lo[2][NT], hi[2][NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    if (fold) {
      const uint64_t m = 2 * half;
      const U64x2 a0 = gld2(src[k], b), a1 = gld2(src[k], b + m);
      const U64x2 b0 = gld2(src[k], b + half), b1 = gld2(src[k], b + half + m);
      lo[0][k] = gl_add(a0.x, gl_mul(r, gl_sub(a1.x, a0.x)));
      lo[1][k] = gl_add(a0.y, gl_mul(r, gl_sub(a1.y, a0.y)));
      hi[0][k] = gl_add(b0.x, gl_mul(r, gl_sub(b1.x, b0.x)));
      hi[1][k] = gl_add(b0.y, gl_mul(r, gl_sub(b1.y, b0.y)));
      gst2(dst[k], b, U64x2{lo[0][k], lo[1][k]});
      gst2(dst[k], b + half, U64x2{hi[0][k], hi[1][k]});
    } else {
      const U64x2 a = gld2(src[k], b), c = gld2(src[k], b + half);
      lo[0][k] = a.x;
      lo[1][k] = a.y;
      hi[0][k] = c.x;
      hi[1][k] = c.y;
    }
  }
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    acc0 = gl_add(acc0, gl_form<NT>(lo[e]));
    uint64_t t2[NT];
#pragma unroll
    for (int k = 0; k < NT; ++k) t2[k] = gl_sub(gl_double(hi[e][k]), lo[e][k]);
    acc2 = gl_add(acc2, gl_form<NT>(t2));
  }
}

// ST_GL_ROUND (NT = 3) / ST_GL_ROUND5 (NT = 5): one grid-wide round of the
// NT-table sum (optional fold by the previous challenge, evaluation at
// t = 0, 2), then in the last tile the round's transcript step. p0..p(NT-1)
// src, pNT..p(2NT-1) dst, then (from B = 2 NT) pB rprev (null: no fold),
// pB+1 S, pB+2 partials, pB+3 r_out, pB+4 msg; q0 half.
template <int NT>
__global__ void __launch_bounds__(kBlock) k_gl_round(Step st) {
  constexpr int B = 2 * NT;
  const uint64_t* src[NT];
  uint64_t* dst[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    src[k] = P<const uint64_t*>(st, k);
    dst[k] = P<uint64_t*>(st, NT + k);
  }
  const uint64_t* rprev = P<const uint64_t*>(st, B);
  GlState* S = P<GlState*>(st, B + 1);
  uint64_t* partials = P<uint64_t*>(st, B + 2);
  const bool fold = rprev != nullptr;
  const uint64_t r = fold ? *rprev : 0;
  const uint64_t half = st.q[0];
  uint64_t acc[2] = {0, 0};
  if ((half & 1) == 0) {
    for (uint64_t b = 2 * GTID; b < half; b += 2 * GSTRIDE) gl_pair2<NT>(src, dst, fold, r, b, half, acc[0], acc[1]);
  } else {
    for (uint64_t b = GTID; b < half; b += GSTRIDE) gl_pair<NT>(src, dst, fold, r, b, half, acc[0], acc[1]);
  }
  gl_block_sum<2>(acc);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = acc[0];
    partials[2 * blockIdx.x + 1] = acc[1];
  }
  if (gl_last_tile(&S->counter, gridDim.x)) {
    uint64_t tot[2] = {0, 0};
    for (uint32_t b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
      tot[0] = gl_add(tot[0], partials[2 * b]);
      tot[1] = gl_add(tot[1], partials[2 * b + 1]);
    }
    gl_block_sum<2>(tot);
    if (threadIdx.x == 0) *P<uint64_t*>(st, B + 3) = gl_round_step(S, tot[0], tot[1], P<uint64_t*>(st, B + 4));
  }
}

// ST_GL_TAIL / ST_GL_TAIL5: the remaining u0 rounds in one workgroup, then
// the final fold; the final value of table 0 goes to *final_out and, when
// proof_value is not null, to the proof and into the transcript. q0 = table
// size before the pending fold (if any). p0..p(NT-1) src, pNT..p(2NT-1) dst,
// then (from B = 2 NT) pB rpending, pB+1 S, pB+2 r_out, pB+3 msg,
// pB+4 final_out, pB+5 proof_value.
template <int NT>
__global__ void __launch_bounds__(kBlock) k_gl_tail(Step st) {
  constexpr int B = 2 * NT;
  const uint64_t* src[NT];
  uint64_t* dst[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    src[k] = P<const uint64_t*>(st, k);
    dst[k] = P<uint64_t*>(st, NT + k);
  }
  const uint64_t* rpending = P<const uint64_t*>(st, B);
  GlState* S = P<GlState*>(st, B + 1);
  uint64_t* r_out = P<uint64_t*>(st, B + 2);
  uint64_t* msg = P<uint64_t*>(st, B + 3);
  __shared__ uint64_t r_sh;
  bool fold = rpending != nullptr;
  if (threadIdx.x == 0) r_sh = fold ? *rpending : 0;
  __syncthreads();
  uint64_t size = st.q[0];
  for (uint32_t j = 0;; ++j) {
    const uint64_t r = r_sh;
    if (fold) {
      const uint64_t m = size / 2;
      for (uint64_t t = threadIdx.x; t < NT * m; t += blockDim.x) {
        const uint32_t k = (uint32_t)(t / m);
        const uint64_t i = t - k * m;
        const uint64_t* sp = src[0];
        uint64_t* dp = dst[0];
#pragma unroll
        for (int q = 1; q < NT; ++q)
          if (k == (uint32_t)q) {
            sp = src[q];
            dp = dst[q];
          }
        const uint64_t a0 = gld(sp, i), a1 = gld(sp, i + m);
        gst(dp, i, gl_add(a0, gl_mul(r, gl_sub(a1, a0))));
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < NT; ++k) src[k] = dst[k];
      size = m;
    }
    if (j == st.u[0]) break;
    const uint64_t half = size / 2;
    uint64_t acc[2] = {0, 0};
    for (uint64_t b = threadIdx.x; b < half; b += blockDim.x) gl_pair<NT>(src, dst, false, 0, b, half, acc[0], acc[1]);
    gl_block_sum<2>(acc);
    if (threadIdx.x == 0) {
      const uint64_t rr = gl_round_step(S, acc[0], acc[1], msg + 3 * j);
      r_out[j] = rr;
      r_sh = rr;
    }
    __syncthreads();
    fold = true;
  }
  if (threadIdx.x == 0) {
    const uint64_t v = gld(src[0], 0);
    *P<uint64_t*>(st, B + 4) = v;
    uint64_t* proof_value = P<uint64_t*>(st, B + 5);
    if (proof_value) {
      *proof_value = v;
      Sha256State sh = gl_load_state(S);
      gl_absorb_value(sh, v);
      gl_save_state(S, sh);
    }
  }
}

#undef GTID
#undef GSTRIDE

void launch_gl_step(const Step& st, hipStream_t s) {
  const int tok = prof_begin(s);
  const dim3 grid(st.ntiles), block(kBlock);
  ProfClass cls = PC_SMALL;
  switch (st.type) {
    case ST_GL_FORWARD: k_gl_forward<<<grid, block, 0, s>>>(st); cls = PC_FORWARD; break;
    case ST_GL_DIGEST: k_gl_digest<<<grid, block, 0, s>>>(st); cls = PC_DIGEST; break;
    case ST_GL_BEGIN: k_gl_begin<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_GL_SQUEEZE: k_gl_squeeze<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_GL_LAYER_BEGIN: k_gl_layer_begin<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_GL_EQ: k_gl_eq<<<grid, block, 0, s>>>(st); cls = PC_EQ; break;
    case ST_GL_WSUM: k_gl_wsum<<<grid, block, 0, s>>>(st); cls = PC_CLAIM; break;
    case ST_GL_P1: k_gl_p1<<<grid, block, 0, s>>>(st); cls = PC_PHASE1_INIT; break;
    case ST_GL_ROUND: k_gl_round<3><<<grid, block, 0, s>>>(st); cls = PC_ROUND_A; break;
    case ST_GL_TAIL: k_gl_tail<3><<<grid, block, 0, s>>>(st); cls = PC_TAIL_A; break;
    case ST_GL_ROUND5: k_gl_round<5><<<grid, block, 0, s>>>(st); cls = PC_ROUND_B; break;
    case ST_GL_TAIL5: k_gl_tail<5><<<grid, block, 0, s>>>(st); cls = PC_TAIL_B; break;
    case ST_GL_COPY_WEIGHTS: k_gl_copy_weights<<<grid, block, 0, s>>>(st); cls = PC_SMALL; break;
    case ST_GL_P2T: k_gl_p2t<<<grid, block, 0, s>>>(st); cls = PC_PHASE2_TABLES; break;
    case ST_GL_COPY_CONTRACT: k_gl_copy_contract<<<grid, block, 0, s>>>(st); cls = PC_COPY_CONTRACT; break;
    case ST_GL_LOCAL_VALUES: k_gl_local_values<<<grid, block, 0, s>>>(st); cls = PC_SMALL; break;
    case ST_GL_LOCAL_CONTRACT: k_gl_local_contract<<<grid, block, 0, s>>>(st); cls = PC_LOCAL_CONTRACT; break;
    case ST_GL_COPY_TABLES: k_gl_copy_tables<<<grid, block, 0, s>>>(st); cls = PC_SMALL; break;
    default: break;
  }
  if (tok >= 0) prof_end(tok, s, cls, st.bytes, st.mulmods);
}

// ---------------------------------------------------------------- proof program (host)

namespace {

constexpr uint32_t kGlSweepTiles = 65535u * 8;
constexpr double kGE = 8.0;  // bytes per element

uint32_t gl_tiles(uint64_t n, uint32_t cap) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

Step gl_mk(uint32_t type, uint32_t ntiles) {
  Step st;
  memset(&st, 0, sizeof(st));
  st.type = type;
  st.ntiles = ntiles < 1 ? 1 : ntiles;
  return st;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

struct GlWs {
  uint64_t* layer[GKR_MAX_DEPTH + 1];
  uint64_t *G, *H, *Wf, *aU, *bV, *Cu, *Cv, *EL, *EC, *partials, *chal;
  uint64_t *U, *V, *P, *Q, *Fa, *Fb, *Ka, *Kb, *Ks, *EqR, *Wc, *Fc, *Kc, *wpart;
  uint32_t *dig_a, *dig_b, *dig_in, *dig_out;
  GlState* S;
};

GlWs gl_bind(const gkr_circuit& c, void* base, const uint64_t* d_inputs, uint64_t* d_outputs) {
  const GlPlan& p = c.gl;
  char* b = static_cast<char*>(base);
  GlWs w;
  memset(&w, 0, sizeof(w));
  auto U = [&](size_t o) { return reinterpret_cast<uint64_t*>(b + o); };
  for (uint32_t i = 1; i < c.depth; ++i) w.layer[i] = U(p.off_layer[i]);
  w.layer[0] = d_outputs;
  w.layer[c.depth] = const_cast<uint64_t*>(d_inputs);
  w.G = U(p.off_G); w.H = U(p.off_H); w.Wf = U(p.off_Wf);
  w.aU = U(p.off_aU); w.bV = U(p.off_bV); w.Cu = U(p.off_Cu); w.Cv = U(p.off_Cv);
  w.EL = U(p.off_EL); w.EC = U(p.off_EC);
  w.U = U(p.off_U); w.V = U(p.off_V); w.P = U(p.off_P); w.Q = U(p.off_Q); w.Fa = U(p.off_Fa); w.Fb = U(p.off_Fb);
  w.Ka = U(p.off_Ka); w.Kb = U(p.off_Kb); w.Ks = U(p.off_Ks); w.EqR = U(p.off_EqR); w.Wc = U(p.off_Wc);
  w.Fc = U(p.off_Fc); w.Kc = U(p.off_Kc); w.wpart = U(p.off_wpart);
  w.partials = U(p.off_partials);
  w.chal = U(p.off_chal);
  w.dig_a = reinterpret_cast<uint32_t*>(b + p.off_dig_a);
  w.dig_b = reinterpret_cast<uint32_t*>(b + p.off_dig_b);
  w.dig_in = reinterpret_cast<uint32_t*>(b + p.off_dig_in);
  w.dig_out = reinterpret_cast<uint32_t*>(b + p.off_dig_out);
  w.S = reinterpret_cast<GlState*>(b + p.off_state);
  return w;
}

void gl_digest(std::vector<Step>& steps, const uint64_t* vec, uint64_t nelem, uint32_t* final_out, const GlWs& w) {
  const uint32_t* in = reinterpret_cast<const uint32_t*>(vec);
  uint64_t nwords = 2 * nelem;
  int swap = 1;
  uint32_t* bufs[2] = {w.dig_a, w.dig_b};
  int which = 0;
  for (;;) {
    const uint64_t nchunks = (nwords + kChunkWords - 1) / kChunkWords;
    uint32_t* out = (nchunks == 1) ? final_out : bufs[which];
    Step st = gl_mk(ST_GL_DIGEST, gl_tiles(nchunks, kGlSweepTiles));
    st.p[0] = in; st.p[1] = out; st.q[0] = nwords; st.q[1] = nchunks; st.u[0] = swap;
    st.bytes = 4.0 * nwords + 32.0 * nchunks;
    steps.push_back(st);
    if (nchunks == 1) break;
    in = out;
    nwords = nchunks * 8;
    swap = 0;
    which ^= 1;
  }
}

void gl_eq(std::vector<Step>& steps, int count, const uint32_t* bits, const uint64_t* const* pts,
           const uint64_t* const* scl, uint64_t* const* outs) {
  Step st = gl_mk(ST_GL_EQ, 1);
  uint64_t total = 0;
  for (int j = 0; j < count; ++j) {
    st.u[j] = bits[j]; st.p[j] = pts[j]; st.p[4 + j] = scl[j]; st.p[8 + j] = outs[j];
    total += 1ull << bits[j];
  }
  st.u[4] = count;
  st.ntiles = gl_tiles(total, 1u << 30);
  st.bytes = kGE * total;
  steps.push_back(st);
}

// One phase: grid-wide rounds while the table exceeds 2^tail_log, then the tail.
// The rounds of one phase over NT tables (3: W X + Y; 5: A B + C D + E):
// grid-wide rounds while the evaluated table exceeds the tail size, then one
// workgroup.
template <int NT>
void gl_phase(std::vector<Step>& steps, const uint64_t* const* src0, uint64_t* const* dst, uint32_t nrounds,
              GlState* S, uint64_t* partials, uint64_t* r_out, uint64_t* msg, uint64_t* final_out,
              uint64_t* proof_value, const Tuning& tun) {
  constexpr int B = 2 * NT;
  const uint64_t* src[NT];
  for (int k = 0; k < NT; ++k) src[k] = src0[k];
  uint64_t eval = 1ull << nrounds;
  uint32_t j = 0;
  const uint64_t* pending = nullptr;
  while (j < nrounds && eval > (1ull << tun.tail_log)) {
    const uint64_t half = eval / 2;
    Step st = gl_mk(NT == 3 ? ST_GL_ROUND : ST_GL_ROUND5, gl_tiles((half + 1) / 2, tun.max_round_blocks));
    for (int k = 0; k < NT; ++k) {
      st.p[k] = src[k];
      st.p[NT + k] = dst[k];
    }
    st.p[B] = pending; st.p[B + 1] = S; st.p[B + 2] = partials; st.p[B + 3] = r_out + j; st.p[B + 4] = msg + 3 * j;
    st.q[0] = half;
    st.bytes = kGE * NT * (pending ? 6.0 : 2.0) * half;
    st.mulmods = (pending ? 2.0 * NT : 0.0) * half + (NT == 3 ? 4.0 : 6.0) * half;
    steps.push_back(st);
    if (pending)
      for (int k = 0; k < NT; ++k) src[k] = dst[k];
    pending = r_out + j;
    ++j;
    eval /= 2;
  }
  Step st = gl_mk(NT == 3 ? ST_GL_TAIL : ST_GL_TAIL5, 1);
  for (int k = 0; k < NT; ++k) {
    st.p[k] = src[k];
    st.p[NT + k] = dst[k];
  }
  st.p[B] = pending; st.p[B + 1] = S; st.p[B + 2] = r_out + j; st.p[B + 3] = msg + 3 * j; st.p[B + 4] = final_out;
  st.p[B + 5] = proof_value;
  st.q[0] = pending ? 2 * eval : eval;
  st.u[0] = nrounds - j;
  st.bytes = kGE * 3.0 * NT * eval;
  steps.push_back(st);
}

// Row chunks of the local contraction: about 2^18 threads in all.
uint32_t gl_ychunks(uint32_t sigma, uint32_t n) {
  const uint64_t want = (n >= 18) ? 1 : (1ull << (18 - n));
  return (uint32_t)std::min<uint64_t>(want, 1ull << sigma);
}

uint64_t gl_layer_proof_words(const gkr_circuit& c, uint32_t i) { return 6ull * c.s(i + 1) + 2; }

void gl_emit_proof(std::vector<Step>& steps, const gkr_circuit& c, const GlWs& w, uint64_t seed, uint64_t* proof,
                   const Tuning& tun) {
  const uint32_t d = c.depth, n = c.n;
  // forward evaluation: layer d is the caller's inputs, layer 0 the caller's outputs
  for (int i = (int)d - 1; i >= 0; --i) {
    Step st = gl_mk(ST_GL_FORWARD, gl_tiles(1ull << c.s(i), kGlSweepTiles));
    st.p[0] = w.layer[i + 1]; st.p[1] = w.layer[i]; st.p[2] = c.wiring[i].gates; st.u[0] = n;
    st.q[0] = 1ull << c.s(i);
    st.bytes = kGE * 3.0 * (1ull << c.s(i));
    st.mulmods = (double)(c.mul_gates[i] << n);
    steps.push_back(st);
  }
  // statement
  gl_digest(steps, w.layer[d], 1ull << c.s(d), w.dig_in, w);
  gl_digest(steps, w.layer[0], 1ull << c.s(0), w.dig_out, w);
  {
    Step st = gl_mk(ST_GL_BEGIN, 1);
    st.p[0] = w.S; st.p[1] = w.dig_in; st.p[2] = w.dig_out;
    uint8_t msg[22];
    memcpy(msg, "SISU-GKR-GL-v1", 14);
    for (int k = 0; k < 8; ++k) msg[14 + k] = (uint8_t)(seed >> (8 * k));
    sha256_bytes(msg, sizeof(msg), st.w);
    memcpy(st.w + 8, c.digest, 32);
    steps.push_back(st);
  }
  // output point and claim
  uint64_t* g = w.chal;
  {
    Step st = gl_mk(ST_GL_SQUEEZE, 1);
    st.p[0] = w.S; st.p[1] = g; st.u[0] = c.s(0);
    steps.push_back(st);
    const uint32_t bits[2] = {c.sigma[0], n};
    const uint64_t* pts[2] = {g, g + c.sigma[0]};
    const uint64_t* scl[2] = {nullptr, nullptr};
    uint64_t* outs[2] = {w.aU, w.Cu};
    gl_eq(steps, 2, bits, pts, scl, outs);
    Step ws = gl_mk(ST_GL_WSUM, gl_tiles(1ull << c.s(0), tun.max_round_blocks));
    ws.p[0] = w.layer[0]; ws.p[1] = w.aU; ws.p[2] = w.Cu; ws.p[3] = w.partials; ws.p[4] = w.S;
    ws.p[5] = &w.S->scratch[0]; ws.u[0] = n; ws.q[0] = 1ull << c.s(0);
    ws.bytes = kGE * (1ull << c.s(0));
    steps.push_back(ws);
  }
  // layers
  uint64_t* chal = g + c.s(0);
  uint64_t* pr = proof;
  for (uint32_t i = 0; i < d; ++i) {
    const uint32_t sg = c.sigma[i], sg1 = c.sigma[i + 1], s1 = c.s(i + 1);
    const uint64_t* u = (i == 0) ? g : chal - 2 * c.s(i);
    const uint64_t* v = (i == 0) ? g : chal - c.s(i);
    uint64_t* rx = chal;
    uint64_t* ry = chal + s1;
    {
      Step st = gl_mk(ST_GL_LAYER_BEGIN, 1);
      st.p[0] = w.S; st.p[1] = (i == 0) ? &w.S->scratch[0] : &w.S->vx; st.p[2] = &w.S->vy; st.u[0] = i == 0;
      steps.push_back(st);
    }
    {
      const uint32_t bits[4] = {sg, sg, n, n};
      const uint64_t* pts[4] = {u, v, u + sg, v + sg};
      const uint64_t* scl[4] = {&w.S->alpha, &w.S->beta, nullptr, nullptr};
      uint64_t* outs[4] = {w.aU, w.bV, w.Cu, w.Cv};
      gl_eq(steps, 4, bits, pts, scl, outs);
    }
    const LayerWiring& lw = c.wiring[i];
    {
      Step st = gl_mk(ST_GL_P1, gl_tiles(1ull << s1, kGlSweepTiles));
      st.p[0] = w.layer[i + 1]; st.p[1] = w.G; st.p[2] = w.H; st.p[3] = lw.xrow; st.p[4] = lw.xent;
      st.p[5] = w.aU; st.p[6] = w.bV; st.p[7] = w.Cu; st.p[8] = w.Cv; st.u[0] = n; st.q[0] = 1ull << s1;
      st.bytes = kGE * (double)((1ull << c.s(i)) + 2 * (1ull << s1));
      st.mulmods = 3.0 * (1ull << c.s(i));
      steps.push_back(st);
    }
    {
      const uint64_t* src[3] = {w.layer[i + 1], w.G, w.H};
      uint64_t* dst[3] = {w.Wf, w.G, w.H};
      gl_phase<3>(steps, src, dst, s1, w.S, w.partials, rx, pr, &w.S->vx, pr + 3 * s1, tun);
    }
    {
      const uint32_t bits[2] = {sg1, n};
      const uint64_t* pts[2] = {rx, rx + sg1};
      const uint64_t* scl[2] = {nullptr, nullptr};
      uint64_t* outs[2] = {w.EL, w.EC};
      gl_eq(steps, 2, bits, pts, scl, outs);
    }
    // phase 2 with the copy factors contracted
    const uint64_t ncop = 1ull << n, rows = 1ull << sg1;
    {
      Step st = gl_mk(ST_GL_COPY_WEIGHTS, 1);
      st.p[0] = w.EC; st.p[1] = w.Cu; st.p[2] = w.Cv; st.p[3] = w.U; st.p[4] = w.V; st.p[5] = w.S; st.q[0] = ncop;
      st.bytes = kGE * 5.0 * ncop; st.mulmods = 2.0 * ncop;
      steps.push_back(st);
    }
    {
      Step st = gl_mk(ST_GL_P2T, gl_tiles(rows, kGlSweepTiles));
      st.p[0] = lw.yrow; st.p[1] = lw.yent; st.p[2] = w.aU; st.p[3] = w.bV; st.p[4] = w.EL; st.p[5] = w.S;
      st.p[6] = w.Fa; st.p[7] = w.Fb; st.p[8] = w.Ka; st.p[9] = w.Kb; st.p[10] = w.Ks; st.q[0] = rows;
      st.bytes = kGE * 5.0 * rows; st.mulmods = 2.0 * (double)(1ull << sg) + 6.0 * rows;
      steps.push_back(st);
    }
    {
      Step st = gl_mk(ST_GL_COPY_CONTRACT, gl_tiles(rows * 64, kGlSweepTiles));
      st.p[0] = w.layer[i + 1]; st.p[1] = w.U; st.p[2] = w.V; st.p[3] = w.P; st.p[4] = w.Q; st.u[0] = n;
      st.q[0] = rows;
      st.bytes = kGE * (double)(rows * ncop); st.mulmods = 2.0 * rows * ncop;
      steps.push_back(st);
    }
    {
      const uint64_t* src[5] = {w.P, w.Fa, w.Q, w.Fb, w.Ks};
      uint64_t* dst[5] = {w.P, w.Fa, w.Q, w.Fb, w.Ks};
      gl_phase<5>(steps, src, dst, sg1, w.S, w.partials, ry, pr + 3 * s1 + 1, &w.S->scratch[1], nullptr, tun);
    }
    {
      const uint32_t bits[1] = {sg1};
      const uint64_t* pts[1] = {ry};
      const uint64_t* scl[1] = {nullptr};
      uint64_t* outs[1] = {w.EqR};
      gl_eq(steps, 1, bits, pts, scl, outs);
    }
    {
      Step st = gl_mk(ST_GL_LOCAL_VALUES, 1);
      st.p[0] = w.EqR; st.p[1] = w.Ka; st.p[2] = w.Kb; st.p[3] = w.S; st.q[0] = rows;
      st.bytes = kGE * 3.0 * rows; st.mulmods = 2.0 * rows;
      steps.push_back(st);
    }
    const uint32_t R = gl_ychunks(sg1, n);
    {
      uint32_t lr = 0;
      while ((1ull << (lr + 1)) * R <= rows) ++lr;  // rows per chunk = rows / R
      Step st = gl_mk(ST_GL_LOCAL_CONTRACT, gl_tiles((uint64_t)R * ncop, kGlSweepTiles));
      st.p[0] = w.layer[i + 1]; st.p[1] = w.EqR; st.p[2] = w.wpart; st.u[0] = n; st.u[1] = lr;
      st.q[0] = (uint64_t)R * ncop;
      st.bytes = kGE * (double)(rows * ncop + (uint64_t)R * ncop); st.mulmods = (double)(rows * ncop);
      steps.push_back(st);
    }
    {
      uint32_t tl = 0;
      while ((1u << (tl + 1)) <= R && tl < 6) ++tl;  // lanes per column, as in the kernel
      Step st = gl_mk(ST_GL_COPY_TABLES, gl_tiles(ncop << tl, kGlSweepTiles));
      st.p[0] = w.wpart; st.p[1] = w.U; st.p[2] = w.V; st.p[3] = w.Fa; st.p[4] = w.Fb; st.p[5] = w.S;
      st.p[6] = w.Wc; st.p[7] = w.Fc; st.p[8] = w.Kc; st.u[0] = R; st.q[0] = ncop;
      st.bytes = kGE * (double)((uint64_t)R * ncop + 5 * ncop); st.mulmods = 4.0 * ncop;
      steps.push_back(st);
    }
    {
      const uint64_t* src[3] = {w.Wc, w.Fc, w.Kc};
      uint64_t* dst[3] = {w.Wc, w.Fc, w.Kc};
      gl_phase<3>(steps, src, dst, n, w.S, w.partials, ry + sg1, pr + 3 * s1 + 1 + 3 * sg1, &w.S->vy,
                  pr + 6 * s1 + 1, tun);
    }
    pr += gl_layer_proof_words(c, i);
    chal += 2 * s1;
  }
}

}  // namespace

void plan_gl_workspace(gkr_circuit& c) {
  GlPlan& p = c.gl;
  memset(&p, 0, sizeof(p));
  const uint32_t d = c.depth, n = c.n;
  uint32_t sp = 0, sig = 0;
  size_t chal = c.s(0);
  for (uint32_t i = 0; i < d; ++i) {
    sp = std::max(sp, c.s(i + 1));
    chal += 2ull * c.s(i + 1);
  }
  for (uint32_t i = 0; i <= d; ++i) sig = std::max(sig, c.sigma[i]);
  const size_t E = 8;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  for (uint32_t i = 1; i < d; ++i) p.off_layer[i] = take(E << c.s(i));
  p.off_G = take(E << sp);
  p.off_H = take(E << sp);
  p.off_Wf = take(E << (sp ? sp - 1 : 0));
  p.off_aU = take(E << sig);
  p.off_bV = take(E << sig);
  p.off_Cu = take(E << n);
  p.off_Cv = take(E << n);
  p.off_EL = take(E << sig);
  p.off_EC = take(E << n);
  p.off_partials = take(E * 2 * (size_t)kMaxRoundBlocks);
  p.off_U = take(E << n);
  p.off_V = take(E << n);
  p.off_P = take(E << sig);
  p.off_Q = take(E << sig);
  p.off_Fa = take(E << sig);
  p.off_Fb = take(E << sig);
  p.off_Ka = take(E << sig);
  p.off_Kb = take(E << sig);
  p.off_Ks = take(E << sig);
  p.off_EqR = take(E << sig);
  p.off_Wc = take(E << n);
  p.off_Fc = take(E << n);
  p.off_Kc = take(E << n);
  {
    uint64_t wp = 1;
    for (uint32_t i = 0; i < d; ++i) wp = std::max<uint64_t>(wp, (uint64_t)gl_ychunks(c.sigma[i + 1], n) << n);
    p.off_wpart = take(E * wp);
  }
  const uint64_t big = 1ull << std::max(c.s(0), c.s(d));
  const uint64_t words = (2 * big + kChunkWords - 1) / kChunkWords * 8;
  p.off_dig_a = take(4 * words);
  p.off_dig_b = take(4 * words);
  p.off_dig_in = take(32);
  p.off_dig_out = take(32);
  p.off_chal = take(E * (chal + 8));
  p.off_state = take(sizeof(GlState));
  c.plan.total = off;
}

size_t gl_proof_bytes(const gkr_circuit& c) {
  size_t t = 0;
  for (uint32_t i = 0; i < c.depth; ++i) t += gl_layer_proof_words(c, i) * 8;
  return t;
}

}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_gl_prove_circuit(const gkr_circuit* c, const uint64_t* d_inputs, uint64_t seed,
                                        uint64_t* d_outputs, uint8_t* d_proof, size_t proof_cap, size_t* proof_len,
                                        void* d_ws, size_t ws_bytes, void* stream) {
  if (!c || !d_inputs || !d_outputs || !d_proof) {
    set_error("null argument");
    return GKR_EINVAL;
  }
  if (c->field != GKR_FIELD_GOLDILOCKS) {
    set_error("gkr_gl_prove_circuit takes circuits created for the Goldilocks field");
    return GKR_EINVAL;
  }
  if ((reinterpret_cast<uintptr_t>(d_inputs) & 15) ||
      ((reinterpret_cast<uintptr_t>(d_outputs) | reinterpret_cast<uintptr_t>(d_proof)) & 7)) {
    set_error("d_inputs must be 16-byte aligned, d_outputs and d_proof 8-byte aligned");
    return GKR_EINVAL;
  }
  const size_t need = gl_proof_bytes(*c);
  if (proof_len) *proof_len = need;
  if (proof_cap < need) {
    set_error("proof buffer too small: " + std::to_string(proof_cap) + " < " + std::to_string(need));
    return GKR_EBUFSZ;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  try {
    const GlWs w = gl_bind(*c, d_ws, d_inputs, d_outputs);
    Program pg;
    gl_emit_proof(pg.steps, *c, w, seed, reinterpret_cast<uint64_t*>(d_proof), current_tuning());
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return GKR_EDEVICE;
  }
  return GKR_OK;
}
