// HIP kernels of the data-parallel GKR prover for gfx950.
//
// Every kernel uses 256-thread workgroups (four 64-wide waves). Field elements
// are 32-byte records in Montgomery form, loaded and stored as two 16-byte
// vectors, so consecutive threads touch consecutive records and every access
// of a table sweep is coalesced. Gate g = z*2^n + c keeps the copy index in the
// low bits: a gather W[(y_z << n) | c] over consecutive c is contiguous.
//
// Reductions over a whole table (the round polynomials of the sumcheck) end in
// the last workgroup to finish: each workgroup writes its partial sums,
// publishes them with a device-scope fence and an atomic counter, and the
// workgroup that brings the counter to the grid size adds the partials and runs
// the Fiat-Shamir step (absorb the message, squeeze the next challenge, move the
// claim) on one thread. Challenges and claims never leave device memory, so a
// proof is a plain sequence of launches on one stream.
#include "gkr_kernels.hpp"
#include "gkr_profile.hpp"

namespace gkr {

// ----------------------------------------------------------------- helpers

__device__ __forceinline__ Fr ldf(const Fr* p, uint64_t i) {
  const uint4* q = reinterpret_cast<const uint4*>(p + i);
  uint4 a = q[0], b = q[1];
  return fr_make(a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
}

__device__ __forceinline__ void stf(Fr* p, uint64_t i, const Fr& v) {
  uint4* q = reinterpret_cast<uint4*>(p + i);
  q[0] = make_uint4(v.v[0], v.v[1], v.v[2], v.v[3]);
  q[1] = make_uint4(v.v[4], v.v[5], v.v[6], v.v[7]);
}

__device__ __forceinline__ Fr shfl_xor_fr(const Fr& a, int mask) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = (uint32_t)__shfl_xor((int)a.v[k], mask, 64);
  return r;
}

__device__ __forceinline__ uint64_t gtid() { return (uint64_t)blockIdx.x * kBlock + threadIdx.x; }
__device__ __forceinline__ uint64_t gstride() { return (uint64_t)gridDim.x * kBlock; }

// Sum of NV values over the workgroup; the totals are valid in thread 0.
template <int NV>
__device__ void block_reduce(Fr (&v)[NV]) {
  __shared__ Fr red[NV][kBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = fr_add(v[k], shfl_xor_fr(v[k], off));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      Fr acc = red[k][0];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) acc = fr_add(acc, red[k][w]);
      v[k] = acc;
    }
  }
  __syncthreads();
}

// Grid-wide sum. Returns true in the last workgroup to finish, where thread 0
// then holds the totals; the counter is back at zero afterwards.
template <int NV>
__device__ bool grid_reduce(Fr (&v)[NV], Fr* partials, uint32_t* counter) {
  block_reduce<NV>(v);
  __shared__ int is_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) stf(partials, (uint64_t)blockIdx.x * NV + k, v[k]);
    __threadfence();
    uint32_t prev = atomicAdd(counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return false;
  __threadfence();
  Fr acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = fr_zero();
  for (uint32_t b = threadIdx.x; b < gridDim.x; b += kBlock) {
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = fr_add(acc[k], ldf(partials, (uint64_t)b * NV + k));
  }
  block_reduce<NV>(acc);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = acc[k];
    atomicExch(counter, 0u);
  }
  return true;
}

// ---------------------------------------------------------- transcript

// SHA-256 of a fixed-length word message (big-endian words), fully unrolled.
template <int L>
__device__ Sha256State sha256_fixed(const uint32_t* w) {
  constexpr int B = (L + 3 + 15) / 16;
  Sha256State st = sha256_iv();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    uint32_t blk[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int idx = b * 16 + i;
      uint32_t v;
      if (idx < L) v = w[idx];
      else if (idx == L) v = 0x80000000u;
      else if (idx == B * 16 - 1) v = (uint32_t)(L * 32);
      else v = 0u;
      blk[i] = v;
    }
    sha256_compress(st, blk);
  }
  return st;
}

__device__ Sha256State load_state(const DevState* S) {
  Sha256State s;
#pragma unroll
  for (int k = 0; k < 8; ++k) s.h[k] = S->st[k];
  return s;
}

__device__ void save_state(DevState* S, const Sha256State& s) {
#pragma unroll
  for (int k = 0; k < 8; ++k) S->st[k] = s.h[k];
}

// Field products of the serial Fiat-Shamir code: one out-of-line copy keeps
// the single-thread paths small.
__device__ __attribute__((noinline)) Fr fr_mul_ni(Fr a, Fr b) { return fr_mul(a, b); }
__device__ __forceinline__ Fr to_mont_ni(const Fr& a) { return fr_mul_ni(a, fr_r2()); }
__device__ __forceinline__ Fr from_mont_ni(const Fr& a) { return fr_mul_ni(a, fr_make(1, 0, 0, 0, 0, 0, 0, 0)); }

// g(r) for the degree-2 polynomial with values e0, e1, e2 at t = 0, 1, 2.
__device__ Fr interp3_ni(const Fr& e0, const Fr& e1, const Fr& e2, const Fr& r) {
  const Fr d1 = fr_sub(e1, e0);
  const Fr d2 = fr_add(fr_sub(e2, fr_double(e1)), e0);
  const Fr rr = fr_mul_ni(fr_mul_ni(r, fr_sub(r, fr_one())), fr_inv2());
  return fr_add(fr_add(e0, fr_mul_ni(r, d1)), fr_mul_ni(rr, d2));
}

// The current state as a challenge: rehash with "GKRC" until the 254-bit
// little-endian value is below p. Each attempt is accepted with probability
// p / 2^254 > 3/4; the bound on attempts only guarantees termination.
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

// Round message (e0, e1 = claim - e0, e2): write it to the proof, absorb
// (e0, e2), take the challenge r from the state, store r and move the claim to g(r).
__device__ void finish_round(DevState* S, const Fr& e0, const Fr& e2, Fr* r_out,
                             uint32_t* msg_out) {
  const Fr c0 = from_mont_ni(e0), c2 = from_mont_ni(e2);
  uint32_t w[25];
  Sha256State st = load_state(S);
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = kTagRound;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    w[9 + k] = bswap32(c0.v[k]);
    w[17 + k] = bswap32(c2.v[k]);
  }
  st = sha256_fixed<25>(w);
  const Fr r = to_mont_ni(accept(st));
  stf(r_out, 0, r);
  save_state(S, st);
  const Fr e1 = fr_sub(S->claim, e0);
  const Fr c1 = from_mont_ni(e1);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    msg_out[k] = c0.v[k];
    msg_out[8 + k] = c1.v[k];
    msg_out[16 + k] = c2.v[k];
  }
  S->claim = interp3_ni(e0, e1, e2, r);
}

// A phase's final value: store it, write it to the proof and absorb it.
__device__ void finish_value(DevState* S, const Fr& v, Fr* v_out, uint32_t* proof_out) {
  const Fr c = from_mont_ni(v);
  Sha256State st = load_state(S);
  absorb_element(st, kTagValue, c);
  save_state(S, st);
  *v_out = v;
#pragma unroll
  for (int k = 0; k < 8; ++k) proof_out[k] = c.v[k];
}

// ------------------------------------------------------------- kernels

__global__ void __launch_bounds__(kBlock) k_to_mont(const gkr_fr* in, Fr* out, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride()) {
    Fr a = ldf(reinterpret_cast<const Fr*>(in), i);
    stf(out, i, fr_to_mont(a));
  }
}

__global__ void __launch_bounds__(kBlock) k_from_mont(const Fr* in, gkr_fr* out, uint64_t n) {
  for (uint64_t i = gtid(); i < n; i += gstride())
    stf(reinterpret_cast<Fr*>(out), i, fr_from_mont(ldf(in, i)));
}

// V_i[z*2^n + c] = W[x_z*2^n + c] (+ or *) W[y_z*2^n + c].
__global__ void __launch_bounds__(kBlock)
    k_forward(const Fr* __restrict__ W, Fr* __restrict__ V, const uint2* __restrict__ gates,
              uint32_t n, uint64_t count) {
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t g = gtid(); g < count; g += gstride()) {
    const uint64_t z = g >> n, c = g & mask;
    const uint2 gate = gates[z];
    const uint64_t x = gate.x & 0x7fffffffu, y = gate.y;
    const Fr a = ldf(W, (x << n) | c), b = ldf(W, (y << n) | c);
    stf(V, g, (gate.x >> 31) ? fr_mul(a, b) : fr_add(a, b));
  }
}

// One level of a tree digest: chunk t of `nwords` words (2048 per chunk) is
// hashed by thread t; element words are byte-swapped (limbs are little-endian).
__global__ void __launch_bounds__(kBlock)
    k_digest_level(const uint32_t* __restrict__ in, uint64_t nwords, int swap,
                   uint32_t* __restrict__ out, uint64_t nchunks) {
  const uint64_t t = gtid();
  if (t >= nchunks) return;
  const uint64_t begin = t * kChunkWords;
  const uint64_t end = (begin + kChunkWords < nwords) ? begin + kChunkWords : nwords;
  const uint64_t len = end - begin;  // a multiple of 8 words
  Sha256State st = sha256_iv();
  const uint4* src = reinterpret_cast<const uint4*>(in + begin);
  const uint64_t full = len / 16;
  for (uint64_t b = 0; b < full; ++b) {
    uint32_t blk[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 v = src[b * 4 + q];
      blk[4 * q + 0] = swap ? bswap32(v.x) : v.x;
      blk[4 * q + 1] = swap ? bswap32(v.y) : v.y;
      blk[4 * q + 2] = swap ? bswap32(v.z) : v.z;
      blk[4 * q + 3] = swap ? bswap32(v.w) : v.w;
    }
    sha256_compress(st, blk);
  }
  uint32_t blk[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) blk[i] = 0;
  const uint64_t rem = len - full * 16;  // 0 or 8
  if (rem == 8) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint4 v = src[full * 4 + q];
      blk[4 * q + 0] = swap ? bswap32(v.x) : v.x;
      blk[4 * q + 1] = swap ? bswap32(v.y) : v.y;
      blk[4 * q + 2] = swap ? bswap32(v.z) : v.z;
      blk[4 * q + 3] = swap ? bswap32(v.w) : v.w;
    }
    blk[8] = 0x80000000u;
  } else {
    blk[0] = 0x80000000u;
  }
  const uint64_t bits = len * 32;
  blk[14] = (uint32_t)(bits >> 32);
  blk[15] = (uint32_t)bits;
  sha256_compress(st, blk);
#pragma unroll
  for (int k = 0; k < 8; ++k) out[t * 8 + k] = st.h[k];
}

// Statement binding: st = seed state, then absorb the three digests.
__global__ void k_transcript_begin(DevState* S, Words8 seed_state, Words8 circuit_digest,
                                   const uint32_t* dig_in, const uint32_t* dig_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Sha256State st;
#pragma unroll
  for (int k = 0; k < 8; ++k) st.h[k] = seed_state.w[k];
  absorb_digest(st, circuit_digest.w);
  absorb_digest(st, dig_in);
  absorb_digest(st, dig_out);
  save_state(S, st);
  S->counter = 0;
}

// Squeeze `count` challenges into out[0..count) (Montgomery form).
__global__ void k_squeeze(DevState* S, Fr* out, uint32_t count) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  Sha256State st = load_state(S);
  for (uint32_t k = 0; k < count; ++k) stf(out, k, to_mont_ni(squeeze(st)));
  save_state(S, st);
}

// Start of a gate layer: draw alpha, beta (layer > 0) and set the claim to
// alpha * vu + beta * vv; on layer 0 alpha = 1, beta = 0 and claim = vu.
__global__ void k_layer_begin(DevState* S, int first, const Fr* vu, const Fr* vv) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (first) {
    S->alpha = fr_one();
    S->beta = fr_zero();
    S->claim = *vu;
    return;
  }
  Sha256State st = load_state(S);
  const Fr a = to_mont_ni(squeeze(st));
  const Fr b = to_mont_ni(squeeze(st));
  save_state(S, st);
  S->alpha = a;
  S->beta = b;
  S->claim = fr_add(fr_mul_ni(a, *vu), fr_mul_ni(b, *vv));
}

// eq tables: out_j[b] = scale_j * prod_k (bit_k(b) ? r_k : 1 - r_k), bit 1 = MSB.
__global__ void __launch_bounds__(kBlock) k_eq_tables(EqJobs jobs) {
  uint64_t t = gtid();
  for (int j = 0; j < jobs.count; ++j) {
    const uint64_t size = 1ull << jobs.bits[j];
    if (t < size) {
      const Fr* r = jobs.point[j];
      const int k = jobs.bits[j];
      Fr acc = jobs.scale[j] ? *jobs.scale[j] : fr_one();
      for (int i = 0; i < k; ++i) {
        const Fr ri = ldf(r, i);
        const bool bit = (t >> (k - 1 - i)) & 1;
        acc = fr_mul(acc, bit ? ri : fr_one_minus(ri));
      }
      stf(jobs.out[j], t, acc);
      return;
    }
    t -= size;
  }
}

// Weighted sum over a layer: sum_e V[e] A[e >> n] B[e & mask] into *dst.
__global__ void __launch_bounds__(kBlock)
    k_weighted_sum(const Fr* __restrict__ V, const Fr* __restrict__ A, const Fr* __restrict__ B,
                   uint32_t n, uint64_t count, Fr* partials, uint32_t* counter, Fr* dst) {
  const uint64_t mask = (1ull << n) - 1;
  Fr acc[1] = {fr_zero()};
  for (uint64_t e = gtid(); e < count; e += gstride())
    acc[0] = fr_add(acc[0], fr_mul(fr_mul(ldf(V, e), ldf(A, e >> n)), ldf(B, e & mask)));
  if (grid_reduce<1>(acc, partials, counter) && threadIdx.x == 0) *dst = acc[0];
}

// Phase-1 bookkeeping tables over (x, c):
//   G[x,c] = sum_{MUL z: x_z=x} T[z,c] W[y_z,c] + sum_{ADD z: x_z=x} T[z,c]
//   H[x,c] = sum_{ADD z: x_z=x} T[z,c] W[y_z,c]
// with T[z,c] = aU[z] Cu[c] + bV[z] Cv[c] (the factored eq of both claims).
__device__ __forceinline__ void phase1_entry(const Fr* __restrict__ W, const uint32_t* __restrict__ xrow,
                                             const uint2* __restrict__ xent, const Fr* __restrict__ aU,
                                             const Fr* __restrict__ bV, const Fr* __restrict__ Cu,
                                             const Fr* __restrict__ Cv, uint32_t n, uint64_t e, Fr& g,
                                             Fr& h) {
  const uint64_t mask = (1ull << n) - 1;
  const uint64_t x = e >> n, c = e & mask;
  const Fr cu = ldf(Cu, c), cv = ldf(Cv, c);
  g = fr_zero();
  h = fr_zero();
  const uint32_t k1 = xrow[x + 1];
  for (uint32_t k = xrow[x]; k < k1; ++k) {
    const uint2 ent = xent[k];
    const uint64_t z = ent.x, y = ent.y & 0x7fffffffu;
    const Fr T = fr_add(fr_mul(ldf(aU, z), cu), fr_mul(ldf(bV, z), cv));
    const Fr tw = fr_mul(T, ldf(W, (y << n) | c));
    if (ent.y >> 31) {
      g = fr_add(g, tw);
    } else {
      g = fr_add(g, T);
      h = fr_add(h, tw);
    }
  }
}

__global__ void __launch_bounds__(kBlock)
    k_phase1_init(const Fr* __restrict__ W, Fr* __restrict__ G, Fr* __restrict__ H,
                  const uint32_t* __restrict__ xrow, const uint2* __restrict__ xent,
                  const Fr* __restrict__ aU, const Fr* __restrict__ bV,
                  const Fr* __restrict__ Cu, const Fr* __restrict__ Cv, uint32_t n,
                  uint64_t count) {
  for (uint64_t e = gtid(); e < count; e += gstride()) {
    Fr g, h;
    phase1_entry(W, xrow, xent, aU, bV, Cu, Cv, n, e, g, h);
    stf(G, e, g);
    stf(H, e, h);
  }
}

// The tables and the first round together: thread b builds entries b and
// b + half, evaluates the round-1 pair at t = 0, 2, and the last workgroup
// runs the Fiat-Shamir step.
__global__ void __launch_bounds__(kBlock)
    k_phase1_init_round(const Fr* __restrict__ W, Fr* __restrict__ G, Fr* __restrict__ H,
                        const uint32_t* __restrict__ xrow, const uint2* __restrict__ xent,
                        const Fr* __restrict__ aU, const Fr* __restrict__ bV,
                        const Fr* __restrict__ Cu, const Fr* __restrict__ Cv, uint32_t n,
                        uint64_t half, DevState* S, Fr* partials, Fr* r_out, uint32_t* msg_out) {
  Fr acc[2] = {fr_zero(), fr_zero()};
  for (uint64_t b = gtid(); b < half; b += gstride()) {
    Fr g0, h0, g1, h1;
    phase1_entry(W, xrow, xent, aU, bV, Cu, Cv, n, b, g0, h0);
    phase1_entry(W, xrow, xent, aU, bV, Cu, Cv, n, b + half, g1, h1);
    stf(G, b, g0);
    stf(H, b, h0);
    stf(G, b + half, g1);
    stf(H, b + half, h1);
    const Fr w0 = ldf(W, b), w1 = ldf(W, b + half);
    acc[0] = fr_add(acc[0], fr_add(fr_mul(w0, g0), h0));
    const Fr w2 = fr_sub(fr_double(w1), w0), g2 = fr_sub(fr_double(g1), g0), h2 = fr_sub(fr_double(h1), h0);
    acc[1] = fr_add(acc[1], fr_add(fr_mul(w2, g2), h2));
  }
  if (grid_reduce<2>(acc, partials, &S->counter) && threadIdx.x == 0)
    finish_round(S, acc[0], acc[1], r_out, msg_out);
}

// ------------------------------------------------------- round kernels

// Fold (if `fold`) and evaluate one pair b of a round: the evaluated table has
// 2*half entries; with folding the source has 4*half entries and the folded
// entries b and b + half are written to dst.
template <class Form>
__device__ __forceinline__ void round_pair(const Tabs<Form::NT>& t, uint64_t b, uint64_t half,
                                           bool fold, const Fr& r, Fr& acc0, Fr& acc2) {
  Fr x0[Form::NT], x2[Form::NT];
#pragma unroll
  for (int k = 0; k < Form::NT; ++k) {
    Fr lo, hi;
    if (fold) {
      const uint64_t m = 2 * half;
      const Fr a0 = ldf(t.src[k], b), a1 = ldf(t.src[k], b + m);
      const Fr b0 = ldf(t.src[k], b + half), b1 = ldf(t.src[k], b + half + m);
      lo = fr_add(a0, fr_mul(r, fr_sub(a1, a0)));
      hi = fr_add(b0, fr_mul(r, fr_sub(b1, b0)));
      stf(t.dst[k], b, lo);
      stf(t.dst[k], b + half, hi);
    } else {
      lo = ldf(t.src[k], b);
      hi = ldf(t.src[k], b + half);
    }
    x0[k] = lo;
    x2[k] = fr_sub(fr_double(hi), lo);  // value at t = 2
  }
  Form::eval(x0, acc0);
  Form::eval(x2, acc2);
}

// One sumcheck round over the whole grid (optional fold by the previous
// challenge, evaluation at t = 0, 2, Fiat-Shamir in the last workgroup).
template <class Form>
__global__ void __launch_bounds__(kBlock)
    k_round(Tabs<Form::NT> t, uint64_t half, const Fr* rprev, DevState* S, Fr* partials,
            Fr* r_out, uint32_t* msg_out) {
  const bool fold = rprev != nullptr;
  const Fr r = fold ? ldf(rprev, 0) : fr_zero();
  Fr acc[2] = {fr_zero(), fr_zero()};
  for (uint64_t b = gtid(); b < half; b += gstride()) round_pair<Form>(t, b, half, fold, r, acc[0], acc[1]);
  if (grid_reduce<2>(acc, partials, &S->counter) && threadIdx.x == 0)
    finish_round(S, acc[0], acc[1], r_out, msg_out);
}

// The remaining rounds of a phase in one workgroup, then the final fold.
// `size` is the table size before the pending fold (if any). Round messages go
// to msg (24 words each) and challenges to r_out[0..rounds); the final value
// of table 0 is stored in *final_out and, if proof_value is not null, written
// to the proof and absorbed.
template <class Form>
__global__ void __launch_bounds__(kBlock)
    k_tail(Tabs<Form::NT> t, uint64_t size, const Fr* rpending, uint32_t rounds, DevState* S,
           Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value) {
  __shared__ Fr r_sh;
  bool fold = rpending != nullptr;
  if (threadIdx.x == 0) r_sh = fold ? ldf(rpending, 0) : fr_zero();
  __syncthreads();
  for (uint32_t j = 0; j < rounds; ++j) {
    const uint64_t eval_size = fold ? size / 2 : size;
    const uint64_t half = eval_size / 2;
    const Fr r = r_sh;
    Fr acc[2] = {fr_zero(), fr_zero()};
    for (uint64_t b = threadIdx.x; b < half; b += kBlock) round_pair<Form>(t, b, half, fold, r, acc[0], acc[1]);
    block_reduce<2>(acc);
    if (threadIdx.x == 0) {
      finish_round(S, acc[0], acc[1], r_out + j, msg + 24 * j);
      r_sh = ldf(r_out + j, 0);
    }
    __syncthreads();
    if (fold) {
#pragma unroll
      for (int k = 0; k < Form::NT; ++k) t.src[k] = t.dst[k];
    }
    fold = true;
    size = eval_size;
  }
  if (fold) {  // size is 2 here
    if (threadIdx.x < Form::NT) {
      const int k = threadIdx.x;
      const Fr r = r_sh;
      const Fr a0 = ldf(t.src[k], 0), a1 = ldf(t.src[k], 1);
      stf(t.dst[k], 0, fr_add(a0, fr_mul(r, fr_sub(a1, a0))));
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const Fr v = ldf(fold ? t.dst[0] : t.src[0], 0);
    if (proof_value) finish_value(S, v, final_out, proof_value);
    else *final_out = v;
  }
}

// U[c] = Cu[c] EC[c], V[c] = Cv[c] EC[c]; SU, SV = their sums (one workgroup).
__global__ void __launch_bounds__(kBlock)
    k_copy_weights(const Fr* Cu, const Fr* Cv, const Fr* EC, Fr* U, Fr* V, uint64_t ncopies,
                   DevState* S) {
  Fr acc[2] = {fr_zero(), fr_zero()};
  for (uint64_t c = threadIdx.x; c < ncopies; c += kBlock) {
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

// Phase-2 sub-circuit tables over y (thread per y), the copy factors kept apart:
//   M[y,c] = U[c] Ma[y] + V[c] Mb[y],  A[y,c] = U[c] Aa[y] + V[c] Ab[y]
//   Ma[y] = sum_{MUL z: y_z=y} aU[z] EL[x_z] (Mb with bV; Aa, Ab over ADD gates)
//   Fa = vx Ma + Aa, Fb = vx Mb + Ab, Ka = vx Aa, Kb = vx Ab, Ks = SU Ka + SV Kb.
__global__ void __launch_bounds__(kBlock)
    k_phase2_tables(const uint32_t* __restrict__ yrow, const uint2* __restrict__ yent,
                    const Fr* __restrict__ aU, const Fr* __restrict__ bV,
                    const Fr* __restrict__ EL, const DevState* S, Fr* Fa, Fr* Fb, Fr* Ka,
                    Fr* Kb, Fr* Ks, uint64_t count) {
  const Fr vx = S->vx, su = S->su, sv = S->sv;
  for (uint64_t y = gtid(); y < count; y += gstride()) {
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
    stf(Fa, y, fr_add(fr_mul(vx, ma), aa));
    stf(Fb, y, fr_add(fr_mul(vx, mb), ab));
    stf(Ka, y, ka);
    stf(Kb, y, kb);
    stf(Ks, y, fr_add(fr_mul(su, ka), fr_mul(sv, kb)));
  }
}

// Row sums over the copies: P[y] = sum_c U[c] W[y,c], Q[y] = sum_c V[c] W[y,c].
// A row of 2^n entries is handled by tpr = min(256, 2^n) threads.
__global__ void __launch_bounds__(kBlock)
    k_copy_contract(const Fr* __restrict__ W, const Fr* __restrict__ U, const Fr* __restrict__ V,
                    Fr* __restrict__ P, Fr* __restrict__ Q, uint32_t n, uint64_t rows) {
  __shared__ Fr sp[kBlock], sq[kBlock];
  const uint32_t tpr_log = n < 8 ? n : 8;
  const uint32_t tpr = 1u << tpr_log;
  const uint64_t row = (uint64_t)blockIdx.x * (kBlock >> tpr_log) + (threadIdx.x >> tpr_log);
  const uint32_t lane = threadIdx.x & (tpr - 1);
  Fr p = fr_zero(), q = fr_zero();
  if (row < rows) {
    const uint64_t ncop = 1ull << n;
    for (uint64_t c = lane; c < ncop; c += tpr) {
      const Fr w = ldf(W, (row << n) | c);
      p = fr_add(p, fr_mul(ldf(U, c), w));
      q = fr_add(q, fr_mul(ldf(V, c), w));
    }
  }
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
    stf(P, row, sp[threadIdx.x]);
    stf(Q, row, sq[threadIdx.x]);
  }
}

// Column sums over the sub-circuit variables, first stage:
// part[c * R + k] = sum_{y in chunk k} EqR[y] W[y,c] (R = ychunks chunks of rows),
// one thread per (column, chunk); each column's partials are contiguous.
__global__ void __launch_bounds__(kBlock)
    k_local_contract(const Fr* __restrict__ W, const Fr* __restrict__ EqR, Fr* __restrict__ part,
                     uint32_t n, uint64_t rows, uint32_t ychunks) {
  const uint64_t ncop = 1ull << n;
  const uint64_t c = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint32_t k = blockIdx.y;
  if (c >= ncop) return;
  const uint64_t per = (rows + ychunks - 1) / ychunks;
  const uint64_t y0 = k * per, y1 = (y0 + per < rows) ? y0 + per : rows;
  Fr acc = fr_zero();
  for (uint64_t y = y0; y < y1; ++y) acc = fr_add(acc, fr_mul(ldf(EqR, y), ldf(W, (y << n) | c)));
  stf(part, c * ychunks + k, acc);
}

// Second stage: the copy tables of phase 2. A column's R partials are summed
// by tpc = min(256, R) threads:
// Wc[c] = sum_k part[c*R + k], Fc[c] = U[c] Fa~ + V[c] Fb~, Kc[c] = U[c] Ka~ + V[c] Kb~.
__global__ void __launch_bounds__(kBlock)
    k_copy_tables(const Fr* __restrict__ part, uint32_t ychunks, const Fr* __restrict__ U,
                  const Fr* __restrict__ V, const Fr* fa_f, const Fr* fb_f, const DevState* S,
                  Fr* Wc, Fr* Fc, Fr* Kc, uint64_t ncop) {
  __shared__ Fr sw[kBlock];
  const uint32_t tpc_log = 31 - __clz(ychunks < kBlock ? ychunks : kBlock);
  const uint32_t tpc = 1u << tpc_log;
  const uint64_t c = (uint64_t)blockIdx.x * (kBlock >> tpc_log) + (threadIdx.x >> tpc_log);
  const uint32_t lane = threadIdx.x & (tpc - 1);
  Fr w = fr_zero();
  if (c < ncop)
    for (uint32_t k = lane; k < ychunks; k += tpc) w = fr_add(w, ldf(part, c * ychunks + k));
  sw[threadIdx.x] = w;
  __syncthreads();
  for (uint32_t s = tpc / 2; s >= 1; s >>= 1) {
    if (lane < s) sw[threadIdx.x] = fr_add(sw[threadIdx.x], sw[threadIdx.x + s]);
    __syncthreads();
  }
  if (lane == 0 && c < ncop) {
    const Fr u = ldf(U, c), v = ldf(V, c);
    stf(Wc, c, sw[threadIdx.x]);
    stf(Fc, c, fr_add(fr_mul(u, *fa_f), fr_mul(v, *fb_f)));
    stf(Kc, c, fr_add(fr_mul(u, S->ka_f), fr_mul(v, S->kb_f)));
  }
}

// Ka~, Kb~ at the phase-2 local point: dot products with EqR (one workgroup).
__global__ void __launch_bounds__(kBlock)
    k_local_values(const Fr* EqR, const Fr* Ka, const Fr* Kb, uint64_t rows, DevState* S) {
  Fr acc[2] = {fr_zero(), fr_zero()};
  for (uint64_t y = threadIdx.x; y < rows; y += kBlock) {
    const Fr e = ldf(EqR, y);
    acc[0] = fr_add(acc[0], fr_mul(e, ldf(Ka, y)));
    acc[1] = fr_add(acc[1], fr_mul(e, ldf(Kb, y)));
  }
  block_reduce<2>(acc);
  if (threadIdx.x == 0) {
    S->ka_f = acc[0];
    S->kb_f = acc[1];
  }
}

// ABI plumbing: transcript state bytes <-> device state, canonical <-> Montgomery scalars.
__global__ void k_state_export(const DevState* S, uint8_t* out) {
  if (threadIdx.x < 8) {
    const uint32_t h = S->st[threadIdx.x];
    out[4 * threadIdx.x + 0] = (uint8_t)(h >> 24);
    out[4 * threadIdx.x + 1] = (uint8_t)(h >> 16);
    out[4 * threadIdx.x + 2] = (uint8_t)(h >> 8);
    out[4 * threadIdx.x + 3] = (uint8_t)h;
  }
}

__global__ void k_state_import(DevState* S, const uint8_t* in) {
  if (threadIdx.x < 8) {
    const uint8_t* b = in + 4 * threadIdx.x;
    S->st[threadIdx.x] = ((uint32_t)b[0] << 24) | ((uint32_t)b[1] << 16) | ((uint32_t)b[2] << 8) | b[3];
  }
  if (threadIdx.x == 0) S->counter = 0;
}

// ------------------------------------------------------------ launchers

static inline uint32_t grid_for(uint64_t n, uint32_t cap) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

constexpr uint32_t kSweepBlocks = 65535u * 8;  // grid-stride cap of plain sweeps
constexpr double kE = 32.0;                     // bytes per field element

// Bracket a launch with the optional timing events of its kernel class.
#define GKR_LAUNCH(cls, bytes, mulmods, stream, ...)            \
  do {                                                          \
    const int tok_ = prof_begin(stream);                        \
    __VA_ARGS__;                                                \
    if (tok_ >= 0) prof_end(tok_, stream, cls, bytes, mulmods); \
  } while (0)

void launch_to_mont(const gkr_fr* in, Fr* out, uint64_t n, hipStream_t s) {
  GKR_LAUNCH(PC_CONVERT, 2 * kE * n, (double)n, s,
             k_to_mont<<<grid_for(n, kSweepBlocks), kBlock, 0, s>>>(in, out, n));
}
void launch_from_mont(const Fr* in, gkr_fr* out, uint64_t n, hipStream_t s) {
  GKR_LAUNCH(PC_CONVERT, 2 * kE * n, (double)n, s,
             k_from_mont<<<grid_for(n, kSweepBlocks), kBlock, 0, s>>>(in, out, n));
}
void launch_forward(const Fr* W, Fr* V, const uint2* gates, uint32_t n, uint64_t count,
                    uint64_t mul_gates, hipStream_t s) {
  GKR_LAUNCH(PC_FORWARD, 3 * kE * count, (double)mul_gates, s,
             k_forward<<<grid_for(count, kSweepBlocks), kBlock, 0, s>>>(W, V, gates, n, count));
}
void launch_digest_level(const uint32_t* in, uint64_t nwords, int swap, uint32_t* out,
                         uint64_t nchunks, hipStream_t s) {
  GKR_LAUNCH(PC_DIGEST, 4.0 * nwords + 32.0 * nchunks, 0.0, s,
             k_digest_level<<<grid_for(nchunks, kSweepBlocks), kBlock, 0, s>>>(in, nwords, swap, out, nchunks));
}
void launch_transcript_begin(DevState* S, const Words8& seed_state, const Words8& circ,
                             const uint32_t* din, const uint32_t* dout, hipStream_t s) {
  GKR_LAUNCH(PC_TRANSCRIPT, 0.0, 0.0, s, k_transcript_begin<<<1, 64, 0, s>>>(S, seed_state, circ, din, dout));
}
void launch_squeeze(DevState* S, Fr* out, uint32_t count, hipStream_t s) {
  GKR_LAUNCH(PC_TRANSCRIPT, 0.0, (double)count, s, k_squeeze<<<1, 64, 0, s>>>(S, out, count));
}
void launch_layer_begin(DevState* S, int first, const Fr* vu, const Fr* vv, hipStream_t s) {
  GKR_LAUNCH(PC_TRANSCRIPT, 0.0, 4.0, s, k_layer_begin<<<1, 64, 0, s>>>(S, first, vu, vv));
}
void launch_eq_tables(const EqJobs& jobs, hipStream_t s) {
  uint64_t total = 0;
  double mm = 0;
  for (int j = 0; j < jobs.count; ++j) {
    total += 1ull << jobs.bits[j];
    mm += (double)(1ull << jobs.bits[j]) * (jobs.bits[j] + 1);
  }
  GKR_LAUNCH(PC_EQ, kE * total, mm, s, k_eq_tables<<<grid_for(total, 1u << 30), kBlock, 0, s>>>(jobs));
}
void launch_weighted_sum(const Fr* V, const Fr* A, const Fr* B, uint32_t n, uint64_t count,
                         Fr* partials, uint32_t* counter, Fr* dst, uint32_t max_blocks, hipStream_t s) {
  GKR_LAUNCH(PC_CLAIM, kE * count, 2.0 * count, s,
             k_weighted_sum<<<grid_for(count, max_blocks), kBlock, 0, s>>>(V, A, B, n, count, partials, counter, dst));
}
void launch_phase1_init_round(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU,
                              const Fr* bV, const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t half,
                              uint64_t gates, DevState* S, Fr* partials, Fr* r_out, uint32_t* msg,
                              uint32_t max_blocks, hipStream_t s) {
  GKR_LAUNCH(PC_PHASE1_INIT, kE * (gates + 6.0 * half), 3.0 * gates + 2.0 * half, s,
             k_phase1_init_round<<<grid_for(half, max_blocks), kBlock, 0, s>>>(W, G, H, lw.xrow, lw.xent, aU, bV, Cu, Cv, n, half, S, partials, r_out, msg));
}
void launch_phase1_init(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU,
                        const Fr* bV, const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t count,
                        uint64_t gates, hipStream_t s) {
  GKR_LAUNCH(PC_PHASE1_INIT, kE * (gates + 2.0 * count), 3.0 * gates, s,
             k_phase1_init<<<grid_for(count, kSweepBlocks), kBlock, 0, s>>>(W, G, H, lw.xrow, lw.xent, aU, bV, Cu, Cv, n, count));
}

// Algorithmic bytes and products of one round over `half` pairs of NT tables.
static inline void round_work(int nt, int eval_products, uint64_t half, bool fold, double& bytes,
                              double& mm) {
  const double h = (double)half;
  bytes += fold ? kE * nt * 6.0 * h : kE * nt * 2.0 * h;
  mm += (fold ? 2.0 * nt * h : 0.0) + eval_products * 2.0 * h;
}

template <class Form>
void launch_round(const Tabs<Form::NT>& t, uint64_t half, const Fr* rprev, DevState* S,
                  Fr* partials, Fr* r_out, uint32_t* msg, uint32_t max_blocks, hipStream_t s) {
  double bytes = 0, mm = 0;
  round_work(Form::NT, Form::NT == 3 ? 1 : 2, half, rprev != nullptr, bytes, mm);
  GKR_LAUNCH(Form::NT == 3 ? PC_ROUND_A : PC_ROUND_B, bytes, mm, s,
             k_round<Form><<<grid_for(half, max_blocks), kBlock, 0, s>>>(t, half, rprev, S, partials, r_out, msg));
}
template <class Form>
void launch_tail(const Tabs<Form::NT>& t, uint64_t size, const Fr* rpending, uint32_t rounds,
                 DevState* S, Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value,
                 hipStream_t s) {
  double bytes = 0, mm = 0;
  bool fold = rpending != nullptr;
  uint64_t sz = size;
  for (uint32_t j = 0; j < rounds; ++j) {
    const uint64_t eval = fold ? sz / 2 : sz;
    round_work(Form::NT, Form::NT == 3 ? 1 : 2, eval / 2, fold, bytes, mm);
    fold = true;
    sz = eval;
  }
  if (fold) mm += Form::NT;
  GKR_LAUNCH(Form::NT == 3 ? PC_TAIL_A : PC_TAIL_B, bytes, mm, s,
             k_tail<Form><<<1, kBlock, 0, s>>>(t, size, rpending, rounds, S, r_out, msg, final_out, proof_value));
}
template void launch_round<FormA>(const Tabs<3>&, uint64_t, const Fr*, DevState*, Fr*, Fr*, uint32_t*, uint32_t, hipStream_t);
template void launch_round<FormB>(const Tabs<5>&, uint64_t, const Fr*, DevState*, Fr*, Fr*, uint32_t*, uint32_t, hipStream_t);
template void launch_tail<FormA>(const Tabs<3>&, uint64_t, const Fr*, uint32_t, DevState*, Fr*, uint32_t*, Fr*, uint32_t*, hipStream_t);
template void launch_tail<FormB>(const Tabs<5>&, uint64_t, const Fr*, uint32_t, DevState*, Fr*, uint32_t*, Fr*, uint32_t*, hipStream_t);

void launch_copy_weights(const Fr* Cu, const Fr* Cv, const Fr* EC, Fr* U, Fr* V, uint64_t ncop,
                         DevState* S, hipStream_t s) {
  GKR_LAUNCH(PC_SMALL, 5 * kE * ncop, 2.0 * ncop, s, k_copy_weights<<<1, kBlock, 0, s>>>(Cu, Cv, EC, U, V, ncop, S));
}
void launch_phase2_tables(const LayerWiring& lw, const Fr* aU, const Fr* bV, const Fr* EL,
                          const DevState* S, Fr* Fa, Fr* Fb, Fr* Ka, Fr* Kb, Fr* Ks, uint64_t count,
                          uint64_t gates, hipStream_t s) {
  GKR_LAUNCH(PC_PHASE2_TABLES, kE * (3.0 * gates + 5.0 * count), 2.0 * gates + 8.0 * count, s,
             k_phase2_tables<<<grid_for(count, kSweepBlocks), kBlock, 0, s>>>(lw.yrow, lw.yent, aU, bV, EL, S, Fa, Fb, Ka, Kb, Ks, count));
}
void launch_copy_contract(const Fr* W, const Fr* U, const Fr* V, Fr* P, Fr* Q, uint32_t n,
                          uint64_t rows, hipStream_t s) {
  const uint32_t tpr_log = n < 8 ? n : 8;
  const uint64_t rows_per_block = kBlock >> tpr_log;
  const uint64_t grid = (rows + rows_per_block - 1) / rows_per_block;
  const double elems = (double)(rows << n);
  GKR_LAUNCH(PC_COPY_CONTRACT, kE * elems, 2.0 * elems, s,
             k_copy_contract<<<(uint32_t)grid, kBlock, 0, s>>>(W, U, V, P, Q, n, rows));
}
void launch_local_contract(const Fr* W, const Fr* EqR, Fr* part, uint32_t n, uint64_t rows,
                           uint32_t ychunks, hipStream_t s) {
  const uint64_t ncop = 1ull << n;
  dim3 grid((uint32_t)((ncop + kBlock - 1) / kBlock), ychunks);
  const double elems = (double)(rows << n);
  GKR_LAUNCH(PC_LOCAL_CONTRACT, kE * elems, elems, s,
             k_local_contract<<<grid, kBlock, 0, s>>>(W, EqR, part, n, rows, ychunks));
}
void launch_copy_tables(const Fr* part, uint32_t ychunks, const Fr* U, const Fr* V, const Fr* fa_f,
                        const Fr* fb_f, const DevState* S, Fr* Wc, Fr* Fc, Fr* Kc, uint64_t ncop,
                        hipStream_t s) {
  uint32_t tpc_log = 0;
  while (tpc_log < 8 && (2u << tpc_log) <= ychunks) ++tpc_log;
  const uint64_t cols_per_block = kBlock >> tpc_log;
  const uint64_t grid = (ncop + cols_per_block - 1) / cols_per_block;
  GKR_LAUNCH(PC_SMALL, kE * (ychunks + 5.0) * ncop, 4.0 * ncop, s,
             k_copy_tables<<<(uint32_t)grid, kBlock, 0, s>>>(part, ychunks, U, V, fa_f, fb_f, S, Wc, Fc, Kc, ncop));
}
void launch_local_values(const Fr* EqR, const Fr* Ka, const Fr* Kb, uint64_t rows, DevState* S,
                         hipStream_t s) {
  GKR_LAUNCH(PC_SMALL, 3 * kE * rows, 2.0 * rows, s, k_local_values<<<1, kBlock, 0, s>>>(EqR, Ka, Kb, rows, S));
}
void launch_state_export(const DevState* S, uint8_t* out, hipStream_t s) {
  GKR_LAUNCH(PC_SMALL, 0.0, 0.0, s, k_state_export<<<1, 64, 0, s>>>(S, out));
}
void launch_state_import(DevState* S, const uint8_t* in, hipStream_t s) {
  GKR_LAUNCH(PC_SMALL, 0.0, 0.0, s, k_state_import<<<1, 64, 0, s>>>(S, in));
}

}  // namespace gkr
