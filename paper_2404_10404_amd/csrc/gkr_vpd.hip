// The commitment to the input layer and its opening at the last layer's two
// points (Section 2.4: the prover commits to V_D~ before the GKR protocol and
// opens it at the two final points; the verifier never reads the inputs):
// kernels for gfx950, the step program and the C ABI of committed proofs.
//
// Construction (one reading of Virgo's transparent delegation, whose details
// the paper leaves to Virgo): the N = 2^s inputs are the coefficients of
// f(X) = sum_b V[b] X^b; the tensor sum_b eq(r, b) Y^b is a product of s
// binomials, so q (the eq weights, reversed) is evaluated by the verifier in
// O(s) at any point. The claims c1 + lam c2 = sum_b V[b] w[b] become the
// univariate-sumcheck identity f q = c + X g' + (X^N - 1) h on H = <w_N>, and
// FRI over L = 5 <w_M>, M = 4N, tests R = a0 f + a1 h + a2 g' + a3 X g' for
// degree < N. Tables over a coset are stored in bit-reversed order, so the
// (x, -x) pair of a fold is adjacent and a fold maps positions 2u, 2u + 1 to u.
//
// Work per opening for N inputs: NTTs of sizes 2N (three) and 4N (two, plus
// one for the commitment), Merkle trees over 2N leaves (f, then h with g'),
// FRI layers of 2N, N, ... entries with their trees.
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gkr_bodies.hpp"
#include "gkr_profile.hpp"
#include "gkr_program.hpp"
#include "gkr_vpd.hpp"

namespace gkr {

static_assert(offsetof(VpdState, beta) == offsetof(VpdState, a) + 4 * sizeof(Fr),
              "a and beta are squeezed as one run");

// ---------------------------------------------------------------- host constants

static Fr fr_pow_limbs(const Fr& base, const uint32_t e[8]) {
  Fr acc = fr_one();
  for (int w = 7; w >= 0; --w)
    for (int b = 31; b >= 0; --b) {
      acc = fr_mul(acc, acc);
      if ((e[w] >> b) & 1) acc = fr_mul(acc, base);
    }
  return acc;
}

Fr fr_pow_u64(const Fr& base, uint64_t e) {
  Fr acc = fr_one(), b = base;
  while (e) {
    if (e & 1) acc = fr_mul(acc, b);
    b = fr_mul(b, b);
    e >>= 1;
  }
  return acc;
}

Fr fr_inverse(const Fr& a) {
  uint32_t e[8];
  for (int k = 0; k < 8; ++k) e[k] = p_limb(k);
  e[0] -= 2;  // p - 2 (the low limb of p is 0xf0000001)
  return fr_pow_limbs(a, e);
}

Fr vpd_shift() { return fr_to_mont(fr_make(5, 0, 0, 0, 0, 0, 0, 0)); }

Fr vpd_root_of_unity(uint32_t log_m) {
  // 5^((p - 1) / 2^28) has order 2^28 (5 is a quadratic non-residue)
  uint32_t e[8];
  for (int k = 0; k < 8; ++k) e[k] = p_limb(k);
  e[0] -= 1;
  for (int k = 0; k < 8; ++k) e[k] = (e[k] >> 28) | (k < 7 ? e[k + 1] << 4 : 0);
  Fr w = fr_pow_limbs(vpd_shift(), e);
  for (uint32_t i = log_m; i < 28; ++i) w = fr_mul(w, w);
  return w;
}

// ---------------------------------------------------------------- plan

static size_t vpd_align(size_t v) { return (v + 255) & ~(size_t)255; }

static uint32_t hi_bits(uint32_t bits) { return bits > kVpdLoBits ? bits - kVpdLoBits : 0; }

VpdPlan plan_vpd(uint32_t s, uint32_t queries, uint32_t n_copy_bits) {
  VpdPlan p;
  p.s = s;
  p.queries = queries;
  p.N = 1ull << s;
  p.M = p.N << kVpdLogBlowup;
  const size_t E = sizeof(Fr);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = vpd_align(off + bytes);
    return o;
  };
  const uint32_t logw = s + kVpdLogBlowup - 1;  // exponents of w_M below M / 2
  p.off_T = take(E * (p.M / 2));
  p.off_wlo = take(E << kVpdLoBits);
  p.off_whi = take(E << hi_bits(logw));
  p.off_wilo = take(E << kVpdLoBits);
  p.off_wihi = take(E << hi_bits(logw));
  p.off_glo = take(E << kVpdLoBits);
  p.off_ghi = take(E << hi_bits(s));
  p.off_fL = take(E * p.M);
  p.off_hL = take(E * p.M);
  p.off_gL = take(E * p.M);
  p.off_fri = take(E * p.M);
  p.off_treeF = take(32 * p.M);
  p.off_treeHG = take(32 * p.M);
  p.off_treeFri = take(32 * p.M);
  const uint32_t sig = s - std::min(s, n_copy_bits);
  p.off_EA = take(E << sig);
  p.off_EB = take(E << sig);
  p.off_EC = take(E << std::min(s, n_copy_bits));
  p.off_ED = take(E << std::min(s, n_copy_bits));
  p.off_state = take(sizeof(VpdState));
  p.total = off;
  return p;
}

static uint64_t query_units(uint32_t s) {
  const uint64_t d0 = s + kVpdLogBlowup - 1;
  uint64_t u = (2 + d0) + (4 + d0);
  for (uint32_t i = 1; i < s; ++i) u += 2 + d0 - i;
  return u;
}

size_t vpd_opening_bytes(uint32_t s, uint32_t queries) {
  return 32 * ((uint64_t)s + 1 + (uint64_t)queries * query_units(s));
}

namespace {

struct VpdBufs {
  Fr *T, *wlo, *whi, *wilo, *wihi, *glo, *ghi, *fL, *hL, *gL, *fri, *EA, *EB, *EC, *ED;
  uint32_t *treeF, *treeHG, *treeFri;
  VpdState* V;
};

VpdBufs vpd_bind(const VpdPlan& p, void* base) {
  char* b = static_cast<char*>(base);
  auto F = [&](size_t o) { return reinterpret_cast<Fr*>(b + o); };
  auto W = [&](size_t o) { return reinterpret_cast<uint32_t*>(b + o); };
  VpdBufs v;
  v.T = F(p.off_T); v.wlo = F(p.off_wlo); v.whi = F(p.off_whi); v.wilo = F(p.off_wilo); v.wihi = F(p.off_wihi);
  v.glo = F(p.off_glo); v.ghi = F(p.off_ghi);
  v.fL = F(p.off_fL); v.hL = F(p.off_hL); v.gL = F(p.off_gL); v.fri = F(p.off_fri);
  v.EA = F(p.off_EA); v.EB = F(p.off_EB); v.EC = F(p.off_EC); v.ED = F(p.off_ED);
  v.treeF = W(p.off_treeF); v.treeHG = W(p.off_treeHG); v.treeFri = W(p.off_treeFri);
  v.V = reinterpret_cast<VpdState*>(b + p.off_state);
  return v;
}

}  // namespace

// Digest index of level `lv` of a tree with nl leaves (levels stored one after another).
__host__ __device__ inline uint64_t level_offset(uint64_t nl, uint32_t lv) { return 2 * nl - 2 * (nl >> lv); }

// First entry of FRI layer i >= 1 in the fri region, and of its tree.
__host__ __device__ inline uint64_t fri_offset(uint64_t M, uint32_t i) { return M - 2 * (M >> i); }

// ---------------------------------------------------------------- device helpers

#define GTID ((uint64_t)blockIdx.x * kBlock + threadIdx.x)
#define GSTRIDE ((uint64_t)gridDim.x * kBlock)

__device__ __forceinline__ Fr words_fr(const uint32_t* w) {
  return fr_make(w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7]);
}

// base^e from the two-level power tables lo[e & 8191] hi[e >> 13].
__device__ __forceinline__ Fr pow2lvl(const Fr* lo, const Fr* hi, uint64_t e) {
  const Fr l = ldf(lo, e & ((1u << kVpdLoBits) - 1));
  const uint64_t h = e >> kVpdLoBits;
  return h ? fr_mul(ldf(hi, h), l) : l;
}

__device__ __forceinline__ uint32_t bitrev_bits(uint32_t v, uint32_t bits) {
  return bits ? (__builtin_bitreverse32(v) >> (32 - bits)) : 0u;
}

__device__ __forceinline__ void load_digest(const uint32_t* d, uint64_t i, uint32_t (&h)[8]) {
  const GlobalU4* q = (const GlobalU4*)(d + 8 * i);
  const U32x4 a = q[0], b = q[1];
  h[0] = a.x; h[1] = a.y; h[2] = a.z; h[3] = a.w; h[4] = b.x; h[5] = b.y; h[6] = b.z; h[7] = b.w;
}

__device__ __forceinline__ void store_digest(uint32_t* d, uint64_t i, const Sha256State& s) {
  GlobalU4* q = (GlobalU4*)(d + 8 * i);
  q[0] = U32x4{s.h[0], s.h[1], s.h[2], s.h[3]};
  q[1] = U32x4{s.h[4], s.h[5], s.h[6], s.h[7]};
}

// One 64-byte block from two elements (Montgomery forms, little-endian bytes).
__device__ __forceinline__ Sha256Block pair_block(const Fr& a, const Fr& b) {
  Sha256Block blk;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    blk.w[k] = bswap32(a.v[k]);
    blk.w[8 + k] = bswap32(b.v[k]);
  }
  return blk;
}

__device__ __forceinline__ Sha256State node_hash(const uint32_t (&l)[8], const uint32_t (&r)[8]) {
  Sha256Block blk;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    blk.w[k] = l[k];
    blk.w[8 + k] = r[k];
  }
  return sha256_compress_v(sha256_iv(), blk);
}

__device__ void absorb_tagged_digest(Sha256State& st, uint32_t tag, const uint32_t* d) {
  uint32_t w[17];
#pragma unroll
  for (int k = 0; k < 8; ++k) w[k] = st.h[k];
  w[8] = tag;
#pragma unroll
  for (int k = 0; k < 8; ++k) w[9 + k] = d[k];
  st = sha256_fixed<17>(w);
}

// ---------------------------------------------------------------- kernels

// ST_VPD_POWERS: p0[i] = base^i for i < q0; base = w[0..7] (Montgomery).
__global__ void __launch_bounds__(kBlock) k_vpd_powers(Step st) {
  Fr* out = P<Fr*>(st, 0);
  const Fr base = words_fr(st.w);
  for (uint64_t i = GTID; i < st.q[0]; i += GSTRIDE) {
    Fr acc = fr_one(), b = base;
    for (uint64_t e = i; e; e >>= 1) {
      if (e & 1) acc = fr_mul(acc, b);
      b = fr_mul(b, b);
    }
    stf(out, i, acc);
  }
}

// ST_VPD_TWIDDLES: p0[t] = w_M^t for t < q0, from the power tables p1 (lo), p2 (hi).
__global__ void __launch_bounds__(kBlock) k_vpd_twiddles(Step st) {
  Fr* T = P<Fr*>(st, 0);
  const Fr *lo = P<const Fr*>(st, 1), *hi = P<const Fr*>(st, 2);
  for (uint64_t t = GTID; t < st.q[0]; t += GSTRIDE) stf(T, t, pow2lvl(lo, hi, t));
}

// ST_VPD_SCALE: the coefficient vector of an NTT input, zero padded to q0 entries:
//   u0 = 0: src[j]                          (j < N)
//   u0 = 1: src[j + N]                      (j < N; h from p)
//   u0 = 2: src[j + 1] + src[j + 1 + N]     (j < N - 1; g' from p)
//   u0 = 3: w[(N - j) mod N], w[b] = EA[b >> n] EC[b & mask] + EB[b >> n] ED[b & mask]  (q)
// times 5^j when u1 != 0. p0 src, p1 dst, p2 glo, p3 ghi, p4..p7 EA, EB, EC, ED, u2 n, q0 size, q1 N.
__global__ void __launch_bounds__(kBlock) k_vpd_scale(Step st) {
  const Fr* src = P<const Fr*>(st, 0);
  Fr* dst = P<Fr*>(st, 1);
  const Fr *glo = P<const Fr*>(st, 2), *ghi = P<const Fr*>(st, 3);
  const uint32_t mode = st.u[0], n = st.u[2];
  const uint64_t N = st.q[1], mask = (1ull << n) - 1;
  for (uint64_t j = GTID; j < st.q[0]; j += GSTRIDE) {
    Fr v = fr_zero();
    if (j < N) {
      if (mode == 0) {
        v = ldf(src, j);
      } else if (mode == 1) {
        v = ldf(src, j + N);
      } else if (mode == 2) {
        if (j + 1 < N) v = fr_add(ldf(src, j + 1), ldf(src, j + 1 + N));
      } else {
        const uint64_t b = (N - j) & (N - 1);
        v = fr_mul_add2(ldf(P<const Fr*>(st, 4), b >> n), ldf(P<const Fr*>(st, 6), b & mask),
                        ldf(P<const Fr*>(st, 5), b >> n), ldf(P<const Fr*>(st, 7), b & mask));
      }
      if (st.u[1]) v = fr_mul(v, pow2lvl(glo, ghi, j));
    }
    stf(dst, j, v);
  }
}

// ST_VPD_NTT: W radix-2 stages j0 .. j0+W-1 of an in-place transform of size
// 2^L over p0, in one pass through LDS. A workgroup takes a tile of 2^W rows
// (the index bits L-j0-W .. L-j0-1) by 2^c columns (consecutive low bits),
// W + c <= 11. Forward (u5 = 0): decimation in frequency, natural order in,
// bit-reversed out; stage j maps (a, b) at distance 2^(L-1-j) to
// (a + b, (a - b) w^k). Inverse (u5 = 1): the stages undone in reverse order,
// (a, b) -> (a + b w^-k, a - b w^-k), then a scale by w[0..7] when u4 has
// bit 8 set. Twiddles w^k = T[k << (j + tshift)] with T[t] = w_{2^(L+tshift)}^t;
// w^-t = -T[n_T/2 - t]. Stages go two at a time: a thread holds the four
// elements that two consecutive stages combine (rows r, r + h/2, r + h,
// r + 3h/2), so a pair of stages costs one LDS round trip and one barrier;
// an odd last stage is a plain radix-2 step.
// p0 x, p1 T, u0 L, u1 j0, u2 W, u3 c, u4 tshift (| 256: scale), u5 inverse, q0 n_T / 2.
constexpr int kNttTile = 2048;
constexpr int kNttThreads = 512;

// v w^(+-1) for twiddle index t (no product when t = 0).
__device__ __forceinline__ Fr tw_mul(const Fr& v, const Fr* T, uint64_t t, uint64_t halfT, bool inverse) {
  if (t == 0) return v;
  return inverse ? fr_neg(fr_mul(v, ldf(T, halfT - t))) : fr_mul(v, ldf(T, t));
}

__global__ void __launch_bounds__(kNttThreads) k_vpd_ntt(Step st) {
  __shared__ Fr tile[kNttTile];
  Fr* x = P<Fr*>(st, 0);
  const Fr* T = P<const Fr*>(st, 1);
  const uint32_t L = st.u[0], j0 = st.u[1], W = st.u[2], c = st.u[3];
  const uint32_t tshift = st.u[4] & 255u;
  const bool do_scale = (st.u[4] >> 8) & 1u;
  const bool inverse = st.u[5] != 0;
  const uint64_t halfT = st.q[0];
  const uint32_t lo = L - j0 - W;
  const uint32_t C = 1u << c;
  const uint32_t nelem = 1u << (W + c);
  const uint64_t colgroup = blockIdx.x & ((1ull << (lo - c)) - 1);
  const uint64_t blk = blockIdx.x >> (lo - c);
  const uint64_t base = (blk << (L - j0)) + (colgroup << c);
  for (uint32_t e = threadIdx.x; e < nelem; e += kNttThreads) {
    const uint32_t r = e >> c, col = e & (C - 1);
    tile[e] = ldf(x, base + ((uint64_t)r << lo) + col);
  }
  __syncthreads();
  const uint32_t npairs = W / 2, nops = npairs + (W & 1);
  for (uint32_t op = 0; op < nops; ++op) {
    const uint32_t fo = inverse ? (nops - 1 - op) : op;  // position in the forward order
    if (fo == npairs) {
      // the odd last stage (jj = W - 1, distance one row)
      const uint32_t j = j0 + W - 1;
      for (uint32_t bi = threadIdx.x; bi < nelem / 2; bi += kNttThreads) {
        const uint32_t col = bi & (C - 1), ra = (bi >> c) * 2;
        const uint64_t t = ((colgroup << c) + col) << (j + tshift);
        const uint32_t ia = (ra << c) + col, ib = ia + C;
        const Fr a = tile[ia], b = tile[ib];
        if (!inverse) {
          tile[ia] = fr_add(a, b);
          tile[ib] = tw_mul(fr_sub(a, b), T, t, halfT, false);
        } else {
          const Fr bw = tw_mul(b, T, t, halfT, true);
          tile[ia] = fr_add(a, bw);
          tile[ib] = fr_sub(a, bw);
        }
      }
    } else {
      const uint32_t jj = 2 * fo, j = j0 + jj;
      const uint32_t sh2 = W - 2 - jj;  // h/2 = 2^sh2 rows, h = 2^(sh2 + 1)
      const uint32_t h2 = 1u << sh2, hr = 2 * h2;
      for (uint32_t g = threadIdx.x; g < nelem / 4; g += kNttThreads) {
        const uint32_t col = g & (C - 1), gr = g >> c;
        const uint32_t r0 = ((gr >> sh2) << (sh2 + 2)) + (gr & (h2 - 1));
        const uint32_t i0 = (r0 << c) + col, i1 = ((r0 + h2) << c) + col;
        const uint32_t i2 = ((r0 + hr) << c) + col, i3 = ((r0 + hr + h2) << c) + col;
        const uint64_t ka = ((uint64_t)(gr & (h2 - 1)) << lo) + (colgroup << c) + col;
        const uint64_t kb = ka + ((uint64_t)h2 << lo);
        const uint64_t ta = ka << (j + tshift), tb = kb << (j + tshift), tc = ka << (j + 1 + tshift);
        const Fr x0 = tile[i0], x1 = tile[i1], x2 = tile[i2], x3 = tile[i3];
        if (!inverse) {
          const Fr a0 = fr_add(x0, x2), a2 = tw_mul(fr_sub(x0, x2), T, ta, halfT, false);
          const Fr a1 = fr_add(x1, x3), a3 = tw_mul(fr_sub(x1, x3), T, tb, halfT, false);
          tile[i0] = fr_add(a0, a1);
          tile[i1] = tw_mul(fr_sub(a0, a1), T, tc, halfT, false);
          tile[i2] = fr_add(a2, a3);
          tile[i3] = tw_mul(fr_sub(a2, a3), T, tc, halfT, false);
        } else {
          const Fr t1 = tw_mul(x1, T, tc, halfT, true), t3 = tw_mul(x3, T, tc, halfT, true);
          const Fr b0 = fr_add(x0, t1), b1 = fr_sub(x0, t1), b2 = fr_add(x2, t3), b3 = fr_sub(x2, t3);
          const Fr u2 = tw_mul(b2, T, ta, halfT, true), u3 = tw_mul(b3, T, tb, halfT, true);
          tile[i0] = fr_add(b0, u2);
          tile[i1] = fr_add(b1, u3);
          tile[i2] = fr_sub(b0, u2);
          tile[i3] = fr_sub(b1, u3);
        }
      }
    }
    __syncthreads();
  }
  const Fr sc = words_fr(st.w);
  for (uint32_t e = threadIdx.x; e < nelem; e += kNttThreads) {
    const uint32_t r = e >> c, col = e & (C - 1);
    const Fr v = do_scale ? fr_mul(opaque(tile[e]), sc) : tile[e];
    stf(x, base + ((uint64_t)r << lo) + col, v);
  }
}

// ST_VPD_MUL: p0[i] *= p1[i] for i < q0.
__global__ void __launch_bounds__(kBlock) k_vpd_mul(Step st) {
  Fr* x = P<Fr*>(st, 0);
  const Fr* y = P<const Fr*>(st, 1);
  for (uint64_t i = GTID; i < st.q[0]; i += GSTRIDE) stf(x, i, fr_mul(ldf(x, i), ldf(y, i)));
}

// ST_VPD_LEAVES: leaf u (u < q0) digests positions 2u, 2u + 1 of p0 (one
// block), then of p1 if not null (a second block): the compression function
// chained from the initial value. p2 digests.
__global__ void __launch_bounds__(kBlock) k_vpd_leaves(Step st) {
  const Fr* A = P<const Fr*>(st, 0);
  const Fr* B = P<const Fr*>(st, 1);
  uint32_t* out = P<uint32_t*>(st, 2);
  for (uint64_t u = GTID; u < st.q[0]; u += GSTRIDE) {
    Sha256State h = sha256_compress_v(sha256_iv(), pair_block(ldf(A, 2 * u), ldf(A, 2 * u + 1)));
    if (B) h = sha256_compress_v(h, pair_block(ldf(B, 2 * u), ldf(B, 2 * u + 1)));
    store_digest(out, u, h);
  }
}

// ST_VPD_NODES: p1[i] = C(IV, p0[2i] || p0[2i + 1]) for i < q0.
__global__ void __launch_bounds__(kBlock) k_vpd_nodes(Step st) {
  const uint32_t* in = P<const uint32_t*>(st, 0);
  uint32_t* out = P<uint32_t*>(st, 1);
  for (uint64_t i = GTID; i < st.q[0]; i += GSTRIDE) {
    uint32_t l[8], r[8];
    load_digest(in, 2 * i, l);
    load_digest(in, 2 * i + 1, r);
    store_digest(out, i, node_hash(l, r));
  }
}

// ST_VPD_TREE_TOP (one workgroup): from a level of q0 <= 512 digests at p0,
// every level up to the root, written one after another from p0 + q0 digests.
constexpr uint32_t kTopMax = 512;

__global__ void __launch_bounds__(kBlock) k_vpd_tree_top(Step st) {
  __shared__ uint32_t lv[kTopMax][8];
  uint32_t* d = P<uint32_t*>(st, 0);
  uint32_t cnt = (uint32_t)st.q[0];
  for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) {
    uint32_t h[8];
    load_digest(d, i, h);
#pragma unroll
    for (int k = 0; k < 8; ++k) lv[i][k] = h[k];
  }
  __syncthreads();
  uint64_t out = cnt;
  while (cnt > 1) {
    const uint32_t half = cnt / 2;
    Sha256State h;
    const bool act = threadIdx.x < half;
    if (act) {
      uint32_t l[8], r[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        l[k] = lv[2 * threadIdx.x][k];
        r[k] = lv[2 * threadIdx.x + 1][k];
      }
      h = node_hash(l, r);
      store_digest(d, out + threadIdx.x, h);
    }
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k = 0; k < 8; ++k) lv[threadIdx.x][k] = h.h[k];
    }
    __syncthreads();
    out += half;
    cnt = half;
  }
}

// ST_VPD_BEGIN (one thread): lam = squeeze. p0 S, p1 V.
__global__ void k_vpd_begin(Step st) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  VpdState* V = P<VpdState*>(st, 1);
  Sha256State sh = load_state(S);
  V->lam = squeeze(sh);
  save_state(S, sh);
}

// ST_VPD_ABSORB (one thread): absorb("GKRM", root p1) and copy the root to
// the proof at p2 (big-endian bytes), then squeeze u0 challenges into p3.
// p0 S.
__global__ void k_vpd_absorb(Step st) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  const uint32_t* root = P<const uint32_t*>(st, 1);
  uint32_t* proof = P<uint32_t*>(st, 2);
  Fr* out = P<Fr*>(st, 3);
  Sha256State sh = load_state(S);
  uint32_t r[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) r[k] = root[k];
  absorb_tagged_digest(sh, kTagCommit, r);
#pragma unroll
  for (int k = 0; k < 8; ++k) proof[k] = bswap32(r[k]);
  for (uint32_t i = 0; i < st.u[0]; ++i) out[i] = squeeze(sh);
  save_state(S, sh);
}

// ST_VPD_ROOT_OUT (one thread): the root p0 as 32 big-endian bytes at p1.
__global__ void k_vpd_root_out(Step st) {
  if (threadIdx.x != 0) return;
  const uint32_t* root = P<const uint32_t*>(st, 0);
  uint32_t* proof = P<uint32_t*>(st, 1);
#pragma unroll
  for (int k = 0; k < 8; ++k) proof[k] = bswap32(root[k]);
}

// ST_VPD_FOLD0: the first fold, with R computed from the committed tables:
// at position pair (2u, 2u + 1) = (x, -x), x = 5 w_M^k, k = bitrev(u),
//   R(+-x) = a0 f + a1 h + (a2 +- a3 x) g',
//   out[u] = (R(x) + R(-x)) / 2 + beta0 (R(x) - R(-x)) / (2x).
// p0 fL, p1 hL, p2 gL, p3 out, p4 V, p5 wlo, p6 whi, p7 wilo, p8 wihi;
// w[0..7] = 5, w[8..15] = 1 / (2 * 5); u0 bits of u; q0 M / 2.
__global__ void __launch_bounds__(kBlock) k_vpd_fold0(Step st) {
  const Fr *fL = P<const Fr*>(st, 0), *hL = P<const Fr*>(st, 1), *gL = P<const Fr*>(st, 2);
  Fr* out = P<Fr*>(st, 3);
  const VpdState* V = P<const VpdState*>(st, 4);
  const Fr *wlo = P<const Fr*>(st, 5), *whi = P<const Fr*>(st, 6);
  const Fr *wilo = P<const Fr*>(st, 7), *wihi = P<const Fr*>(st, 8);
  const Fr gam = words_fr(st.w), ginv2 = words_fr(st.w + 8);
  const Fr a0 = opaque(V->a[0]), a1 = opaque(V->a[1]), a2 = opaque(V->a[2]), a3 = opaque(V->a[3]);
  const Fr cb = opaque(fr_mul(opaque(V->beta[0]), ginv2));
  for (uint64_t u = GTID; u < st.q[0]; u += GSTRIDE) {
    const uint64_t k = bitrev_bits((uint32_t)u, st.u[0]);
    const Fr x = fr_mul(gam, pow2lvl(wlo, whi, k));
    const Fr ax = fr_mul(a3, x);
    const Fr R0 = fr_add(fr_mul_add2(a0, ldf(fL, 2 * u), a1, ldf(hL, 2 * u)), fr_mul(fr_add(a2, ax), ldf(gL, 2 * u)));
    const Fr R1 = fr_add(fr_mul_add2(a0, ldf(fL, 2 * u + 1), a1, ldf(hL, 2 * u + 1)),
                         fr_mul(fr_sub(a2, ax), ldf(gL, 2 * u + 1)));
    const Fr winv = pow2lvl(wilo, wihi, k);
    stf(out, u, fr_add(fr_half(fr_add(R0, R1)), fr_mul(fr_mul(cb, fr_sub(R0, R1)), winv)));
  }
}

// ST_VPD_FOLD: layer i (p0, 2 q0 entries over the coset 5^(2^i) <w_M^(2^i)>)
// to layer i + 1 (p1): out[u] = (a + b) / 2 + beta_i (a - b) / (2x), with
// 1/x = 5^-(2^i) w_M^-(k 2^i), k = bitrev(u). p2 V, p3 wilo, p4 wihi;
// w[0..7] = 5^-(2^i) / 2; u0 bits of u, u1 i; q0 entries out.
__global__ void __launch_bounds__(kBlock) k_vpd_fold(Step st) {
  const Fr* in = P<const Fr*>(st, 0);
  Fr* out = P<Fr*>(st, 1);
  const VpdState* V = P<const VpdState*>(st, 2);
  const Fr *wilo = P<const Fr*>(st, 3), *wihi = P<const Fr*>(st, 4);
  const uint32_t i = st.u[1];
  const Fr cb = opaque(fr_mul(opaque(V->beta[i]), words_fr(st.w)));
  for (uint64_t u = GTID; u < st.q[0]; u += GSTRIDE) {
    const uint64_t k = bitrev_bits((uint32_t)u, st.u[0]);
    const Fr a = ldf(in, 2 * u), b = ldf(in, 2 * u + 1);
    const Fr winv = pow2lvl(wilo, wihi, k << i);
    stf(out, u, fr_add(fr_half(fr_add(a, b)), fr_mul(fr_mul(cb, fr_sub(a, b)), winv)));
  }
}

// ST_VPD_FINAL (one thread): the constant of the last layer p0 into the proof
// (p2, canonical) and the transcript ("GKRV"), then u0 query leaves
// (challenge mod q0) into V->idx. p1 S, p3 V.
__global__ void k_vpd_final(Step st) {
  if (threadIdx.x != 0) return;
  const Fr* last = P<const Fr*>(st, 0);
  DevState* S = P<DevState*>(st, 1);
  uint32_t* proof = P<uint32_t*>(st, 2);
  VpdState* V = P<VpdState*>(st, 3);
  const Fr c = fr_from_mont(opaque(last[0]));
  Sha256State sh = load_state(S);
  absorb_element(sh, kTagValue, c);
#pragma unroll
  for (int k = 0; k < 8; ++k) proof[k] = c.v[k];
  for (uint32_t q = 0; q < st.u[0]; ++q) {
    const Fr r = fr_from_mont(squeeze(sh));
    V->idx[q] = r.v[0] & (uint32_t)(st.q[0] - 1);
  }
  save_state(S, sh);
}

// ST_VPD_QUERIES: thread (query q, part) writes its part of query q's
// opening: part 0 the f leaf and path, part 1 the (h, g') leaf and path,
// part i + 1 (1 <= i < s) FRI layer i's leaf idx >> i and path. Elements
// canonical, digests as big-endian bytes. p0 V, p1 fL, p2 hL, p3 gL, p4 fri,
// p5 treeF, p6 treeHG, p7 treeFri, p8 proof (queries start); u0 s, u1 queries; q0 M.
__global__ void __launch_bounds__(kBlock) k_vpd_queries(Step st) {
  const VpdState* V = P<const VpdState*>(st, 0);
  const uint32_t s = st.u[0], nq = st.u[1];
  const uint64_t M = st.q[0];
  const uint32_t d0 = s + kVpdLogBlowup - 1;
  uint64_t qunits = (2 + d0) + (4 + d0);
  for (uint32_t i = 1; i < s; ++i) qunits += 2 + d0 - i;
  const uint64_t total = (uint64_t)nq * (s + 1);
  for (uint64_t g = GTID; g < total; g += GSTRIDE) {
    const uint32_t q = (uint32_t)(g / (s + 1)), part = (uint32_t)(g % (s + 1));
    const uint32_t u = V->idx[q];
    uint32_t* out = P<uint32_t*>(st, 8) + 8 * (qunits * q);
    const Fr* tabs[2];
    int ntab;
    const uint32_t* tree;
    uint64_t nl, leaf;
    if (part == 0) {
      out += 0;
      tabs[0] = P<const Fr*>(st, 1); ntab = 1;
      tree = P<const uint32_t*>(st, 5); nl = M / 2; leaf = u;
    } else if (part == 1) {
      out += 8 * (2 + d0);
      tabs[0] = P<const Fr*>(st, 2); tabs[1] = P<const Fr*>(st, 3); ntab = 2;
      tree = P<const uint32_t*>(st, 6); nl = M / 2; leaf = u;
    } else {
      const uint32_t i = part - 1;
      uint64_t off = (2 + d0) + (4 + d0);
      for (uint32_t k = 1; k < i; ++k) off += 2 + d0 - k;
      out += 8 * off;
      tabs[0] = P<const Fr*>(st, 4) + fri_offset(M, i); ntab = 1;
      tree = P<const uint32_t*>(st, 7) + 8 * fri_offset(M, i); nl = M >> (i + 1); leaf = u >> i;
    }
    uint32_t w = 0;
    for (int t = 0; t < ntab; ++t)
      for (int e = 0; e < 2; ++e) {
        const Fr c = fr_from_mont(ldf(tabs[t], 2 * leaf + e));
#pragma unroll
        for (int k = 0; k < 8; ++k) out[w + k] = c.v[k];
        w += 8;
      }
    const uint32_t depth = 31 - __builtin_clz((uint32_t)nl);
    for (uint32_t lv = 0; lv < depth; ++lv) {
      uint32_t h[8];
      load_digest(tree, level_offset(nl, lv) + ((leaf >> lv) ^ 1), h);
#pragma unroll
      for (int k = 0; k < 8; ++k) out[w + k] = bswap32(h[k]);
      w += 8;
    }
  }
}

#undef GTID
#undef GSTRIDE

void launch_vpd_step(const Step& st, hipStream_t s) {
  const int tok = prof_begin(s);
  const dim3 grid(st.ntiles), block(kBlock);
  ProfClass cls = PC_VPD_OTHER;
  switch (st.type) {
    case ST_VPD_POWERS: k_vpd_powers<<<grid, block, 0, s>>>(st); break;
    case ST_VPD_TWIDDLES: k_vpd_twiddles<<<grid, block, 0, s>>>(st); break;
    case ST_VPD_SCALE: k_vpd_scale<<<grid, block, 0, s>>>(st); break;
    case ST_VPD_NTT: k_vpd_ntt<<<grid, dim3(kNttThreads), 0, s>>>(st); cls = PC_VPD_NTT; break;
    case ST_VPD_MUL: k_vpd_mul<<<grid, block, 0, s>>>(st); break;
    case ST_VPD_LEAVES: k_vpd_leaves<<<grid, block, 0, s>>>(st); cls = PC_VPD_MERKLE; break;
    case ST_VPD_NODES: k_vpd_nodes<<<grid, block, 0, s>>>(st); cls = PC_VPD_MERKLE; break;
    case ST_VPD_TREE_TOP: k_vpd_tree_top<<<grid, block, 0, s>>>(st); cls = PC_VPD_MERKLE; break;
    case ST_VPD_BEGIN: k_vpd_begin<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_VPD_ABSORB: k_vpd_absorb<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_VPD_ROOT_OUT: k_vpd_root_out<<<grid, block, 0, s>>>(st); break;
    case ST_VPD_FOLD0: k_vpd_fold0<<<grid, block, 0, s>>>(st); cls = PC_VPD_FRI; break;
    case ST_VPD_FOLD: k_vpd_fold<<<grid, block, 0, s>>>(st); cls = PC_VPD_FRI; break;
    case ST_VPD_FINAL: k_vpd_final<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_VPD_QUERIES: k_vpd_queries<<<grid, block, 0, s>>>(st); break;
    default: break;
  }
  if (tok >= 0) prof_end(tok, s, cls, st.bytes, st.mulmods);
}

// ---------------------------------------------------------------- step program (host)

namespace {

constexpr uint32_t kVpdSweepTiles = 65535u * 8;
constexpr double kVE = 32.0;

uint32_t vtiles(uint64_t n) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > kVpdSweepTiles) g = kVpdSweepTiles;
  return (uint32_t)g;
}

Step vmk(uint32_t type, uint32_t ntiles) {
  Step st;
  memset(&st, 0, sizeof(st));
  st.type = type;
  st.ntiles = ntiles < 1 ? 1 : ntiles;
  return st;
}

void put_fr(uint32_t* w, const Fr& a) { memcpy(w, a.v, 32); }

void powers(Program& pg, Fr* out, const Fr& base, uint64_t count) {
  Step st = vmk(ST_VPD_POWERS, vtiles(count));
  st.p[0] = out; st.q[0] = count;
  put_fr(st.w, base);
  st.bytes = kVE * count; st.mulmods = 28.0 * count;
  pg.steps.push_back(st);
}

void scale(Program& pg, const VpdBufs& b, uint32_t mode, bool coset, const Fr* src, Fr* dst, uint64_t size,
           uint64_t N, uint32_t n) {
  Step st = vmk(ST_VPD_SCALE, vtiles(size));
  st.p[0] = src; st.p[1] = dst; st.p[2] = b.glo; st.p[3] = b.ghi;
  st.p[4] = b.EA; st.p[5] = b.EB; st.p[6] = b.EC; st.p[7] = b.ED;
  st.u[0] = mode; st.u[1] = coset ? 1 : 0; st.u[2] = n;
  st.q[0] = size; st.q[1] = N;
  st.bytes = kVE * (size + (mode == 2 ? 2 : 1) * N);
  st.mulmods = (coset ? 2.0 : 0.0) * N + (mode == 3 ? 2.0 * N : 0.0);
  pg.steps.push_back(st);
}

// Pass plan of a transform of size 2^L: strided passes of W <= 9 stages over
// the top L - 11 bits (as many columns as fit in a 2^11-element tile), then
// one contiguous pass over the last 11 stages.
struct NttPass {
  uint32_t j0, W, c;
};

std::vector<NttPass> ntt_plan(uint32_t L) {
  std::vector<NttPass> out;
  if (L <= 11) {
    out.push_back({0, L, 0});
    return out;
  }
  const uint32_t top = L - 11, k = (top + 8) / 9;
  uint32_t j0 = 0;
  for (uint32_t i = 0; i < k; ++i) {
    const uint32_t W = top / k + (i < top % k ? 1 : 0);
    const uint32_t lo = L - j0 - W;
    out.push_back({j0, W, std::min(11 - W, lo)});
    j0 += W;
  }
  out.push_back({j0, 11, 0});
  return out;
}

// Forward (natural -> bit-reversed) or inverse (bit-reversed -> natural,
// scaled by 1/2^L) transform of x (2^L entries); T holds w_{2^LT}^t, t < 2^(LT-1).
void ntt(Program& pg, Fr* x, uint32_t L, const Fr* T, uint32_t LT, bool inverse) {
  std::vector<NttPass> plan = ntt_plan(L);
  if (inverse) std::reverse(plan.begin(), plan.end());
  for (size_t i = 0; i < plan.size(); ++i) {
    const NttPass& ps = plan[i];
    Step st = vmk(ST_VPD_NTT, (uint32_t)(1ull << (L - ps.W - ps.c)));
    st.p[0] = x; st.p[1] = T;
    st.u[0] = L; st.u[1] = ps.j0; st.u[2] = ps.W; st.u[3] = ps.c; st.u[4] = LT - L; st.u[5] = inverse ? 1 : 0;
    st.q[0] = 1ull << (LT - 1);
    if (inverse && i + 1 == plan.size()) {
      st.u[4] |= 256u;
      put_fr(st.w, fr_inverse(fr_to_mont(fr_make(1u << L, 0, 0, 0, 0, 0, 0, 0))));  // L <= 28
    }
    const double n = (double)(1ull << L);
    st.bytes = 2 * kVE * n;
    st.mulmods = n / 2 * ps.W;
    pg.steps.push_back(st);
  }
}

// Merkle tree over nl leaves of (A, B) pairs; digests at tree (levels in order).
void tree(Program& pg, const Fr* A, const Fr* B, uint32_t* tree, uint64_t nl) {
  Step st = vmk(ST_VPD_LEAVES, vtiles(nl));
  st.p[0] = A; st.p[1] = B; st.p[2] = tree; st.q[0] = nl;
  st.bytes = kVE * 2 * nl * (B ? 2 : 1) + 32.0 * nl;
  pg.steps.push_back(st);
  uint64_t cnt = nl;
  uint32_t* lv = tree;
  while (cnt > kTopMax) {
    Step nd = vmk(ST_VPD_NODES, vtiles(cnt / 2));
    nd.p[0] = lv; nd.p[1] = lv + 8 * cnt; nd.q[0] = cnt / 2;
    nd.bytes = 32.0 * cnt * 1.5;
    pg.steps.push_back(nd);
    lv += 8 * cnt;
    cnt /= 2;
  }
  Step top = vmk(ST_VPD_TREE_TOP, 1);
  top.p[0] = lv; top.q[0] = cnt;
  top.bytes = 32.0 * cnt * 2;
  pg.steps.push_back(top);
}

}  // namespace

const uint32_t* vpd_root_words(const VpdPlan& vp, const void* base) {
  const uint32_t* t = reinterpret_cast<const uint32_t*>(static_cast<const char*>(base) + vp.off_treeF);
  return t + 8 * (vp.M - 2);  // level_offset(M/2, depth) = 2 (M/2) - 2
}

void emit_vpd_commit(Program& pg, const VpdPlan& vp, void* base, const Fr* d_vals) {
  const VpdBufs b = vpd_bind(vp, base);
  const uint32_t logM = vp.s + kVpdLogBlowup, logw = logM - 1;
  const Fr w = vpd_root_of_unity(logM), wi = fr_inverse(w), g = vpd_shift();
  const uint64_t lo = 1ull << kVpdLoBits;
  powers(pg, b.wlo, w, lo);
  powers(pg, b.whi, fr_pow_u64(w, lo), 1ull << hi_bits(logw));
  powers(pg, b.wilo, wi, lo);
  powers(pg, b.wihi, fr_pow_u64(wi, lo), 1ull << hi_bits(logw));
  powers(pg, b.glo, g, lo);
  powers(pg, b.ghi, fr_pow_u64(g, lo), 1ull << hi_bits(vp.s));
  {
    Step st = vmk(ST_VPD_TWIDDLES, vtiles(vp.M / 2));
    st.p[0] = b.T; st.p[1] = b.wlo; st.p[2] = b.whi; st.q[0] = vp.M / 2;
    st.bytes = kVE * (vp.M / 2); st.mulmods = (double)(vp.M / 2);
    pg.steps.push_back(st);
  }
  scale(pg, b, 0, true, d_vals, b.fL, vp.M, vp.N, 0);
  ntt(pg, b.fL, logM, b.T, logM, false);
  tree(pg, b.fL, nullptr, b.treeF, vp.M / 2);
}

void emit_vpd_root_out(Program& pg, const VpdPlan& vp, void* base, uint8_t* proof_out) {
  Step st = vmk(ST_VPD_ROOT_OUT, 1);
  st.p[0] = vpd_root_words(vp, base); st.p[1] = proof_out;
  pg.steps.push_back(st);
}

void emit_vpd_open(Program& pg, const VpdPlan& vp, void* base, const Fr* d_vals, DevState* S, const Fr* rx,
                   const Fr* ry, uint32_t sigma, uint32_t n, uint8_t* proof_out) {
  const VpdBufs b = vpd_bind(vp, base);
  const uint32_t s = vp.s, logM = s + kVpdLogBlowup;
  const uint64_t N = vp.N, M = vp.M;
  uint32_t* proof = reinterpret_cast<uint32_t*>(proof_out);
  {
    Step st = vmk(ST_VPD_BEGIN, 1);
    st.p[0] = S; st.p[1] = b.V;
    pg.steps.push_back(st);
  }
  {
    const uint32_t bits[4] = {sigma, sigma, n, n};
    const Fr* pts[4] = {rx, ry, rx + sigma, ry + sigma};
    const Fr* scl[4] = {nullptr, &b.V->lam, nullptr, nullptr};
    Fr* outs[4] = {b.EA, b.EB, b.EC, b.ED};
    pg.eq(4, bits, pts, scl, outs);
  }
  // p = f q through transforms of size 2N (the fri region is free until the first fold)
  Fr* buf1 = b.fri;
  Fr* buf2 = b.fri + 2 * N;
  scale(pg, b, 0, false, d_vals, buf1, 2 * N, N, 0);
  scale(pg, b, 3, false, nullptr, buf2, 2 * N, N, n);
  ntt(pg, buf1, s + 1, b.T, logM, false);
  ntt(pg, buf2, s + 1, b.T, logM, false);
  {
    Step st = vmk(ST_VPD_MUL, vtiles(2 * N));
    st.p[0] = buf1; st.p[1] = buf2; st.q[0] = 2 * N;
    st.bytes = 3 * kVE * 2 * N; st.mulmods = 2.0 * N;
    pg.steps.push_back(st);
  }
  ntt(pg, buf1, s + 1, b.T, logM, true);
  // h and g' on L
  scale(pg, b, 1, true, buf1, b.hL, M, N, 0);
  scale(pg, b, 2, true, buf1, b.gL, M, N, 0);
  ntt(pg, b.hL, logM, b.T, logM, false);
  ntt(pg, b.gL, logM, b.T, logM, false);
  tree(pg, b.hL, b.gL, b.treeHG, M / 2);
  auto absorb = [&](const uint32_t* root, uint32_t* pdst, Fr* out, uint32_t count) {
    Step st = vmk(ST_VPD_ABSORB, 1);
    st.p[0] = S; st.p[1] = root; st.p[2] = pdst; st.p[3] = out; st.u[0] = count;
    pg.steps.push_back(st);
  };
  absorb(b.treeHG + 8 * (M - 2), proof, b.V->a, 5);  // a0..a3, beta0
  const Fr g = vpd_shift(), inv2 = fr_inv2();
  {
    Step st = vmk(ST_VPD_FOLD0, vtiles(M / 2));
    st.p[0] = b.fL; st.p[1] = b.hL; st.p[2] = b.gL; st.p[3] = b.fri + fri_offset(M, 1); st.p[4] = b.V;
    st.p[5] = b.wlo; st.p[6] = b.whi; st.p[7] = b.wilo; st.p[8] = b.wihi;
    put_fr(st.w, g);
    put_fr(st.w + 8, fr_mul(fr_inverse(g), inv2));
    st.u[0] = logM - 1; st.q[0] = M / 2;
    st.bytes = kVE * (3 * M + M / 2); st.mulmods = 12.0 * (M / 2);
    pg.steps.push_back(st);
  }
  Fr gi = fr_mul(g, g);  // 5^(2^i)
  for (uint32_t i = 1; i < s; ++i) {
    const uint64_t m = M >> i;  // entries of layer i
    Fr* layer = b.fri + fri_offset(M, i);
    uint32_t* t = b.treeFri + 8 * fri_offset(M, i);
    tree(pg, layer, nullptr, t, m / 2);
    absorb(t + 8 * (m - 2), proof + 8 * i, &b.V->beta[i], 1);
    Step st = vmk(ST_VPD_FOLD, vtiles(m / 2));
    st.p[0] = layer; st.p[1] = b.fri + fri_offset(M, i + 1); st.p[2] = b.V; st.p[3] = b.wilo; st.p[4] = b.wihi;
    put_fr(st.w, fr_mul(fr_inverse(gi), inv2));
    st.u[0] = (uint32_t)(logM - i - 1); st.u[1] = i; st.q[0] = m / 2;
    st.bytes = kVE * (m + m / 2); st.mulmods = 3.0 * (m / 2);
    pg.steps.push_back(st);
    gi = fr_mul(gi, gi);
  }
  {
    Step st = vmk(ST_VPD_FINAL, 1);
    st.p[0] = b.fri + fri_offset(M, s); st.p[1] = S; st.p[2] = proof + 8 * s; st.p[3] = b.V;
    st.u[0] = vp.queries; st.q[0] = M / 2;
    pg.steps.push_back(st);
  }
  {
    const uint64_t total = (uint64_t)vp.queries * (s + 1);
    Step st = vmk(ST_VPD_QUERIES, vtiles(total));
    st.p[0] = b.V; st.p[1] = b.fL; st.p[2] = b.hL; st.p[3] = b.gL; st.p[4] = b.fri;
    st.p[5] = b.treeF; st.p[6] = b.treeHG; st.p[7] = b.treeFri; st.p[8] = proof + 8 * (s + 1);
    st.u[0] = s; st.u[1] = vp.queries; st.q[0] = M;
    st.bytes = (double)vpd_opening_bytes(s, vp.queries);
    pg.steps.push_back(st);
  }
}

}  // namespace gkr
