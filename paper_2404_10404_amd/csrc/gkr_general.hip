// General circuits with accumulation gates on gfx950: circuit objects, the
// workspace plan, the proof program and the kernels of the steps only general
// circuits use (the rounds, tails, eq tables and weighted sums are the
// layered circuit's steps).
//
// Section 2.7 (general arithmetic circuit): a gate of layer i may read any
// later layer j as long as one input is in layer i+1, and for a pair of layers
// only the gates of j that i reads are indexed. Section 3.4.3 (accumulation
// gate): a gate holds nested fan-in-2 gates and its value is their sum.
// A nested gate (z, x, j, y, type) adds V_{i+1}[x] op V_j[y] into gate z of
// layer i. Layer i's right inputs are gathered into R_i: the used gates of
// each source layer as consecutive blocks (block b = the b-th source layer in
// increasing order, 2^tau entries per block, zero padded), copies in the low
// bits. Each layer runs the two-phase sumcheck: phase 1 over x on (V_{i+1}, G,
// H), phase 2 over R_i's index on (R_i, F, K); then the prover sends the value
// of every source block at the local part of r_y, and those values become
// linear claims on the source layers, combined with squeezed coefficients at
// the start of each layer together with the eq claim vx of phase 1.
#include <string.h>

#include <algorithm>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "gkr_bodies.hpp"
#include "gkr_general.hpp"
#include "gkr_profile.hpp"
#include "gkr_program.hpp"
#include "gkr_tuning.hpp"

namespace gkr {

// ---------------------------------------------------------------- device bodies

#define GTID ((uint64_t)tile * kBlock + threadIdx.x)
#define GSTRIDE ((uint64_t)ntiles * kBlock)

// ST_G_GATHER: one block of R_i, R[(k << n) | c] = V[(U[k] << n) | c] for k < cnt
// and 0 for cnt <= k < rows. p0 V (source layer), p1 U, p2 R (block base), u0 n,
// q0 rows, q1 cnt.
__device__ __forceinline__ void body_g_gather(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ V = P<const Fr*>(st, 0);
  const uint32_t* __restrict__ U = P<const uint32_t*>(st, 1);
  Fr* __restrict__ R = P<Fr*>(st, 2);
  const uint32_t n = st.u[0];
  const uint64_t total = st.q[0] << n, cnt = st.q[1], mask = (1ull << n) - 1;
  for (uint64_t e = GTID; e < total; e += GSTRIDE) {
    const uint64_t k = e >> n;
    stf(R, e, k < cnt ? ldf(V, ((uint64_t)U[k] << n) | (e & mask)) : fr_zero());
  }
}

// ST_G_FORWARD: V[(z << n) | c] = sum over z's nested gates of
// W[(x << n) | c] (+ or *) R[(y' << n) | c]. p0 W = V_{i+1}, p1 R_i, p2 V_i,
// p3 zrow, p4 zent (x | type << 31, y'), u0 n, q0 count = 2^{s_i}.
__device__ __forceinline__ void body_g_forward(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ W = P<const Fr*>(st, 0);
  const Fr* __restrict__ R = P<const Fr*>(st, 1);
  Fr* __restrict__ V = P<Fr*>(st, 2);
  const uint32_t* __restrict__ zrow = P<const uint32_t*>(st, 3);
  const uint2* __restrict__ zent = P<const uint2*>(st, 4);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t g = GTID; g < st.q[0]; g += GSTRIDE) {
    const uint64_t z = g >> n, c = g & mask;
    Fr acc = fr_zero();
    const uint32_t k1 = zrow[z + 1];
    for (uint32_t k = zrow[z]; k < k1; ++k) {
      const uint2 e = zent[k];
      const Fr a = ldf(W, ((uint64_t)(e.x & 0x7fffffffu) << n) | c), b = ldf(R, ((uint64_t)e.y << n) | c);
      acc = fr_add(acc, (e.x >> 31) ? fr_mul(a, b) : fr_add(a, b));
    }
    stf(V, g, acc);
  }
}

// ST_G_SCATTER: the local weights of a subset claim, L[z] = E[pos[z]] where
// gate z is the pos[z]-th used gate, 0 for gates not used (pos = ~0).
// p0 E, p1 pos, p2 L, q0 count = 2^{sigma}.
__device__ __forceinline__ void body_g_scatter(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ E = P<const Fr*>(st, 0);
  const uint32_t* __restrict__ pos = P<const uint32_t*>(st, 1);
  Fr* __restrict__ L = P<Fr*>(st, 2);
  for (uint64_t z = GTID; z < st.q[0]; z += GSTRIDE) {
    const uint32_t k = pos[z];
    stf(L, z, k == 0xffffffffu ? fr_zero() : ldf(E, k));
  }
}

// ST_G_TTABLE: the layer's combined claim weights T[(z << n) | c] = sum_k
// L_k[z] C_k[c] (one reduction per entry), added to T when u2 = 1.
// p[2k] L_k, p[2k + 1] C_k (k < u1 <= 7), p14 T, u0 n, q0 count.
__device__ __forceinline__ void body_g_ttable(const Step& st, uint32_t tile, uint32_t ntiles) {
  Fr* __restrict__ T = P<Fr*>(st, 14);
  const uint32_t n = st.u[0], K = st.u[1];
  const bool accumulate = st.u[2] != 0;
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t g = GTID; g < st.q[0]; g += GSTRIDE) {
    const uint64_t z = g >> n, c = g & mask;
    FrWide acc = frw_zero();
    for (uint32_t k = 0; k < K; ++k) frw_mac(acc, ldf(P<const Fr*>(st, 2 * k), z), ldf(P<const Fr*>(st, 2 * k + 1), c));
    Fr t = frw_reduce<7>(acc);
    if (accumulate) t = fr_add(t, ldf(T, g));
    stf(T, g, t);
  }
}

// ST_G_P1: phase-1 tables over the left inputs x,
//   G[(x << n) | c] = sum_{MUL} T[(z << n) | c] R[(y' << n) | c] + sum_{ADD} T[(z << n) | c]
//   H[(x << n) | c] = sum_{ADD} T[(z << n) | c] R[(y' << n) | c]
// over the nested gates with left input x. p0 T, p1 R, p2 G, p3 H, p4 xrow,
// p5 xent (z, y' | type << 31), u0 n, q0 count = 2^{s_{i+1}}.
__device__ __forceinline__ void body_g_p1(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ T = P<const Fr*>(st, 0);
  const Fr* __restrict__ R = P<const Fr*>(st, 1);
  Fr* __restrict__ G = P<Fr*>(st, 2);
  Fr* __restrict__ H = P<Fr*>(st, 3);
  const uint32_t* __restrict__ xrow = P<const uint32_t*>(st, 4);
  const uint2* __restrict__ xent = P<const uint2*>(st, 5);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t e = GTID; e < st.q[0]; e += GSTRIDE) {
    const uint64_t x = e >> n, c = e & mask;
    Fr g = fr_zero(), h = fr_zero();
    const uint32_t k1 = xrow[x + 1];
    for (uint32_t k = xrow[x]; k < k1; ++k) {
      const uint2 r = xent[k];
      const Fr t = ldf(T, ((uint64_t)r.x << n) | c);
      const Fr tr = fr_mul(t, ldf(R, ((uint64_t)(r.y & 0x7fffffffu) << n) | c));
      if (r.y >> 31) {
        g = fr_add(g, tr);
      } else {
        g = fr_add(g, t);
        h = fr_add(h, tr);
      }
    }
    stf(G, e, g);
    stf(H, e, h);
  }
}

// ST_G_P2: phase-2 tables over R_i's index y', with E = eq(r_x, .) = EL x EC:
//   M[(y' << n) | c] = EC[c] sum_{MUL} T[(z << n) | c] EL[x],  A likewise over ADD,
//   F = vx M + A, K = vx A.
// p0 T, p1 EL, p2 EC, p3 vx (one element), p4 F, p5 K, p6 yrow, p7 yent
// (z, x | type << 31), u0 n, q0 count = 2^{rho_i}.
__device__ __forceinline__ void body_g_p2(const Step& st, uint32_t tile, uint32_t ntiles) {
  const Fr* __restrict__ T = P<const Fr*>(st, 0);
  const Fr* __restrict__ EL = P<const Fr*>(st, 1);
  const Fr* __restrict__ EC = P<const Fr*>(st, 2);
  const Fr vx = *P<const Fr*>(st, 3);
  Fr* __restrict__ F = P<Fr*>(st, 4);
  Fr* __restrict__ K = P<Fr*>(st, 5);
  const uint32_t* __restrict__ yrow = P<const uint32_t*>(st, 6);
  const uint2* __restrict__ yent = P<const uint2*>(st, 7);
  const uint32_t n = st.u[0];
  const uint64_t mask = (1ull << n) - 1;
  for (uint64_t e = GTID; e < st.q[0]; e += GSTRIDE) {
    const uint64_t y = e >> n, c = e & mask;
    Fr m = fr_zero(), a = fr_zero();
    const uint32_t k1 = yrow[y + 1];
    for (uint32_t k = yrow[y]; k < k1; ++k) {
      const uint2 r = yent[k];
      const Fr te = fr_mul(ldf(T, ((uint64_t)r.x << n) | c), ldf(EL, r.y & 0x7fffffffu));
      if (r.y >> 31) m = fr_add(m, te);
      else a = fr_add(a, te);
    }
    const Fr ec = ldf(EC, c);
    m = fr_mul(m, ec);
    a = fr_mul(a, ec);
    stf(F, e, fr_add(fr_mul(vx, m), a));
    stf(K, e, fr_mul(vx, a));
  }
}

// ST_G_LAYER_BEGIN: the layer's claim coefficients and combined claim. u0 = K
// claims, u1 = 1 on the output layer (single claim, coefficient 1); otherwise
// K coefficients are squeezed. p0 S, p1 coef (K elements out), p2.. p(2+K-1)
// the claimed values. S->claim = sum_k coef_k value_k; no round pending.
__device__ __forceinline__ void body_g_layer_begin(const Step& st, uint32_t, uint32_t) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  Fr* coef = P<Fr*>(st, 1);
  const uint32_t K = st.u[0];
  Sha256State sh = load_state(S);
  Fr claim = fr_zero();
  for (uint32_t k = 0; k < K; ++k) {
    const Fr a = st.u[1] ? fr_one() : squeeze(sh);
    stf(coef, k, a);
    claim = fr_add(claim, fr_mul(a, opaque(*P<const Fr*>(st, 2 + k))));
  }
  if (!st.u[1]) save_state(S, sh);
  S->claim = claim;
  S->pending = 0;
}

// ST_G_VALUES: the layer's block values (Montgomery, u0 of them at p1) go to
// the proof (canonical, p2) and into the transcript, one "GKRV" absorb each.
__device__ __forceinline__ void body_g_values(const Step& st, uint32_t, uint32_t) {
  if (threadIdx.x != 0) return;
  DevState* S = P<DevState*>(st, 0);
  const Fr* vals = P<const Fr*>(st, 1);
  uint32_t* proof = P<uint32_t*>(st, 2);
  Sha256State sh = load_state(S);
  for (uint32_t b = 0; b < st.u[0]; ++b) {
    const Fr c = fr_from_mont(ldf(vals, b));
    absorb_element(sh, kTagValue, c);
#pragma unroll
    for (int k = 0; k < 8; ++k) proof[8 * b + k] = c.v[k];
  }
  save_state(S, sh);
}

#undef GTID
#undef GSTRIDE

#define GKR_G_KERNEL(NAME, BODY)                                       \
  __global__ void __launch_bounds__(kBlock) NAME(Step st) { BODY(st, blockIdx.x, gridDim.x); }
GKR_G_KERNEL(k_g_gather, body_g_gather)
GKR_G_KERNEL(k_g_forward, body_g_forward)
GKR_G_KERNEL(k_g_scatter, body_g_scatter)
GKR_G_KERNEL(k_g_ttable, body_g_ttable)
GKR_G_KERNEL(k_g_p1, body_g_p1)
GKR_G_KERNEL(k_g_p2, body_g_p2)
GKR_G_KERNEL(k_g_layer_begin, body_g_layer_begin)
GKR_G_KERNEL(k_g_values, body_g_values)
#undef GKR_G_KERNEL

void launch_general_step(const Step& st, hipStream_t s) {
  const int tok = prof_begin(s);
  const dim3 grid(st.ntiles), block(kBlock);
  ProfClass cls = PC_SMALL;
  switch (st.type) {
    case ST_G_GATHER: k_g_gather<<<grid, block, 0, s>>>(st); cls = PC_G_GATHER; break;
    case ST_G_FORWARD: k_g_forward<<<grid, block, 0, s>>>(st); cls = PC_G_FORWARD; break;
    case ST_G_SCATTER: k_g_scatter<<<grid, block, 0, s>>>(st); cls = PC_G_CLAIMS; break;
    case ST_G_TTABLE: k_g_ttable<<<grid, block, 0, s>>>(st); cls = PC_G_CLAIMS; break;
    case ST_G_P1: k_g_p1<<<grid, block, 0, s>>>(st); cls = PC_G_PHASE1_INIT; break;
    case ST_G_P2: k_g_p2<<<grid, block, 0, s>>>(st); cls = PC_G_PHASE2_TABLES; break;
    case ST_G_LAYER_BEGIN: k_g_layer_begin<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    case ST_G_VALUES: k_g_values<<<grid, block, 0, s>>>(st); cls = PC_TRANSCRIPT; break;
    default: break;
  }
  if (tok >= 0) prof_end(tok, s, cls, st.bytes, st.mulmods);
}

// ---------------------------------------------------------------- step builders

namespace {

constexpr uint32_t kGSweepTiles = 65535u * 8;
constexpr double kE = 32.0;

uint32_t g_tiles(uint64_t n) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > kGSweepTiles) g = kGSweepTiles;
  return (uint32_t)g;
}

Step g_mk(uint32_t type, uint32_t ntiles) {
  Step st;
  memset(&st, 0, sizeof(st));
  st.type = type;
  st.ntiles = ntiles < 1 ? 1 : ntiles;
  return st;
}

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// ---------------------------------------------------------------- workspace plan

// Layered-plan fields the shared emission uses (layers, G/H/Wf, the output
// claim's eq tables, partials, digests, challenges, state), then the general
// buffers.
static void plan_general(gkr_circuit& c) {
  GeneralInfo& g = *c.general;
  const uint32_t d = c.depth, n = c.n;
  uint32_t gh = 0, smax = 0, sigmax = 0, taumax = 0, kmax = 1;
  size_t chal = c.s(0);
  for (uint32_t i = 0; i < d; ++i) {
    gh = std::max(gh, std::max(c.s(i + 1), g.rho(i)));
    taumax = std::max(taumax, g.layers[i].tau);
    kmax = std::max<uint32_t>(kmax, (uint32_t)g.claims[i].size());
    chal += c.s(i + 1) + g.rho(i);
  }
  for (uint32_t i = 0; i <= d; ++i) {
    smax = std::max(smax, c.s(i));
    sigmax = std::max(sigmax, c.sigma[i]);
  }
  const size_t E = sizeof(Fr);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  Plan& p = c.plan;
  memset(&p, 0, sizeof(p));
  for (uint32_t i = 0; i <= d; ++i) p.off_layer[i] = take(E << c.s(i));
  p.off_G = take(E << gh);
  p.off_H = take(E << gh);
  p.off_Wf = take(E << (gh ? gh - 1 : 0));
  p.off_aU = take(E << c.sigma[0]);
  p.off_Cu = take(E << n);
  p.off_partials = take(E * (size_t)kMaxRoundBlocks * kMaxPartialValues);
  const uint64_t big = 1ull << std::max(c.s(0), c.s(d));
  const uint64_t chunks0 = (big * 8 + kChunkWords - 1) / kChunkWords;
  p.dig_level_words = chunks0 * 8;
  p.off_dig_a = take(4 * p.dig_level_words);
  p.off_dig_b = take(4 * p.dig_level_words);
  p.off_dig_in = take(32);
  p.off_dig_out = take(32);
  p.off_chal = take(E * (chal + 8));
  p.off_state = take(sizeof(DevState));
  // general buffers
  g.off_R.resize(d);
  for (uint32_t i = 0; i < d; ++i) g.off_R[i] = take(E << g.rho(i));
  g.off_T = take(E << smax);
  g.off_L = take(E * ((size_t)kmax << sigmax));
  g.off_C = take(E * ((size_t)kmax << n));
  g.off_EqL = take(E << std::max(taumax, sigmax));
  g.off_EqC = take(E << n);
  g.off_EL = take(E << sigmax);
  g.off_EC = take(E << n);
  size_t ncoef = 0, nvals = 0;
  g.coef_index.resize(d);
  g.val_index.resize(d);
  g.rx_index.resize(d);
  g.ry_index.resize(d);
  size_t ci = c.s(0);
  for (uint32_t i = 0; i < d; ++i) {
    g.coef_index[i] = ncoef;
    ncoef += g.claims[i].size();
    g.val_index[i] = nvals;
    nvals += 1 + g.layers[i].sources.size();
    g.rx_index[i] = ci;
    ci += c.s(i + 1);
    g.ry_index[i] = ci;
    ci += g.rho(i);
  }
  g.off_coef = take(E * (ncoef + 1));
  g.off_vals = take(E * (nvals + 1));
  g.kmax = kmax;
  p.total = off;
}

// ---------------------------------------------------------------- proof program

struct GWs {
  Workspace w;
  Fr *T, *L, *C, *EqL, *EqC, *EL, *EC, *coef, *vals;
  std::vector<Fr*> R;
};

static GWs bind_general(const gkr_circuit& c, void* base) {
  GWs gw;
  gw.w = bind_workspace(c, base);
  const GeneralInfo& g = *c.general;
  char* b = static_cast<char*>(base);
  auto F = [&](size_t o) { return reinterpret_cast<Fr*>(b + o); };
  gw.T = F(g.off_T);
  gw.L = F(g.off_L);
  gw.C = F(g.off_C);
  gw.EqL = F(g.off_EqL);
  gw.EqC = F(g.off_EqC);
  gw.EL = F(g.off_EL);
  gw.EC = F(g.off_EC);
  gw.coef = F(g.off_coef);
  gw.vals = F(g.off_vals);
  for (size_t o : g.off_R) gw.R.push_back(F(o));
  return gw;
}

static void g_eq(Program& pg, int count, const uint32_t* bits, const Fr* const* pts, const Fr* const* scl,
                 Fr* const* outs) {
  pg.eq(count, bits, pts, scl, outs);
}

// Forward evaluation: V_i from V_{i+1} and R_i (gathered from the source layers).
static void emit_general_forward(Program& pg, const gkr_circuit& c, const GWs& gw) {
  const GeneralInfo& g = *c.general;
  const uint32_t n = c.n;
  for (int i = (int)c.depth - 1; i >= 0; --i) {
    const GeneralLayer& L = g.layers[i];
    const uint64_t rows = 1ull << L.tau;
    const uint64_t nblocks = 1ull << L.beta;
    for (uint64_t b = 0; b < nblocks; ++b) {
      const bool real = b < L.sources.size();
      Step st = g_mk(ST_G_GATHER, g_tiles(rows << n));
      st.p[0] = real ? gw.w.layer[L.sources[b]] : gw.w.layer[i + 1];
      st.p[1] = real ? L.used_dev[b] : nullptr;
      st.p[2] = gw.R[i] + (b * rows << n);
      st.u[0] = n;
      st.q[0] = rows;
      st.q[1] = real ? L.used[b].size() : 0;
      st.bytes = kE * ((double)(st.q[1] << n) + (double)(rows << n));
      pg.steps.push_back(st);
    }
    Step st = g_mk(ST_G_FORWARD, g_tiles(1ull << c.s(i)));
    st.p[0] = gw.w.layer[i + 1];
    st.p[1] = gw.R[i];
    st.p[2] = gw.w.layer[i];
    st.p[3] = L.zrow;
    st.p[4] = L.zent;
    st.u[0] = n;
    st.q[0] = 1ull << c.s(i);
    st.bytes = kE * ((2.0 * L.recs.size() * (1ull << n)) + (double)(1ull << c.s(i)));
    st.mulmods = (double)(L.mul_recs << n);
    pg.steps.push_back(st);
  }
}

// One general gate layer.
static void emit_general_layer(Program& pg, const gkr_circuit& c, uint32_t i, const GWs& gw, uint32_t* proof,
                               const Tuning& tun) {
  const GeneralInfo& g = *c.general;
  const GeneralLayer& L = g.layers[i];
  const uint32_t n = c.n, sg = c.sigma[i], s1 = c.s(i + 1), rho = g.rho(i);
  DevState* S = gw.w.state;
  const std::vector<ClaimRef>& claims = g.claims[i];
  const uint32_t K = (uint32_t)claims.size();
  Fr* coef = gw.coef + g.coef_index[i];
  Fr* chal = gw.w.chal;
  // claim values and points
  auto value_of = [&](const ClaimRef& cr) -> const Fr* {
    if (cr.h < 0) return &S->scratch[0];
    return gw.vals + g.val_index[cr.h] + (cr.b < 0 ? 0 : 1 + cr.b);
  };
  {
    Step st = g_mk(ST_G_LAYER_BEGIN, 1);
    st.p[0] = S;
    st.p[1] = coef;
    for (uint32_t k = 0; k < K; ++k) st.p[2 + k] = value_of(claims[k]);
    st.u[0] = K;
    st.u[1] = i == 0 ? 1 : 0;
    st.mulmods = K;
    pg.steps.push_back(st);
  }
  // claim weight tables L_k (local, scaled by the coefficient) and C_k (copies)
  for (uint32_t k = 0; k < K; ++k) {
    const ClaimRef& cr = claims[k];
    Fr* Lk = gw.L + ((size_t)k << sg);
    Fr* Ck = gw.C + ((size_t)k << n);
    if (cr.b < 0) {
      const Fr* pt = cr.h < 0 ? chal : chal + g.rx_index[cr.h];
      const uint32_t bits[2] = {sg, n};
      const Fr* pts[2] = {pt, pt + sg};
      const Fr* scl[2] = {coef + k, nullptr};
      Fr* outs[2] = {Lk, Ck};
      g_eq(pg, 2, bits, pts, scl, outs);
    } else {
      const GeneralLayer& H = g.layers[cr.h];
      const Fr* pt = chal + g.ry_index[cr.h] + H.beta;  // local (tau_h bits), then copy bits
      const uint32_t bits[2] = {H.tau, n};
      const Fr* pts[2] = {pt, pt + H.tau};
      const Fr* scl[2] = {coef + k, nullptr};
      Fr* outs[2] = {gw.EqL, Ck};
      g_eq(pg, 2, bits, pts, scl, outs);
      Step st = g_mk(ST_G_SCATTER, g_tiles(1ull << sg));
      st.p[0] = gw.EqL;
      st.p[1] = H.pos_dev[cr.b];
      st.p[2] = Lk;
      st.q[0] = 1ull << sg;
      st.bytes = kE * (double)(1ull << sg);
      pg.steps.push_back(st);
    }
  }
  for (uint32_t k0 = 0; k0 < K; k0 += 7) {
    const uint32_t kk = std::min<uint32_t>(7, K - k0);
    Step st = g_mk(ST_G_TTABLE, g_tiles(1ull << c.s(i)));
    for (uint32_t k = 0; k < kk; ++k) {
      st.p[2 * k] = gw.L + ((size_t)(k0 + k) << sg);
      st.p[2 * k + 1] = gw.C + ((size_t)(k0 + k) << n);
    }
    st.p[14] = gw.T;
    st.u[0] = n;
    st.u[1] = kk;
    st.u[2] = k0 > 0 ? 1 : 0;
    st.q[0] = 1ull << c.s(i);
    st.bytes = kE * (double)(1ull << c.s(i)) * (k0 > 0 ? 2.0 : 1.0);
    st.mulmods = (double)kk * (1ull << c.s(i)) * 0.5;
    pg.steps.push_back(st);
  }
  // phase 1 over x
  Fr* rx = chal + g.rx_index[i];
  Fr* ry = chal + g.ry_index[i];
  Fr* vals = gw.vals + g.val_index[i];
  const uint32_t off_vx = 24 * s1, off_p2 = off_vx + 8, off_vy = off_p2 + 24 * rho, off_blocks = off_vy + 8;
  {
    Step st = g_mk(ST_G_P1, g_tiles(1ull << s1));
    st.p[0] = gw.T;
    st.p[1] = gw.R[i];
    st.p[2] = gw.w.G;
    st.p[3] = gw.w.H;
    st.p[4] = L.xrow;
    st.p[5] = L.xent;
    st.u[0] = n;
    st.q[0] = 1ull << s1;
    st.bytes = kE * (2.0 * (L.recs.size() << n) + 2.0 * (1ull << s1));
    st.mulmods = (double)(L.recs.size() << n);
    pg.steps.push_back(st);
  }
  {
    const Fr* src[3] = {gw.w.layer[i + 1], gw.w.G, gw.w.H};
    Fr* dst[3] = {gw.w.Wf, gw.w.G, gw.w.H};
    emit_phase_a(pg, src, dst, s1, S, gw.w.partials, rx, proof, vals, proof + off_vx, tun);
  }
  // phase 2 over R_i's index
  {
    const uint32_t bits[2] = {c.sigma[i + 1], n};
    const Fr* pts[2] = {rx, rx + c.sigma[i + 1]};
    const Fr* scl[2] = {nullptr, nullptr};
    Fr* outs[2] = {gw.EL, gw.EC};
    g_eq(pg, 2, bits, pts, scl, outs);
  }
  {
    Step st = g_mk(ST_G_P2, g_tiles(1ull << rho));
    st.p[0] = gw.T;
    st.p[1] = gw.EL;
    st.p[2] = gw.EC;
    st.p[3] = vals;  // vx
    st.p[4] = gw.w.G;  // F
    st.p[5] = gw.w.H;  // K
    st.p[6] = L.yrow;
    st.p[7] = L.yent;
    st.u[0] = n;
    st.q[0] = 1ull << rho;
    st.bytes = kE * ((double)(L.recs.size() << n) + 2.0 * (1ull << rho));
    st.mulmods = (double)(L.recs.size() << n) + 4.0 * (1ull << rho);
    pg.steps.push_back(st);
  }
  {
    const Fr* src[3] = {gw.R[i], gw.w.G, gw.w.H};
    Fr* dst[3] = {gw.w.Wf, gw.w.G, gw.w.H};
    emit_phase_a(pg, src, dst, rho, S, gw.w.partials, ry, proof + off_p2, &S->scratch[1], proof + off_vy, tun);
  }
  // the source blocks' values at the local part of r_y
  {
    const uint32_t bits[2] = {L.tau, n};
    const Fr* pts[2] = {ry + L.beta, ry + L.beta + L.tau};
    const Fr* scl[2] = {nullptr, nullptr};
    Fr* outs[2] = {gw.EqL, gw.EqC};
    g_eq(pg, 2, bits, pts, scl, outs);
  }
  const uint64_t bsize = 1ull << (L.tau + n);
  for (size_t b = 0; b < L.sources.size(); ++b)
    pg.wsum(gw.R[i] + b * bsize, gw.EqL, gw.EqC, n, bsize, gw.w.partials, S, vals + 1 + b, tun);
  {
    Step st = g_mk(ST_G_VALUES, 1);
    st.p[0] = S;
    st.p[1] = vals + 1;
    st.p[2] = proof + off_blocks;
    st.u[0] = (uint32_t)L.sources.size();
    pg.steps.push_back(st);
  }
}

void emit_prove_general(Program& pg, const gkr_circuit& c, void* d_ws, const gkr_fr* d_inputs, uint64_t seed,
                        gkr_fr* d_outputs, uint8_t* d_proof, const Tuning& tun) {
  const GWs gw = bind_general(c, d_ws);
  pg.to_mont(d_inputs, gw.w.layer[c.depth], 1ull << c.s(c.depth));
  emit_general_forward(pg, c, gw);
  pg.from_mont(gw.w.layer[0], d_outputs, 1ull << c.s(0));
  emit_statement_and_output_claim(pg, c, gw.w, d_inputs, d_outputs, seed, tun);
  uint32_t* proof = reinterpret_cast<uint32_t*>(d_proof);
  for (uint32_t i = 0; i < c.depth; ++i) {
    emit_general_layer(pg, c, i, gw, proof, tun);
    proof += general_layer_proof_bytes(c, i) / 4;
  }
}

// ---------------------------------------------------------------- circuit objects

size_t general_layer_proof_bytes(const gkr_circuit& c, uint32_t i) {
  const GeneralInfo& g = *c.general;
  return (3ull * c.s(i + 1) + 3ull * g.rho(i) + 2 + g.layers[i].sources.size()) * 32;
}

size_t general_proof_bytes(const gkr_circuit& c) {
  size_t t = 0;
  for (uint32_t i = 0; i < c.depth; ++i) t += general_layer_proof_bytes(c, i);
  return t;
}

void general_destroy(GeneralInfo* g) { delete g; }

static uint32_t bits_for(size_t count) {
  uint32_t b = 0;
  while ((1ull << b) < count) ++b;
  return b;
}

}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_general_circuit_create(uint32_t depth, uint32_t log_copies, const uint32_t* log_sub_width,
                                              const uint64_t* counts, const gkr_nested_gate* const* gates,
                                              gkr_circuit** out) {
  try {
    if (!out || !log_sub_width || !counts || !gates) {
      set_error("null argument");
      return GKR_EINVAL;
    }
    *out = nullptr;
    if (depth < 1 || depth > GKR_MAX_DEPTH) {
      set_error("depth must be in [1, " + std::to_string(GKR_MAX_DEPTH) + "]");
      return GKR_EINVAL;
    }
    if (log_copies > GKR_MAX_LOG_COPIES) {
      set_error("log_copies too large");
      return GKR_EUNSUPPORTED;
    }
    for (uint32_t i = 0; i <= depth; ++i) {
      if (log_sub_width[i] + log_copies > GKR_MAX_LOG_WIDTH) {
        set_error("layer " + std::to_string(i) + " is wider than 2^" + std::to_string(GKR_MAX_LOG_WIDTH));
        return GKR_EUNSUPPORTED;
      }
    }
    std::unique_ptr<gkr_circuit> c(new gkr_circuit());
    c->depth = depth;
    c->n = log_copies;
    c->sigma.assign(log_sub_width, log_sub_width + depth + 1);
    c->general = new GeneralInfo();
    GeneralInfo& g = *c->general;
    g.n = log_copies;
    g.layers.resize(depth);
    for (uint32_t i = 0; i < depth; ++i) {
      GeneralLayer& L = g.layers[i];
      if (!gates[i] || counts[i] == 0) {
        set_error("gate layer " + std::to_string(i) + " has no nested gates");
        return GKR_EINVAL;
      }
      if (counts[i] > (1ull << 31)) {
        set_error("gate layer " + std::to_string(i) + " has too many nested gates");
        return GKR_EUNSUPPORTED;
      }
      L.recs.assign(gates[i], gates[i] + counts[i]);
      std::vector<std::vector<uint32_t>> used_by_src(depth + 1);
      for (size_t k = 0; k < L.recs.size(); ++k) {
        const gkr_nested_gate& r = L.recs[k];
        if (r.z >= (1ull << c->sigma[i]) || r.x >= (1ull << c->sigma[i + 1]) || r.src <= i || r.src > depth ||
            r.y >= (1ull << c->sigma[r.src]) || r.type > 1) {
          set_error("gate layer " + std::to_string(i) + " nested gate " + std::to_string(k) + " is invalid");
          return GKR_EINVAL;
        }
        used_by_src[r.src].push_back(r.y);
        L.mul_recs += r.type == GKR_GATE_MUL;
      }
      for (uint32_t j = i + 1; j <= depth; ++j) {
        if (used_by_src[j].empty()) continue;
        std::vector<uint32_t>& u = used_by_src[j];
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        L.sources.push_back(j);
        L.used.push_back(u);
      }
      L.beta = bits_for(L.sources.size());
      L.tau = 0;
      for (const auto& u : L.used) L.tau = std::max(L.tau, bits_for(u.size()));
      if (g.rho(i) > GKR_MAX_LOG_WIDTH) {
        set_error("gate layer " + std::to_string(i) + ": right-input index wider than 2^" +
                  std::to_string(GKR_MAX_LOG_WIDTH));
        return GKR_EUNSUPPORTED;
      }
    }
    // claims per gate layer, in production order: by producing layer, the eq
    // claim of phase 1 before that layer's block claims
    g.claims.assign(depth + 1, {});
    g.claims[0].push_back({-1, -1});
    for (uint32_t h = 0; h < depth; ++h) {
      g.claims[h + 1].push_back({(int)h, -1});
      for (size_t b = 0; b < g.layers[h].sources.size(); ++b) g.claims[g.layers[h].sources[b]].push_back({(int)h, (int)b});
    }
    for (uint32_t i = 0; i < depth; ++i) {
      if (g.claims[i].size() > kGeneralMaxClaims) {
        set_error("gate layer " + std::to_string(i) + " receives " + std::to_string(g.claims[i].size()) +
                  " claims; at most " + std::to_string(kGeneralMaxClaims) + " are supported");
        return GKR_EUNSUPPORTED;
      }
    }
    // circuit digest: SHA256("GKR-GENERAL-v1" || LE32 d, n, sigma_0..d || per layer
    // LE32 count || per nested gate LE32 z, x, src, y || u8 type)
    {
      std::vector<uint8_t> msg(14);
      memcpy(msg.data(), "GKR-GENERAL-v1", 14);
      auto put32 = [&](uint32_t v) {
        for (int k = 0; k < 4; ++k) msg.push_back((uint8_t)(v >> (8 * k)));
      };
      put32(depth);
      put32(log_copies);
      for (uint32_t i = 0; i <= depth; ++i) put32(c->sigma[i]);
      for (uint32_t i = 0; i < depth; ++i) {
        put32((uint32_t)g.layers[i].recs.size());
        for (const gkr_nested_gate& r : g.layers[i].recs) {
          put32(r.z);
          put32(r.x);
          put32(r.src);
          put32(r.y);
          msg.push_back(r.type);
        }
      }
      sha256_bytes(msg.data(), msg.size(), c->digest);
    }
    // host indexes: right index of each nested gate, CSRs by z, x and y', used
    // lists and the inverse maps of the used sets
    struct Blk {
      size_t off;
      size_t bytes;
    };
    size_t total = 0;
    auto take = [&](size_t bytes) {
      size_t o = total;
      total = (total + bytes + 255) & ~(size_t)255;
      return Blk{o, bytes};
    };
    struct LayerOffs {
      Blk zrow, zent, xrow, xent, yrow, yent;
      std::vector<Blk> used, pos;
    };
    std::vector<LayerOffs> lo(depth);
    for (uint32_t i = 0; i < depth; ++i) {
      const GeneralLayer& L = g.layers[i];
      const size_t cnt = L.recs.size();
      lo[i].zrow = take(4 * ((1ull << c->sigma[i]) + 1));
      lo[i].zent = take(8 * cnt);
      lo[i].xrow = take(4 * ((1ull << c->sigma[i + 1]) + 1));
      lo[i].xent = take(8 * cnt);
      lo[i].yrow = take(4 * ((1ull << (L.beta + L.tau)) + 1));
      lo[i].yent = take(8 * cnt);
      for (size_t b = 0; b < L.sources.size(); ++b) {
        lo[i].used.push_back(take(4 * L.used[b].size()));
        lo[i].pos.push_back(take(4 * (1ull << c->sigma[L.sources[b]])));
      }
    }
    std::vector<uint8_t> host(total, 0);
    auto W32 = [&](const Blk& b) { return reinterpret_cast<uint32_t*>(host.data() + b.off); };
    for (uint32_t i = 0; i < depth; ++i) {
      const GeneralLayer& L = g.layers[i];
      const size_t cnt = L.recs.size();
      std::vector<uint32_t> yl(cnt);
      std::vector<std::vector<uint32_t>> posmap(L.sources.size());
      for (size_t b = 0; b < L.sources.size(); ++b) {
        posmap[b].assign(1ull << c->sigma[L.sources[b]], 0xffffffffu);
        for (size_t k = 0; k < L.used[b].size(); ++k) posmap[b][L.used[b][k]] = (uint32_t)k;
        memcpy(W32(lo[i].used[b]), L.used[b].data(), 4 * L.used[b].size());
        memcpy(W32(lo[i].pos[b]), posmap[b].data(), 4 * posmap[b].size());
      }
      for (size_t k = 0; k < cnt; ++k) {
        const gkr_nested_gate& r = L.recs[k];
        const size_t b = std::find(L.sources.begin(), L.sources.end(), r.src) - L.sources.begin();
        yl[k] = ((uint32_t)b << L.tau) | posmap[b][r.y];
      }
      auto csr = [&](const Blk& row, const Blk& ent, size_t rows, auto key, auto val) {
        uint32_t* rp = W32(row);
        uint32_t* ep = W32(ent);
        for (size_t k = 0; k < cnt; ++k) rp[key(k) + 1]++;
        for (size_t r = 0; r < rows; ++r) rp[r + 1] += rp[r];
        std::vector<uint32_t> fill(rp, rp + rows);
        for (size_t k = 0; k < cnt; ++k) {
          const uint32_t at = fill[key(k)]++;
          const uint2 v = val(k);
          ep[2 * at] = v.x;
          ep[2 * at + 1] = v.y;
        }
      };
      const auto tbit = [&](size_t k) { return (uint32_t)L.recs[k].type << 31; };
      csr(lo[i].zrow, lo[i].zent, 1ull << c->sigma[i], [&](size_t k) { return L.recs[k].z; },
          [&](size_t k) { return make_uint2(L.recs[k].x | tbit(k), yl[k]); });
      csr(lo[i].xrow, lo[i].xent, 1ull << c->sigma[i + 1], [&](size_t k) { return L.recs[k].x; },
          [&](size_t k) { return make_uint2(L.recs[k].z, yl[k] | tbit(k)); });
      csr(lo[i].yrow, lo[i].yent, 1ull << (L.beta + L.tau), [&](size_t k) { return yl[k]; },
          [&](size_t k) { return make_uint2(L.recs[k].z, L.recs[k].x | tbit(k)); });
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
      (void)hipGetLastError();
      c->device = -1;
      plan_general(*c);
      *out = c.release();
      return GKR_OK;
    }
    hipGetDevice(&c->device);
    if (hipMalloc(&c->dev_block, std::max<size_t>(total, 256)) != hipSuccess) {
      (void)hipGetLastError();
      c->dev_block = nullptr;
      set_error("device allocation of the wiring failed");
      return GKR_ENOMEM;
    }
    if (hipMemcpy(c->dev_block, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      set_error("upload of the wiring failed");
      return GKR_EDEVICE;
    }
    char* base = static_cast<char*>(c->dev_block);
    for (uint32_t i = 0; i < depth; ++i) {
      GeneralLayer& L = g.layers[i];
      L.zrow = reinterpret_cast<const uint32_t*>(base + lo[i].zrow.off);
      L.zent = reinterpret_cast<const uint2*>(base + lo[i].zent.off);
      L.xrow = reinterpret_cast<const uint32_t*>(base + lo[i].xrow.off);
      L.xent = reinterpret_cast<const uint2*>(base + lo[i].xent.off);
      L.yrow = reinterpret_cast<const uint32_t*>(base + lo[i].yrow.off);
      L.yent = reinterpret_cast<const uint2*>(base + lo[i].yent.off);
      for (size_t b = 0; b < L.sources.size(); ++b) {
        L.used_dev.push_back(reinterpret_cast<const uint32_t*>(base + lo[i].used[b].off));
        L.pos_dev.push_back(reinterpret_cast<const uint32_t*>(base + lo[i].pos[b].off));
      }
    }
    plan_general(*c);
    *out = c.release();
    return GKR_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  } catch (...) {
    set_error("unexpected failure");
    return GKR_EINVAL;
  }
}
