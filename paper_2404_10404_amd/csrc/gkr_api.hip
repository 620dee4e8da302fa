// Host driver and C ABI of the GKR prover: circuit objects, workspace layout,
// and the launch sequence of a proof (all on the caller's stream, no host
// synchronisation, no allocation while proving).
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gkr_general.hpp"
#include "gkr_gl.hpp"
#include "gkr_kernels.hpp"
#include "gkr_program.hpp"
#include "gkr_contract.hpp"
#include "gkr_tuning.hpp"
#include "gkr_vpd.hpp"

namespace gkr {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

// ------------------------------------------------------------------ SHA-256 (host)

void sha256_bytes(const uint8_t* data, size_t len, uint32_t out[8]) {
  Sha256State st = sha256_iv();
  uint32_t blk[16];
  size_t off = 0;
  while (len - off >= 64) {
    for (int i = 0; i < 16; ++i) {
      const uint8_t* b = data + off + 4 * i;
      blk[i] = ((uint32_t)b[0] << 24) | ((uint32_t)b[1] << 16) | ((uint32_t)b[2] << 8) | b[3];
    }
    sha256_compress(st, blk);
    off += 64;
  }
  uint8_t tail[128];
  memset(tail, 0, sizeof(tail));
  const size_t rem = len - off;
  memcpy(tail, data + off, rem);
  tail[rem] = 0x80;
  const size_t tl = (rem + 9 <= 64) ? 64 : 128;
  const uint64_t bits = (uint64_t)len * 8;
  for (int k = 0; k < 8; ++k) tail[tl - 1 - k] = (uint8_t)(bits >> (8 * k));
  for (size_t o = 0; o < tl; o += 64) {
    for (int i = 0; i < 16; ++i) {
      const uint8_t* b = tail + o + 4 * i;
      blk[i] = ((uint32_t)b[0] << 24) | ((uint32_t)b[1] << 16) | ((uint32_t)b[2] << 8) | b[3];
    }
    sha256_compress(st, blk);
  }
  for (int k = 0; k < 8; ++k) out[k] = st.h[k];
}

static Words8 seed_state(uint64_t seed) {
  uint8_t msg[19];
  memcpy(msg, "SISU-GKR-v1", 11);
  for (int k = 0; k < 8; ++k) msg[11 + k] = (uint8_t)(seed >> (8 * k));
  Words8 w;
  sha256_bytes(msg, sizeof(msg), w.w);
  return w;
}

// ------------------------------------------------------------------ workspace plan

static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t plan_workspace(const gkr_circuit& c, Plan& p) {
  const uint32_t d = c.depth, n = c.n;
  uint32_t sp_max = 0, sigp_max = 0, sig_max = 0, s_max = 0;
  for (uint32_t i = 0; i < d; ++i) {
    sp_max = std::max(sp_max, c.s(i + 1));
    sigp_max = std::max(sigp_max, c.sigma[i + 1]);
    sig_max = std::max(sig_max, c.sigma[i]);
  }
  for (uint32_t i = 0; i <= d; ++i) s_max = std::max(s_max, c.s(i));
  const size_t E = sizeof(Fr);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = align_up(off + bytes);
    return o;
  };
  for (uint32_t i = 0; i <= d; ++i) p.off_layer[i] = take(E << c.s(i));
  p.off_G = take(E << sp_max);
  p.off_H = take(E << sp_max);
  p.off_Wf = take(E << (sp_max ? sp_max - 1 : 0));
  p.off_aU = take(E << sig_max);
  p.off_bV = take(E << sig_max);
  p.off_Cu = take(E << n);
  p.off_Cv = take(E << n);
  p.off_U = take(E << n);
  p.off_V = take(E << n);
  p.off_EC = take(E << n);
  p.off_EL = take(E << sigp_max);
  p.off_EqR = take(E << sigp_max);
  p.off_P = take(E << sigp_max);
  p.off_Q = take(E << sigp_max);
  p.off_Fa = take(E << sigp_max);
  p.off_Fb = take(E << sigp_max);
  p.off_Ks = take(E << sigp_max);
  p.off_Ka = take(E << sigp_max);
  p.off_Kb = take(E << sigp_max);
  p.off_Wc = take(E << n);
  p.off_Fc = take(E << n);
  p.off_Kc = take(E << n);
  // row split of the copy-table pass: about 2^18 threads in total (a power of
  // two), so each thread contracts several rows before its partial is stored
  uint64_t want = (n >= 18) ? 1 : (1ull << (18 - n));
  uint64_t rows = 1ull << sigp_max;
  p.ychunks = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, std::min<uint64_t>(rows, 1ull << 15)));
  p.off_wpart = take(E * ((size_t)p.ychunks << n));
  p.off_partials = take(E * (size_t)kMaxRoundBlocks * kMaxPartialValues);
  const uint64_t big = 1ull << std::max(c.s(0), c.s(d));
  const uint64_t chunks0 = (big * 8 + kChunkWords - 1) / kChunkWords;
  p.dig_level_words = chunks0 * 8;
  p.off_dig_a = take(4 * p.dig_level_words);
  p.off_dig_b = take(4 * p.dig_level_words);
  p.off_dig_in = take(32);
  p.off_dig_out = take(32);
  p.off_chal = take(E * ((size_t)c.s(0) + 2ull * d * sp_max + 2ull * s_max + 8));
  p.off_state = take(sizeof(DevState));
  p.cc_bytes = 0;
  for (uint32_t i = 0; i < d; ++i) p.cc_bytes = std::max(p.cc_bytes, cc_scratch_bytes(n, c.sigma[i + 1]));
  p.off_cc = take(p.cc_bytes);
  p.total = off;
  return off;
}

static uint32_t sp_max_of(const gkr_circuit& c) {
  uint32_t m = 0;
  for (uint32_t i = 0; i < c.depth; ++i) m = std::max(m, c.s(i + 1));
  return m;
}
static uint32_t s_max_of(const gkr_circuit& c) {
  uint32_t m = 0;
  for (uint32_t i = 0; i <= c.depth; ++i) m = std::max(m, c.s(i));
  return m;
}

uint32_t host_chal_index_rx(const gkr_circuit& c, uint32_t layer) {
  return c.s(0) + 2 * layer * sp_max_of(c);
}
uint32_t host_chal_index_ry(const gkr_circuit& c, uint32_t layer) {
  return c.s(0) + 2 * layer * sp_max_of(c) + sp_max_of(c);
}
// Scratch points (u, v) and claims of gkr_prove_layer live after the challenges.
static uint32_t chal_index_scratch(const gkr_circuit& c) { return c.s(0) + 2 * c.depth * sp_max_of(c); }

Workspace bind_workspace(const gkr_circuit& c, void* base) {
  Workspace w;
  memset(&w, 0, sizeof(w));
  char* b = static_cast<char*>(base);
  const Plan& p = c.plan;
  for (uint32_t i = 0; i <= c.depth; ++i) w.layer[i] = reinterpret_cast<Fr*>(b + p.off_layer[i]);
  auto F = [&](size_t o) { return reinterpret_cast<Fr*>(b + o); };
  w.G = F(p.off_G); w.H = F(p.off_H); w.Wf = F(p.off_Wf);
  w.aU = F(p.off_aU); w.bV = F(p.off_bV); w.Cu = F(p.off_Cu); w.Cv = F(p.off_Cv);
  w.U = F(p.off_U); w.V = F(p.off_V); w.EC = F(p.off_EC); w.EL = F(p.off_EL); w.EqR = F(p.off_EqR);
  w.P = F(p.off_P); w.Q = F(p.off_Q); w.Fa = F(p.off_Fa); w.Fb = F(p.off_Fb); w.Ks = F(p.off_Ks);
  w.Ka = F(p.off_Ka); w.Kb = F(p.off_Kb); w.Wc = F(p.off_Wc); w.Fc = F(p.off_Fc); w.Kc = F(p.off_Kc);
  w.wpart = F(p.off_wpart);
  w.partials = F(p.off_partials);
  w.dig_a = reinterpret_cast<uint32_t*>(b + p.off_dig_a);
  w.dig_b = reinterpret_cast<uint32_t*>(b + p.off_dig_b);
  w.dig_in = reinterpret_cast<uint32_t*>(b + p.off_dig_in);
  w.dig_out = reinterpret_cast<uint32_t*>(b + p.off_dig_out);
  w.chal = F(p.off_chal);
  w.state = reinterpret_cast<DevState*>(b + p.off_state);
  w.cc = p.cc_bytes ? static_cast<void*>(b + p.off_cc) : nullptr;
  w.bytes = p.total;
  return w;
}

// ------------------------------------------------------------------ step builders

constexpr uint32_t kSweepTiles = 65535u * 8;  // grid-stride cap of plain sweeps
constexpr double kE = 32.0;                   // bytes per field element

constexpr uint32_t kInitRoundBlocks = 2048;  // workgroups of the fused table build + first round

static uint32_t tiles_for(uint64_t n, uint32_t cap) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (uint32_t)g;
}

static Step mk(uint32_t type, uint32_t ntiles) {
  Step st;
  memset(&st, 0, sizeof(st));
  st.type = type;
  st.ntiles = ntiles < 1 ? 1 : ntiles;
  return st;
}

void Program::to_mont(const gkr_fr* in, Fr* out, uint64_t n) {
  Step st = mk(ST_TO_MONT, tiles_for(n, kSweepTiles));
  st.p[0] = in; st.p[1] = out; st.q[0] = n;
  st.bytes = 2 * kE * n; st.mulmods = (double)n;
  steps.push_back(st);
}
void Program::from_mont(const Fr* in, gkr_fr* out, uint64_t n) {
  Step st = mk(ST_FROM_MONT, tiles_for(n, kSweepTiles));
  st.p[0] = in; st.p[1] = out; st.q[0] = n;
  st.bytes = 2 * kE * n; st.mulmods = (double)n;
  steps.push_back(st);
}
void Program::forward(const Fr* W, Fr* V, const uint2* gates, uint32_t n, uint64_t count, uint64_t mul_gates) {
  Step st = mk(ST_FORWARD, tiles_for(count, kSweepTiles));
  st.p[0] = W; st.p[1] = V; st.p[2] = gates; st.u[0] = n; st.q[0] = count;
  st.bytes = 3 * kE * count; st.mulmods = (double)mul_gates;
  steps.push_back(st);
}
void Program::digest(const gkr_fr* vec, uint64_t nelem, uint32_t* final_out, const Workspace& w) {
  const uint32_t* in = reinterpret_cast<const uint32_t*>(vec);
  uint64_t nwords = nelem * 8;
  int swap = 1;
  uint32_t* bufs[2] = {w.dig_a, w.dig_b};
  int which = 0;
  for (;;) {
    const uint64_t nchunks = (nwords + kChunkWords - 1) / kChunkWords;
    uint32_t* out = (nchunks == 1) ? final_out : bufs[which];
    Step st = mk(ST_DIGEST, tiles_for(nchunks, kSweepTiles));
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
void Program::transcript_begin(DevState* S, const Words8& seed_state, const uint32_t* circ,
                               const uint32_t* din, const uint32_t* dout) {
  Step st = mk(ST_TRANSCRIPT_BEGIN, 1);
  st.p[0] = S; st.p[1] = din; st.p[2] = dout;
  memcpy(st.w, seed_state.w, 32);
  memcpy(st.w + 8, circ, 32);
  steps.push_back(st);
}
void Program::squeeze(DevState* S, Fr* out, uint32_t count) {
  Step st = mk(ST_SQUEEZE, 1);
  st.p[0] = S; st.p[1] = out; st.u[0] = count; st.mulmods = count;
  steps.push_back(st);
}
void Program::layer_begin(DevState* S, bool first, const Fr* vu, const Fr* vv) {
  Step st = mk(ST_LAYER_BEGIN, 1);
  st.p[0] = S; st.p[1] = vu; st.p[2] = vv; st.u[0] = first ? 1 : 0; st.mulmods = 4;
  steps.push_back(st);
}
void Program::eq(int count, const uint32_t* bits, const Fr* const* points, const Fr* const* scales, Fr* const* outs) {
  uint64_t total = 0;
  double mm = 0;
  Step st = mk(ST_EQ, 1);
  for (int j = 0; j < count; ++j) {
    st.u[j] = bits[j];
    st.p[j] = points[j];
    st.p[4 + j] = scales[j];
    st.p[8 + j] = outs[j];
    total += 1ull << bits[j];
    mm += (double)(1ull << bits[j]) * (bits[j] + 1);
  }
  st.u[4] = count;
  st.ntiles = tiles_for(total, 1u << 30);
  st.bytes = kE * total; st.mulmods = mm;
  steps.push_back(st);
}
void Program::wsum(const Fr* V, const Fr* A, const Fr* B, uint32_t n, uint64_t count, Fr* partials,
                   DevState* S, Fr* dst, const Tuning& tun) {
  Step st = mk(ST_WSUM, tiles_for(count, tun.max_round_blocks));
  st.p[0] = V; st.p[1] = A; st.p[2] = B; st.p[3] = partials; st.p[4] = S; st.p[5] = dst;
  st.u[0] = n; st.q[0] = count;
  st.bytes = kE * count; st.mulmods = 2.0 * count;
  steps.push_back(st);
}
static void p1_common(Step& st, const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU,
                      const Fr* bV, const Fr* Cu, const Fr* Cv, uint32_t n) {
  st.p[0] = W; st.p[1] = G; st.p[2] = H; st.p[3] = lw.xrow; st.p[4] = lw.xent;
  st.p[5] = aU; st.p[6] = bV; st.p[7] = Cu; st.p[8] = Cv; st.u[0] = n;
}
void Program::p1_init(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU, const Fr* bV,
                      const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t count, uint64_t gates) {
  Step st = mk(ST_P1_INIT, tiles_for(count, kSweepTiles));
  p1_common(st, W, G, H, lw, aU, bV, Cu, Cv, n);
  st.q[0] = count;
  st.bytes = kE * (gates + 2.0 * count); st.mulmods = 2.5 * gates;  // T (1.5) and T W (1) per gate
  steps.push_back(st);
}
void Program::p1_init_round(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU,
                            const Fr* bV, const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t half,
                            uint64_t gates, DevState* S, Fr* partials, Fr* r_out, uint32_t* msg,
                            const Tuning& tun) {
  // at least four pairs per thread, up to kInitRoundBlocks workgroups (full
  // occupancy on the big tables whatever the round cap)
  Step st = mk(ST_P1_INIT_ROUND, tiles_for((half + 3) / 4, kInitRoundBlocks));
  p1_common(st, W, G, H, lw, aU, bV, Cu, Cv, n);
  st.q[0] = half;
  st.p[9] = S; st.p[10] = partials; st.p[11] = r_out; st.p[12] = msg;
  st.bytes = kE * (gates + 6.0 * half); st.mulmods = 2.5 * gates + 1.5 * half;  // + lazy w0 g0, product w2 g2
  steps.push_back(st);
}

// Algorithmic bytes and products of one round over `half` pairs of NT tables
// (eval_products products per evaluation point).
// Work of a step in product equivalents: a full Montgomery product is one, an
// unreduced 8x8-limb product and a reduction are a half each (a*b + c*d with
// one reduction is 1.5).
static void round_work(int nt, double eval_products, uint64_t half, bool fold, double& bytes, double& mm) {
  const double h = (double)half;
  bytes += fold ? kE * nt * 6.0 * h : kE * nt * 2.0 * h;
  mm += (fold ? 2.0 * nt * h : 0.0) + eval_products * 2.0 * h;
}

template <int NT>
void Program::round(const Fr* const* src, Fr* const* dst, uint64_t half, const Fr* rprev, DevState* S,
                    Fr* partials, Fr* r_out, uint32_t* msg, const Tuning& tun) {
  using R = RoundPtrs<NT>;
  Step st = mk(NT == 3 ? ST_ROUND_A : ST_ROUND_B,
               tiles_for((half + tun.pairs_per_thread - 1) / tun.pairs_per_thread, tun.max_round_blocks));
  for (int k = 0; k < NT; ++k) {
    st.p[k] = src[k];
    st.p[NT + k] = dst[k];
  }
  st.p[R::kR] = rprev; st.p[R::kS] = S; st.p[R::kPart] = partials; st.p[R::kROut] = r_out; st.p[R::kMsg] = msg;
  st.q[0] = half;
  round_work(NT, NT == 3 ? 1.0 : 1.5, half, rprev != nullptr, st.bytes, st.mulmods);
  steps.push_back(st);
}
template <int NT>
void Program::tail(const Fr* const* src, Fr* const* dst, uint64_t size, const Fr* rpending, uint32_t rounds,
                   DevState* S, Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value) {
  Step st = mk(NT == 3 ? ST_TAIL_A : ST_TAIL_B, 1);
  for (int k = 0; k < NT; ++k) {
    st.p[k] = src[k];
    st.p[NT + k] = dst[k];
  }
  st.p[2 * NT] = rpending; st.p[2 * NT + 1] = S; st.p[2 * NT + 2] = r_out; st.p[2 * NT + 3] = msg;
  st.p[2 * NT + 4] = final_out; st.p[2 * NT + 5] = proof_value;
  st.q[0] = size; st.u[0] = rounds;
  bool fold = rpending != nullptr;
  uint64_t sz = size;
  for (uint32_t j = 0; j < rounds; ++j) {
    const uint64_t ev = fold ? sz / 2 : sz;
    round_work(NT, NT == 3 ? 1.0 : 1.5, ev / 2, fold, st.bytes, st.mulmods);
    fold = true;
    sz = ev;
  }
  if (fold) st.mulmods += NT;
  steps.push_back(st);
}
void Program::copy_weights(const Fr* Cu, const Fr* Cv, const Fr* EC, Fr* U, Fr* V, uint64_t ncop, DevState* S) {
  Step st = mk(ST_COPY_WEIGHTS, 1);
  st.p[0] = Cu; st.p[1] = Cv; st.p[2] = EC; st.p[3] = U; st.p[4] = V; st.p[5] = S; st.q[0] = ncop;
  st.bytes = 5 * kE * ncop; st.mulmods = 2.0 * ncop;
  steps.push_back(st);
}
void Program::p2_tables(const LayerWiring& lw, const Fr* aU, const Fr* bV, const Fr* EL, const DevState* S,
                        Fr* Fa, Fr* Fb, Fr* Ka, Fr* Kb, Fr* Ks, uint64_t count, uint64_t gates) {
  Step st = mk(ST_P2_TABLES, tiles_for(count, kSweepTiles));
  st.p[0] = lw.yrow; st.p[1] = lw.yent; st.p[2] = aU; st.p[3] = bV; st.p[4] = EL; st.p[5] = S;
  st.p[6] = Fa; st.p[7] = Fb; st.p[8] = Ka; st.p[9] = Kb; st.p[10] = Ks; st.q[0] = count;
  st.bytes = kE * (3.0 * gates + 5.0 * count); st.mulmods = 2.0 * gates + 8.0 * count;
  steps.push_back(st);
}
void Program::copy_contract(const Fr* W, const Fr* U, const Fr* V, Fr* Pt, Fr* Qt, uint32_t n, uint64_t rows) {
  const uint32_t tpr_log = n < 8 ? n : 8;
  const uint64_t rows_per_tile = kBlock >> tpr_log;
  Step st = mk(ST_COPY_CONTRACT, (uint32_t)std::min<uint64_t>((rows + rows_per_tile - 1) / rows_per_tile, kSweepTiles));
  st.p[0] = W; st.p[1] = U; st.p[2] = V; st.p[3] = Pt; st.p[4] = Qt; st.u[0] = n; st.q[0] = rows;
  const double elems = (double)(rows << n);
  st.bytes = kE * elems; st.mulmods = elems;  // two unreduced products per entry
  steps.push_back(st);
}
void Program::local_contract(const Fr* W, const Fr* EqR, Fr* part, uint32_t n, uint64_t rows, uint32_t R) {
  const uint64_t xb = ((1ull << n) + kBlock - 1) / kBlock;
  Step st = mk(ST_LOCAL_CONTRACT, (uint32_t)std::min<uint64_t>(xb * R, kSweepTiles));
  st.p[0] = W; st.p[1] = EqR; st.p[2] = part; st.u[0] = n; st.u[1] = R; st.q[0] = rows;
  const double elems = (double)(rows << n);
  st.bytes = kE * elems; st.mulmods = 0.5 * elems;  // one unreduced product per entry
  steps.push_back(st);
}
void Program::copy_tables(const Fr* part, uint32_t R, const Fr* U, const Fr* V, const Fr* fa_f, const Fr* fb_f,
                          const DevState* S, Fr* Wc, Fr* Fc, Fr* Kc, uint64_t ncop) {
  uint32_t tpc_log = 0;  // lanes per column: min(R, 64), as the body computes it
  while (tpc_log < 6 && (2u << tpc_log) <= R) ++tpc_log;
  const uint64_t cols_per_tile = kBlock >> tpc_log;
  Step st = mk(ST_COPY_TABLES, (uint32_t)std::min<uint64_t>((ncop + cols_per_tile - 1) / cols_per_tile, kSweepTiles));
  st.p[0] = part; st.p[1] = U; st.p[2] = V; st.p[3] = fa_f; st.p[4] = fb_f; st.p[5] = S;
  st.p[6] = Wc; st.p[7] = Fc; st.p[8] = Kc; st.u[0] = R; st.q[0] = ncop;
  st.bytes = kE * (R + 5.0) * ncop; st.mulmods = 3.0 * ncop;
  steps.push_back(st);
}
void Program::local_values(const Fr* EqR, const Fr* Ka, const Fr* Kb, uint64_t rows, DevState* S, Fr* partials) {
  // two rows per thread: a short product chain per thread, then a grid reduction
  Step st = mk(ST_LOCAL_VALUES, tiles_for((rows + 1) / 2, 64));
  st.p[0] = EqR; st.p[1] = Ka; st.p[2] = Kb; st.p[3] = S; st.p[4] = partials; st.q[0] = rows;
  st.bytes = 3 * kE * rows; st.mulmods = 2.0 * rows;
  steps.push_back(st);
}
void Program::state_export(const DevState* S, uint8_t* out) {
  Step st = mk(ST_STATE_EXPORT, 1);
  st.p[0] = S; st.p[1] = out;
  steps.push_back(st);
}
void Program::state_import(DevState* S, const uint8_t* in) {
  Step st = mk(ST_STATE_IMPORT, 1);
  st.p[0] = S; st.p[1] = in;
  steps.push_back(st);
}

void Program::run(hipStream_t s) const {
  for (const Step& st : steps) {
    if (st.type >= ST_CC_BUILD) launch_cc_step(st, s);
    else if (st.type >= ST_VPD_POWERS) launch_vpd_step(st, s);
    else if (st.type >= ST_GL_FORWARD) launch_gl_step(st, s);
    else if (st.type >= ST_G_GATHER) launch_general_step(st, s);
    else launch_step(st, s);
  }
}

// ------------------------------------------------------------------ proof programs

// The round schedule of one phase over NT-table forms: grid-wide rounds while
// the evaluated table exceeds the tail size, then one workgroup. With
// first_round > 0 the rounds before it were already evaluated (their
// challenge is pending) and the tables have 2^(nrounds - first_round + 1) entries.
template <int NT>
static void emit_phase(Program& pg, const Fr* const* src0, Fr* const* dst, uint32_t nrounds, DevState* S,
                       Fr* partials, Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value,
                       const Tuning& tun, uint32_t first_round = 0) {
  const Fr* src[NT];
  for (int k = 0; k < NT; ++k) src[k] = src0[k];
  uint64_t eval = 1ull << (nrounds - first_round);
  uint32_t j = first_round;
  const Fr* pending = first_round ? r_out + first_round - 1 : nullptr;
  while (j < nrounds && eval > (1ull << tun.tail_log)) {
    pg.round<NT>(src, dst, eval / 2, pending, S, partials, r_out + j, msg + 24 * j, tun);
    if (pending) {
      for (int k = 0; k < NT; ++k) src[k] = dst[k];
    }
    pending = r_out + j;
    ++j;
    eval /= 2;
  }
  const uint64_t size = pending ? 2 * eval : eval;
  pg.tail<NT>(src, dst, size, pending, nrounds - j, S, r_out + j, msg + 24 * j, final_out, proof_value);
}

void emit_phase_a(Program& pg, const Fr* const* src0, Fr* const* dst, uint32_t nrounds, DevState* S, Fr* partials,
                  Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value, const Tuning& tun) {
  emit_phase<3>(pg, src0, dst, nrounds, S, partials, r_out, msg, final_out, proof_value, tun);
}

// One gate layer (A3-A7). W = V_{i+1} in Montgomery form; u, v points of
// layer i (s_i entries each, v = u on layer 0); vu, vv the claimed values.
void emit_layer(Program& pg, const gkr_circuit& c, uint32_t i, const Workspace& w, const Fr* W, const Fr* u,
                const Fr* v, const Fr* vu, const Fr* vv, Fr* rx, Fr* ry, uint32_t* proof, const Tuning& tun) {
  const uint32_t n = c.n, sg = c.sigma[i], sg1 = c.sigma[i + 1], s1 = c.s(i + 1);
  DevState* S = w.state;
  pg.layer_begin(S, i == 0, vu, vv);
  {
    const uint32_t bits[4] = {sg, sg, n, n};
    const Fr* pts[4] = {u, v, u + sg, v + sg};
    const Fr* scl[4] = {&S->alpha, &S->beta, nullptr, nullptr};
    Fr* outs[4] = {w.aU, w.bV, w.Cu, w.Cv};
    pg.eq(4, bits, pts, scl, outs);
  }
  // Phase 1: tables (and, for big tables, round 1 in the same pass), then the rounds.
  const Fr* ta_src[3] = {W, w.G, w.H};
  Fr* ta_dst[3] = {w.Wf, w.G, w.H};
  const uint32_t off_vx = 24 * s1, off_p2 = off_vx + 8, off_vy = off_p2 + 24 * s1;
  if (s1 > tun.tail_log) {
    pg.p1_init_round(W, w.G, w.H, c.wiring[i], w.aU, w.bV, w.Cu, w.Cv, n, 1ull << (s1 - 1), 1ull << c.s(i), S,
                     w.partials, rx, proof, tun);
    emit_phase<3>(pg, ta_src, ta_dst, s1, S, w.partials, rx, proof, &S->vx, proof + off_vx, tun, 1);
  } else {
    pg.p1_init(W, w.G, w.H, c.wiring[i], w.aU, w.bV, w.Cu, w.Cv, n, 1ull << s1, 1ull << c.s(i));
    emit_phase<3>(pg, ta_src, ta_dst, s1, S, w.partials, rx, proof, &S->vx, proof + off_vx, tun);
  }
  // Phase 2: sub-circuit rounds with the copy factors contracted, then the copy rounds.
  {
    const uint32_t bits[2] = {sg1, n};
    const Fr* pts[2] = {rx, rx + sg1};
    const Fr* scl[2] = {nullptr, nullptr};
    Fr* outs[2] = {w.EL, w.EC};
    pg.eq(2, bits, pts, scl, outs);
  }
  pg.copy_weights(w.Cu, w.Cv, w.EC, w.U, w.V, 1ull << n, S);
  pg.p2_tables(c.wiring[i], w.aU, w.bV, w.EL, S, w.Fa, w.Fb, w.Ka, w.Kb, w.Ks, 1ull << sg1, 1ull << sg);
  if (pg.matrix_cores && tun.matrix_cores && w.cc && cc_applies(n, sg1)) emit_copy_contract_mfma(pg, W, w.U, w.V, w.P, w.Q, n, sg1, w.cc);
  else pg.copy_contract(W, w.U, w.V, w.P, w.Q, n, 1ull << sg1);
  Fr* tb[5] = {w.P, w.Fa, w.Q, w.Fb, w.Ks};
  const Fr* tb_src[5] = {w.P, w.Fa, w.Q, w.Fb, w.Ks};
  emit_phase<5>(pg, tb_src, tb, sg1, S, w.partials, ry, proof + off_p2, &S->scratch[1], nullptr, tun);
  {
    const uint32_t bits[1] = {sg1};
    const Fr* pts[1] = {ry};
    const Fr* scl[1] = {nullptr};
    Fr* outs[1] = {w.EqR};
    pg.eq(1, bits, pts, scl, outs);
  }
  pg.local_values(w.EqR, w.Ka, w.Kb, 1ull << sg1, S, w.partials);
  pg.local_contract(W, w.EqR, w.wpart, n, 1ull << sg1, c.plan.ychunks);
  pg.copy_tables(w.wpart, c.plan.ychunks, w.U, w.V, w.Fa, w.Fb, S, w.Wc, w.Fc, w.Kc, 1ull << n);
  Fr* tc[3] = {w.Wc, w.Fc, w.Kc};
  const Fr* tc_src[3] = {w.Wc, w.Fc, w.Kc};
  emit_phase<3>(pg, tc_src, tc, n, S, w.partials, ry + sg1, proof + off_p2 + 24 * sg1, &S->vy, proof + off_vy, tun);
}

// Forward evaluation of every layer from Montgomery inputs in layer[d].
static void emit_forward(Program& pg, const gkr_circuit& c, const Workspace& w) {
  for (int i = (int)c.depth - 1; i >= 0; --i)
    pg.forward(w.layer[i + 1], w.layer[i], c.wiring[i].gates, c.n, 1ull << c.s(i), (uint64_t)c.mul_gates[i] << c.n);
}

// g and the output claim V_0~(g) (into S->scratch[0]); needs layer[0] in Montgomery form.
static void emit_output_claim(Program& pg, const gkr_circuit& c, const Workspace& w, const Tuning& tun) {
  DevState* S = w.state;
  Fr* g = w.chal;
  pg.squeeze(S, g, c.s(0));
  const uint32_t bits[2] = {c.sigma[0], c.n};
  const Fr* pts[2] = {g, g + c.sigma[0]};
  const Fr* scl[2] = {nullptr, nullptr};
  Fr* outs[2] = {w.aU, w.Cu};
  pg.eq(2, bits, pts, scl, outs);
  pg.wsum(w.layer[0], w.aU, w.Cu, c.n, 1ull << c.s(0), w.partials, S, &S->scratch[0], tun);
}

static size_t layer_proof_words(const gkr_circuit& c, uint32_t i) {
  if (c.general) return general_layer_proof_bytes(c, i) / 4;
  if (c.field == GKR_FIELD_GOLDILOCKS) return (6ull * c.s(i + 1) + 2) * 2;
  return (6ull * c.s(i + 1) + 2) * 8;
}

void emit_statement_and_output_claim(Program& pg, const gkr_circuit& c, const Workspace& w, const gkr_fr* d_inputs,
                                     const gkr_fr* d_outputs, uint64_t seed, const Tuning& tun) {
  pg.digest(d_inputs, 1ull << c.s(c.depth), w.dig_in, w);
  pg.digest(d_outputs, 1ull << c.s(0), w.dig_out, w);
  pg.transcript_begin(w.state, seed_state(seed), c.digest, w.dig_in, w.dig_out);
  emit_output_claim(pg, c, w, tun);
}

// The whole proof of gkr_prove_circuit as a step program.
void emit_prove_circuit(Program& pg, const gkr_circuit& c, const Workspace& w, const gkr_fr* d_inputs,
                        uint64_t seed, gkr_fr* d_outputs, uint8_t* d_proof, const Tuning& tun) {
  pg.to_mont(d_inputs, w.layer[c.depth], 1ull << c.s(c.depth));
  emit_forward(pg, c, w);
  pg.from_mont(w.layer[0], d_outputs, 1ull << c.s(0));
  pg.digest(d_inputs, 1ull << c.s(c.depth), w.dig_in, w);
  pg.digest(d_outputs, 1ull << c.s(0), w.dig_out, w);
  pg.transcript_begin(w.state, seed_state(seed), c.digest, w.dig_in, w.dig_out);
  emit_output_claim(pg, c, w, tun);
  uint32_t* proof = reinterpret_cast<uint32_t*>(d_proof);
  DevState* S = w.state;
  for (uint32_t i = 0; i < c.depth; ++i) {
    const Fr* u = (i == 0) ? w.chal : w.chal + host_chal_index_rx(c, i - 1);
    const Fr* v = (i == 0) ? w.chal : w.chal + host_chal_index_ry(c, i - 1);
    const Fr* vu = (i == 0) ? &S->scratch[0] : &S->vx;
    emit_layer(pg, c, i, w, w.layer[i + 1], u, v, vu, &S->vy, w.chal + host_chal_index_rx(c, i),
               w.chal + host_chal_index_ry(c, i), proof, tun);
    proof += layer_proof_words(c, i);
  }
}

// The proof of gkr_prove_circuit_committed: the inputs are committed
// (Section 2.4) before the statement is bound, the statement absorbs the
// commitment root in place of the input digest, the layers are proved as in
// emit_prove_circuit, and the commitment is opened at the last layer's two
// points. Proof: root (32 bytes) || layers || opening.
void emit_prove_committed(Program& pg, const gkr_circuit& c, const Workspace& w, const VpdPlan& vp, void* vbase,
                          const gkr_fr* d_inputs, uint64_t seed, gkr_fr* d_outputs, uint8_t* d_proof,
                          const Tuning& tun) {
  const uint32_t d = c.depth;
  pg.to_mont(d_inputs, w.layer[d], 1ull << c.s(d));
  emit_forward(pg, c, w);
  pg.from_mont(w.layer[0], d_outputs, 1ull << c.s(0));
  emit_vpd_commit(pg, vp, vbase, w.layer[d]);
  emit_vpd_root_out(pg, vp, vbase, d_proof);
  pg.digest(d_outputs, 1ull << c.s(0), w.dig_out, w);
  pg.transcript_begin(w.state, seed_state(seed), c.digest, vpd_root_words(vp, vbase), w.dig_out);
  emit_output_claim(pg, c, w, tun);
  uint32_t* proof = reinterpret_cast<uint32_t*>(d_proof + 32);
  DevState* S = w.state;
  for (uint32_t i = 0; i < d; ++i) {
    const Fr* u = (i == 0) ? w.chal : w.chal + host_chal_index_rx(c, i - 1);
    const Fr* v = (i == 0) ? w.chal : w.chal + host_chal_index_ry(c, i - 1);
    const Fr* vu = (i == 0) ? &S->scratch[0] : &S->vx;
    emit_layer(pg, c, i, w, w.layer[i + 1], u, v, vu, &S->vy, w.chal + host_chal_index_rx(c, i),
               w.chal + host_chal_index_ry(c, i), proof, tun);
    proof += layer_proof_words(c, i);
  }
  emit_vpd_open(pg, vp, vbase, w.layer[d], S, w.chal + host_chal_index_rx(c, d - 1),
                w.chal + host_chal_index_ry(c, d - 1), c.sigma[d], c.n, reinterpret_cast<uint8_t*>(proof));
}

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

static int32_t check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return GKR_EDEVICE;
  }
  return GKR_OK;
}

// The BN254 proving calls refuse Goldilocks circuits.
static int32_t check_bn254(const gkr_circuit* c) {
  if (c && c->field != GKR_FIELD_BN254) {
    set_error("this circuit is over the Goldilocks field: use gkr_gl_prove_circuit / gkr_gl_verify");
    return GKR_EINVAL;
  }
  return GKR_OK;
}

int32_t check_ws(const gkr_circuit* c, const void* ws, size_t ws_bytes) {
  if (c->device < 0) {
    set_error("circuit was created without a HIP device (host-only: verification only)");
    return GKR_EDEVICE;
  }
  if (!ws || !aligned16(ws)) {
    set_error("workspace pointer is null or not 16-byte aligned");
    return GKR_EINVAL;
  }
  if (ws_bytes < c->plan.total) {
    set_error("workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(c->plan.total));
    return GKR_EBUFSZ;
  }
  return GKR_OK;
}

}  // namespace gkr

gkr_circuit::~gkr_circuit() {
  if (dev_block) hipFree(dev_block);
  gkr::general_destroy(general);
}

using namespace gkr;

// ====================================================================== C ABI

extern "C" {

const char* gkr_last_error(void) { return g_last_error.c_str(); }

int32_t gkr_circuit_create(uint32_t depth, uint32_t log_copies, const uint32_t* log_sub_width,
                           const gkr_gate* const* gates, gkr_circuit** out) {
  try {
    if (!out || !log_sub_width || !gates) {
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
      if (log_sub_width[i] > GKR_MAX_LOG_WIDTH || log_sub_width[i] + log_copies > GKR_MAX_LOG_WIDTH) {
        set_error("layer " + std::to_string(i) + " is wider than 2^" + std::to_string(GKR_MAX_LOG_WIDTH));
        return GKR_EUNSUPPORTED;
      }
    }
    gkr_circuit* c = new gkr_circuit();
    c->depth = depth;
    c->n = log_copies;
    c->sigma.assign(log_sub_width, log_sub_width + depth + 1);
    c->gates.resize(depth);
    // (on the failure paths below `delete c` also frees the device block)
    for (uint32_t i = 0; i < depth; ++i) {
      if (!gates[i]) {
        delete c;
        set_error("null gate list for layer " + std::to_string(i));
        return GKR_EINVAL;
      }
      const uint64_t cnt = 1ull << c->sigma[i];
      const uint64_t lim = 1ull << c->sigma[i + 1];
      c->gates[i].assign(gates[i], gates[i] + cnt);
      c->mul_gates.push_back(0);
      for (uint64_t z = 0; z < cnt; ++z) {
        const gkr_gate& g = c->gates[i][z];
        c->mul_gates.back() += g.type == GKR_GATE_MUL;
        if (g.x >= lim || g.y >= lim || g.type > 1) {
          delete c;
          set_error("layer " + std::to_string(i) + " gate " + std::to_string(z) + " is invalid");
          return GKR_EINVAL;
        }
      }
    }
    // circuit digest
    {
      std::vector<uint8_t> msg;
      auto put32 = [&](uint32_t v) {
        for (int k = 0; k < 4; ++k) msg.push_back((uint8_t)(v >> (8 * k)));
      };
      put32(depth);
      put32(log_copies);
      for (uint32_t i = 0; i <= depth; ++i) put32(c->sigma[i]);
      for (uint32_t i = 0; i < depth; ++i)
        for (const gkr_gate& g : c->gates[i]) {
          put32(g.x);
          put32(g.y);
          msg.push_back((uint8_t)g.type);
        }
      sha256_bytes(msg.data(), msg.size(), c->digest);
    }
    // wiring indexes: gate records, CSR by x and by y, in one device block
    std::vector<size_t> offs(5 * depth);
    size_t total = 0;
    auto take = [&](size_t bytes) {
      size_t o = total;
      total = (total + bytes + 255) & ~(size_t)255;
      return o;
    };
    for (uint32_t i = 0; i < depth; ++i) {
      const size_t cnt = 1ull << c->sigma[i], rows = (1ull << c->sigma[i + 1]) + 1;
      offs[5 * i + 0] = take(8 * cnt);
      offs[5 * i + 1] = take(4 * rows);
      offs[5 * i + 2] = take(8 * cnt);
      offs[5 * i + 3] = take(4 * rows);
      offs[5 * i + 4] = take(8 * cnt);
    }
    std::vector<uint8_t> host(total, 0);
    for (uint32_t i = 0; i < depth; ++i) {
      const size_t cnt = 1ull << c->sigma[i], rows = 1ull << c->sigma[i + 1];
      uint32_t* rec = reinterpret_cast<uint32_t*>(host.data() + offs[5 * i + 0]);
      uint32_t* xrow = reinterpret_cast<uint32_t*>(host.data() + offs[5 * i + 1]);
      uint32_t* xent = reinterpret_cast<uint32_t*>(host.data() + offs[5 * i + 2]);
      uint32_t* yrow = reinterpret_cast<uint32_t*>(host.data() + offs[5 * i + 3]);
      uint32_t* yent = reinterpret_cast<uint32_t*>(host.data() + offs[5 * i + 4]);
      const std::vector<gkr_gate>& gl = c->gates[i];
      for (size_t z = 0; z < cnt; ++z) {
        rec[2 * z] = gl[z].x | ((uint32_t)gl[z].type << 31);
        rec[2 * z + 1] = gl[z].y;
        xrow[gl[z].x + 1]++;
        yrow[gl[z].y + 1]++;
      }
      for (size_t r = 0; r < rows; ++r) {
        xrow[r + 1] += xrow[r];
        yrow[r + 1] += yrow[r];
      }
      std::vector<uint32_t> fx(xrow, xrow + rows), fy(yrow, yrow + rows);
      for (size_t z = 0; z < cnt; ++z) {
        const uint32_t kx = fx[gl[z].x]++, ky = fy[gl[z].y]++;
        xent[2 * kx] = (uint32_t)z;
        xent[2 * kx + 1] = gl[z].y | ((uint32_t)gl[z].type << 31);
        yent[2 * ky] = (uint32_t)z;
        yent[2 * ky + 1] = gl[z].x | ((uint32_t)gl[z].type << 31);
      }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) {
      // No HIP device: a host-only circuit, usable by gkr_verify.
      (void)hipGetLastError();
      c->device = -1;
      plan_workspace(*c, c->plan);
      *out = c;
      return GKR_OK;
    }
    hipGetDevice(&c->device);
    if (hipMalloc(&c->dev_block, total) != hipSuccess) {
      (void)hipGetLastError();
      c->dev_block = nullptr;
      delete c;
      set_error("device allocation of the wiring failed");
      return GKR_ENOMEM;
    }
    if (hipMemcpy(c->dev_block, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      delete c;
      set_error("upload of the wiring failed");
      return GKR_EDEVICE;
    }
    c->wiring.resize(depth);
    char* base = static_cast<char*>(c->dev_block);
    for (uint32_t i = 0; i < depth; ++i) {
      c->wiring[i].gates = reinterpret_cast<const uint2*>(base + offs[5 * i + 0]);
      c->wiring[i].xrow = reinterpret_cast<const uint32_t*>(base + offs[5 * i + 1]);
      c->wiring[i].xent = reinterpret_cast<const uint2*>(base + offs[5 * i + 2]);
      c->wiring[i].yrow = reinterpret_cast<const uint32_t*>(base + offs[5 * i + 3]);
      c->wiring[i].yent = reinterpret_cast<const uint2*>(base + offs[5 * i + 4]);
    }
    plan_workspace(*c, c->plan);
    *out = c;
    return GKR_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  } catch (...) {
    set_error("unexpected failure");
    return GKR_EINVAL;
  }
}

void gkr_circuit_destroy(gkr_circuit* c) { delete c; }

int32_t gkr_circuit_create_field(uint32_t field, uint32_t depth, uint32_t log_copies, const uint32_t* log_sub_width,
                                 const gkr_gate* const* gates, gkr_circuit** out) {
  if (field != GKR_FIELD_BN254 && field != GKR_FIELD_GOLDILOCKS) {
    set_error("unknown field " + std::to_string(field));
    return GKR_EINVAL;
  }
  const int32_t rc = gkr_circuit_create(depth, log_copies, log_sub_width, gates, out);
  if (rc != GKR_OK || field == GKR_FIELD_BN254) return rc;
  (*out)->field = GKR_FIELD_GOLDILOCKS;
  plan_gl_workspace(**out);
  return GKR_OK;
}

size_t gkr_workspace_bytes(const gkr_circuit* c) { return c ? c->plan.total : 0; }

size_t gkr_layer_proof_bytes(const gkr_circuit* c, uint32_t layer) {
  if (!c || layer >= c->depth) return 0;
  return layer_proof_words(*c, layer) * 4;
}

size_t gkr_proof_bytes(const gkr_circuit* c) {
  if (!c) return 0;
  if (c->general) return general_proof_bytes(*c);
  if (c->field == GKR_FIELD_GOLDILOCKS) return gl_proof_bytes(*c);
  size_t t = 0;
  for (uint32_t i = 0; i < c->depth; ++i) t += layer_proof_words(*c, i) * 4;
  return t;
}

uint64_t gkr_gate_layers(const gkr_circuit* c) {
  if (!c) return 0;
  uint64_t t = 0;
  for (uint32_t i = 0; i < c->depth; ++i) t += 1ull << c->s(i);
  return t;
}

int32_t gkr_transcript_init(const gkr_circuit* c, uint64_t seed, const gkr_fr* d_inputs,
                            const gkr_fr* d_outputs, gkr_transcript* d_transcript, void* d_ws, size_t ws_bytes,
                            void* stream) {
  if (int32_t rc = check_bn254(c)) return rc;
  uint8_t* d_state = d_transcript ? d_transcript->state : nullptr;
  if (!c || !d_inputs || !d_outputs || !d_state || !aligned16(d_inputs) || !aligned16(d_outputs)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  try {
    Workspace w = bind_workspace(*c, d_ws);
    Program pg;
    pg.digest(d_inputs, 1ull << c->s(c->depth), w.dig_in, w);
    pg.digest(d_outputs, 1ull << c->s(0), w.dig_out, w);
    pg.transcript_begin(w.state, seed_state(seed), c->digest, w.dig_in, w.dig_out);
    pg.state_export(w.state, d_state);
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  return check_launch();
}

int32_t gkr_output_claim(const gkr_circuit* c, const gkr_fr* d_outputs, gkr_transcript* d_transcript,
                         gkr_fr* d_g, gkr_fr* d_claim, void* d_ws, size_t ws_bytes, void* stream) {
  if (int32_t rc = check_bn254(c)) return rc;
  uint8_t* d_state = d_transcript ? d_transcript->state : nullptr;
  if (!c || !d_outputs || !d_state || !d_claim || (!d_g && c->s(0) > 0) || !aligned16(d_outputs) ||
      (d_g && !aligned16(d_g)) || !aligned16(d_claim)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  try {
    Workspace w = bind_workspace(*c, d_ws);
    Program pg;
    pg.state_import(w.state, d_state);
    pg.to_mont(d_outputs, w.layer[0], 1ull << c->s(0));
    emit_output_claim(pg, *c, w, current_tuning());
    if (c->s(0) > 0) pg.from_mont(w.chal, d_g, c->s(0));
    pg.from_mont(&w.state->scratch[0], d_claim, 1);
    pg.state_export(w.state, d_state);
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  return check_launch();
}

int32_t gkr_prove_layer(const gkr_circuit* c, uint32_t layer, const gkr_fr* d_next,
                        const gkr_fr* d_u, const gkr_fr* d_v, const gkr_fr* d_claim_u,
                        const gkr_fr* d_claim_v, gkr_transcript* d_transcript, gkr_fr* d_rx, gkr_fr* d_ry,
                        gkr_fr* d_vx, gkr_fr* d_vy, uint8_t* d_layer_proof, void* d_ws,
                        size_t ws_bytes, void* stream) {
  if (!c || layer >= c->depth) {
    set_error("bad circuit or layer");
    return GKR_EINVAL;
  }
  if (c->general) {
    set_error("gkr_prove_layer takes layered circuits only (a general circuit's layers share claims)");
    return GKR_EUNSUPPORTED;
  }
  if (int32_t rc = check_bn254(c)) return rc;
  const bool first = layer == 0;
  const uint32_t si = c->s(layer), s1 = c->s(layer + 1);
  uint8_t* d_state = d_transcript ? d_transcript->state : nullptr;
  if (!d_next || !d_claim_u || !d_state || !d_vx || !d_vy || !d_layer_proof ||
      (si > 0 && !d_u) || (!first && (!d_claim_v || (si > 0 && !d_v))) ||
      (s1 > 0 && (!d_rx || !d_ry))) {
    set_error("null argument");
    return GKR_EINVAL;
  }
  const void* ptrs[] = {d_next, d_u, d_v, d_claim_u, d_claim_v, d_rx, d_ry, d_vx, d_vy, d_layer_proof};
  for (const void* p : ptrs)
    if (p && !aligned16(p)) {
      set_error("device buffers must be 16-byte aligned");
      return GKR_EINVAL;
    }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  try {
    Workspace w = bind_workspace(*c, d_ws);
    const uint32_t sc = chal_index_scratch(*c);
    const uint32_t smax = s_max_of(*c);
    Fr* u = w.chal + sc;
    Fr* v = u + smax;
    Fr* cl = v + smax;  // cl[0] = claim_u, cl[1] = claim_v
    Program pg;
    pg.state_import(w.state, d_state);
    pg.to_mont(d_next, w.layer[layer + 1], 1ull << s1);
    if (si > 0) {
      pg.to_mont(d_u, u, si);
      pg.to_mont(first ? d_u : d_v, v, si);
    }
    pg.to_mont(d_claim_u, cl, 1);
    pg.to_mont(first ? d_claim_u : d_claim_v, cl + 1, 1);
    Fr* rx = w.chal + host_chal_index_rx(*c, layer);
    Fr* ry = w.chal + host_chal_index_ry(*c, layer);
    emit_layer(pg, *c, layer, w, w.layer[layer + 1], u, v, cl, cl + 1, rx, ry,
               reinterpret_cast<uint32_t*>(d_layer_proof), current_tuning());
    if (s1 > 0) {
      pg.from_mont(rx, d_rx, s1);
      pg.from_mont(ry, d_ry, s1);
    }
    pg.from_mont(&w.state->vx, d_vx, 1);
    pg.from_mont(&w.state->vy, d_vy, 1);
    pg.state_export(w.state, d_state);
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  return check_launch();
}

int32_t gkr_prove_circuit(const gkr_circuit* c, const gkr_fr* d_inputs, uint64_t seed,
                          gkr_fr* d_outputs, uint8_t* d_proof, size_t proof_cap, size_t* proof_len,
                          void* d_ws, size_t ws_bytes, void* stream) {
  if (!c || !d_inputs || !d_outputs || !d_proof || !aligned16(d_inputs) || !aligned16(d_outputs) ||
      !aligned16(d_proof)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  if (int32_t rc0 = check_bn254(c)) return rc0;
  const size_t need = gkr_proof_bytes(c);
  if (proof_len) *proof_len = need;
  if (proof_cap < need) {
    set_error("proof buffer too small: " + std::to_string(proof_cap) + " < " + std::to_string(need));
    return GKR_EBUFSZ;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  try {
    Program pg;
    if (c->general) {
      emit_prove_general(pg, *c, d_ws, d_inputs, seed, d_outputs, d_proof, current_tuning());
    } else {
      Workspace w = bind_workspace(*c, d_ws);
      emit_prove_circuit(pg, *c, w, d_inputs, seed, d_outputs, d_proof, current_tuning());
    }
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  return check_launch();
}

// ---------------------------------------------------------------- committed inputs

static int32_t check_committed(const gkr_circuit* c, uint32_t queries) {
  if (!c) {
    set_error("null circuit");
    return GKR_EINVAL;
  }
  if (c->general || c->field != GKR_FIELD_BN254) {
    set_error("committed proofs cover layered circuits over BN254");
    return GKR_EUNSUPPORTED;
  }
  if (c->depth < 1) {
    set_error("a committed proof needs at least one gate layer");
    return GKR_EINVAL;
  }
  const uint32_t s = c->s(c->depth);
  if (s < 1 || s > kVpdMaxLogN) {
    set_error("the commitment takes 2^1 .. 2^" + std::to_string(kVpdMaxLogN) + " inputs, not 2^" + std::to_string(s));
    return GKR_EUNSUPPORTED;
  }
  if (queries < 1 || queries > GKR_MAX_QUERIES) {
    set_error("queries must be in 1 .. " + std::to_string(GKR_MAX_QUERIES));
    return GKR_EINVAL;
  }
  return GKR_OK;
}

int32_t gkr_committed_sizes(const gkr_circuit* c, uint32_t queries, size_t* ws_bytes, size_t* proof_bytes) {
  if (int32_t rc = check_committed(c, queries)) return rc;
  const VpdPlan vp = plan_vpd(c->s(c->depth), queries, c->n);
  if (ws_bytes) *ws_bytes = ((c->plan.total + 255) & ~(size_t)255) + vp.total;
  if (proof_bytes) *proof_bytes = 32 + gkr_proof_bytes(c) + vpd_opening_bytes(vp.s, queries);
  return GKR_OK;
}

int32_t gkr_prove_circuit_committed(const gkr_circuit* c, const gkr_fr* d_inputs, uint64_t seed, uint32_t queries,
                                    gkr_fr* d_outputs, uint8_t* d_proof, size_t proof_cap, void* d_ws,
                                    size_t ws_bytes, void* stream) {
  if (int32_t rc = check_committed(c, queries)) return rc;
  if (!d_inputs || !d_outputs || !d_proof || !aligned16(d_inputs) || !aligned16(d_outputs) || !aligned16(d_proof)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  size_t need_ws = 0, need_proof = 0;
  gkr_committed_sizes(c, queries, &need_ws, &need_proof);
  if (proof_cap < need_proof) {
    set_error("proof buffer too small: " + std::to_string(proof_cap) + " < " + std::to_string(need_proof));
    return GKR_EBUFSZ;
  }
  if (int32_t rc = check_ws(c, d_ws, ws_bytes)) return rc;
  if (ws_bytes < need_ws) {
    set_error("workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(need_ws));
    return GKR_EBUFSZ;
  }
  try {
    Program pg;
    Workspace w = bind_workspace(*c, d_ws);
    const VpdPlan vp = plan_vpd(c->s(c->depth), queries, c->n);
    void* vbase = static_cast<char*>(d_ws) + ((c->plan.total + 255) & ~(size_t)255);
    emit_prove_committed(pg, *c, w, vp, vbase, d_inputs, seed, d_outputs, d_proof, current_tuning());
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  return check_launch();
}

int32_t gkr_vpd_workspace_bytes(uint32_t log_n, size_t* bytes) {
  if (log_n < 1 || log_n > kVpdMaxLogN) {
    set_error("the commitment takes 2^1 .. 2^" + std::to_string(kVpdMaxLogN) + " values");
    return GKR_EUNSUPPORTED;
  }
  if (bytes) *bytes = (((sizeof(Fr) << log_n) + 255) & ~(size_t)255) + plan_vpd(log_n, 1, 0).total;
  return GKR_OK;
}

int32_t gkr_vpd_commit(uint32_t log_n, const gkr_fr* d_values, uint8_t* d_root, void* d_ws, size_t ws_bytes,
                       void* stream) {
  size_t need = 0;
  if (int32_t rc = gkr_vpd_workspace_bytes(log_n, &need)) return rc;
  if (!d_values || !d_root || !d_ws || !aligned16(d_values) || !aligned16(d_ws)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  if (ws_bytes < need) {
    set_error("workspace too small: " + std::to_string(ws_bytes) + " < " + std::to_string(need));
    return GKR_EBUFSZ;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0) {
    set_error("no HIP device");
    return GKR_EDEVICE;
  }
  try {
    Program pg;
    Fr* mont = static_cast<Fr*>(d_ws);
    void* vbase = static_cast<char*>(d_ws) + (((sizeof(Fr) << log_n) + 255) & ~(size_t)255);
    const VpdPlan vp = plan_vpd(log_n, 1, 0);
    pg.to_mont(d_values, mont, 1ull << log_n);
    emit_vpd_commit(pg, vp, vbase, mont);
    emit_vpd_root_out(pg, vp, vbase, d_root);
    pg.run(static_cast<hipStream_t>(stream));
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
  return check_launch();
}

}  // extern "C"
