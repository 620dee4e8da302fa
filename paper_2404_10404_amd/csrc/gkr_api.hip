// Host driver and C ABI of the GKR prover: circuit objects, workspace layout,
// and the launch sequence of a proof (all on the caller's stream, no host
// synchronisation, no allocation while proving).
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gkr_kernels.hpp"
#include "gkr_tuning.hpp"

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
  // row split of the copy-table pass: about 2^20 threads in total (a power of two)
  uint64_t want = (n >= 20) ? 1 : (1ull << (20 - n));
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
  w.bytes = p.total;
  return w;
}

// ------------------------------------------------------------------ proof pieces

static void run_digest(const gkr_fr* vec, uint64_t nelem, uint32_t* final_out, const Workspace& w,
                       hipStream_t s) {
  const uint32_t* in = reinterpret_cast<const uint32_t*>(vec);
  uint64_t nwords = nelem * 8;
  int swap = 1;
  uint32_t* bufs[2] = {w.dig_a, w.dig_b};
  int which = 0;
  for (;;) {
    const uint64_t nchunks = (nwords + kChunkWords - 1) / kChunkWords;
    uint32_t* out = (nchunks == 1) ? final_out : bufs[which];
    launch_digest_level(in, nwords, swap, out, nchunks, s);
    if (nchunks == 1) break;
    in = out;
    nwords = nchunks * 8;
    swap = 0;
    which ^= 1;
  }
}

// The round schedule of one phase over FormA/FormB tables: grid-wide rounds
// while the evaluated table exceeds the tail size, then one workgroup.
template <class Form>
static void run_phase(Tabs<Form::NT> t, uint32_t nrounds, DevState* S, Fr* partials, Fr* r_out,
                      uint32_t* msg, Fr* final_out, uint32_t* proof_value, const Tuning& tun,
                      hipStream_t s, uint32_t first_round = 0) {
  // first_round > 0: the rounds before it were already evaluated (their
  // challenge is pending) and the tables have 2^(nrounds - first_round + 1) entries.
  uint64_t eval = 1ull << (nrounds - first_round);
  uint32_t j = first_round;
  const Fr* pending = first_round ? r_out + first_round - 1 : nullptr;
  while (j < nrounds && eval > (1ull << tun.tail_log)) {
    launch_round<Form>(t, eval / 2, pending, S, partials, r_out + j, msg + 24 * j,
                       tun.max_round_blocks, s);
    if (pending) {
      for (int k = 0; k < Form::NT; ++k) t.src[k] = t.dst[k];
    }
    pending = r_out + j;
    ++j;
    eval /= 2;
  }
  const uint64_t size = pending ? 2 * eval : eval;
  launch_tail<Form>(t, size, pending, nrounds - j, S, r_out + j, msg + 24 * j, final_out,
                    proof_value, s);
}

// One gate layer (A3-A7). W = V_{i+1} in Montgomery form; u, v points of
// layer i (s_i entries each, v = u on layer 0); vu, vv the claimed values.
static void run_layer(const gkr_circuit& c, uint32_t i, const Workspace& w, const Fr* W,
                      const Fr* u, const Fr* v, const Fr* vu, const Fr* vv, Fr* rx, Fr* ry,
                      uint32_t* proof, const Tuning& tun, hipStream_t s) {
  const uint32_t n = c.n, sg = c.sigma[i], sg1 = c.sigma[i + 1], s1 = c.s(i + 1);
  DevState* S = w.state;
  launch_layer_begin(S, i == 0, vu, vv, s);

  EqJobs e1{};
  e1.count = 4;
  e1.bits[0] = sg; e1.point[0] = u; e1.scale[0] = &S->alpha; e1.out[0] = w.aU;
  e1.bits[1] = sg; e1.point[1] = v; e1.scale[1] = &S->beta; e1.out[1] = w.bV;
  e1.bits[2] = n; e1.point[2] = u + sg; e1.scale[2] = nullptr; e1.out[2] = w.Cu;
  e1.bits[3] = n; e1.point[3] = v + sg; e1.scale[3] = nullptr; e1.out[3] = w.Cv;
  launch_eq_tables(e1, s);

  // Phase 1: tables (and, for big tables, round 1 in the same pass), then the rounds.
  Tabs<3> ta;
  ta.src[0] = W; ta.src[1] = w.G; ta.src[2] = w.H;
  ta.dst[0] = w.Wf; ta.dst[1] = w.G; ta.dst[2] = w.H;
  const uint32_t off_vx = 24 * s1, off_p2 = off_vx + 8, off_vy = off_p2 + 24 * s1;
  if (s1 > tun.tail_log) {
    launch_phase1_init_round(W, w.G, w.H, c.wiring[i], w.aU, w.bV, w.Cu, w.Cv, n, 1ull << (s1 - 1),
                             1ull << c.s(i), S, w.partials, rx, proof, tun.max_round_blocks, s);
    run_phase<FormA>(ta, s1, S, w.partials, rx, proof, &S->vx, proof + off_vx, tun, s, 1);
  } else {
    launch_phase1_init(W, w.G, w.H, c.wiring[i], w.aU, w.bV, w.Cu, w.Cv, n, 1ull << s1,
                       1ull << c.s(i), s);
    run_phase<FormA>(ta, s1, S, w.partials, rx, proof, &S->vx, proof + off_vx, tun, s);
  }

  // Phase 2: sub-circuit rounds with the copy factors contracted, then the copy rounds.
  EqJobs e2{};
  e2.count = 2;
  e2.bits[0] = sg1; e2.point[0] = rx; e2.scale[0] = nullptr; e2.out[0] = w.EL;
  e2.bits[1] = n; e2.point[1] = rx + sg1; e2.scale[1] = nullptr; e2.out[1] = w.EC;
  launch_eq_tables(e2, s);
  launch_copy_weights(w.Cu, w.Cv, w.EC, w.U, w.V, 1ull << n, S, s);
  launch_phase2_tables(c.wiring[i], w.aU, w.bV, w.EL, S, w.Fa, w.Fb, w.Ka, w.Kb, w.Ks, 1ull << sg1,
                       1ull << sg, s);
  launch_copy_contract(W, w.U, w.V, w.P, w.Q, n, 1ull << sg1, s);
  Tabs<5> tb;
  tb.src[0] = w.P; tb.src[1] = w.Fa; tb.src[2] = w.Q; tb.src[3] = w.Fb; tb.src[4] = w.Ks;
  for (int k = 0; k < 5; ++k) tb.dst[k] = const_cast<Fr*>(tb.src[k]);
  run_phase<FormB>(tb, sg1, S, w.partials, ry, proof + off_p2, &S->scratch[1], nullptr, tun, s);

  EqJobs e3{};
  e3.count = 1;
  e3.bits[0] = sg1; e3.point[0] = ry; e3.scale[0] = nullptr; e3.out[0] = w.EqR;
  launch_eq_tables(e3, s);
  launch_local_values(w.EqR, w.Ka, w.Kb, 1ull << sg1, S, s);
  launch_local_contract(W, w.EqR, w.wpart, n, 1ull << sg1, c.plan.ychunks, s);
  launch_copy_tables(w.wpart, c.plan.ychunks, w.U, w.V, w.Fa, w.Fb, S, w.Wc, w.Fc, w.Kc, 1ull << n, s);
  Tabs<3> tc;
  tc.src[0] = w.Wc; tc.src[1] = w.Fc; tc.src[2] = w.Kc;
  tc.dst[0] = w.Wc; tc.dst[1] = w.Fc; tc.dst[2] = w.Kc;
  run_phase<FormA>(tc, n, S, w.partials, ry + sg1, proof + off_p2 + 24 * sg1, &S->vy,
                   proof + off_vy, tun, s);
}

// Forward evaluation of every layer from Montgomery inputs in layer[d].
static void run_forward(const gkr_circuit& c, const Workspace& w, hipStream_t s) {
  for (int i = (int)c.depth - 1; i >= 0; --i)
    launch_forward(w.layer[i + 1], w.layer[i], c.wiring[i].gates, c.n, 1ull << c.s(i),
                   (uint64_t)c.mul_gates[i] << c.n, s);
}

// g and the output claim V_0~(g) (into S->scratch[0]); needs layer[0] in Montgomery form.
static void run_output_claim(const gkr_circuit& c, const Workspace& w, hipStream_t s) {
  DevState* S = w.state;
  Fr* g = w.chal;
  launch_squeeze(S, g, c.s(0), s);
  EqJobs e{};
  e.count = 2;
  e.bits[0] = c.sigma[0]; e.point[0] = g; e.scale[0] = nullptr; e.out[0] = w.aU;
  e.bits[1] = c.n; e.point[1] = g + c.sigma[0]; e.scale[1] = nullptr; e.out[1] = w.Cu;
  launch_eq_tables(e, s);
  launch_weighted_sum(w.layer[0], w.aU, w.Cu, c.n, 1ull << c.s(0), w.partials, &S->counter,
                      &S->scratch[0], current_tuning().max_round_blocks, s);
}

static size_t layer_proof_words(const gkr_circuit& c, uint32_t i) { return (6ull * c.s(i + 1) + 2) * 8; }

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

static int32_t check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return GKR_EDEVICE;
  }
  return GKR_OK;
}

static int32_t check_ws(const gkr_circuit* c, void* ws, size_t ws_bytes) {
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
        rec[2 * z] = gl[z].x | (gl[z].type << 31);
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
        xent[2 * kx + 1] = gl[z].y | (gl[z].type << 31);
        yent[2 * ky] = (uint32_t)z;
        yent[2 * ky + 1] = gl[z].x | (gl[z].type << 31);
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
      delete c;
      set_error("device allocation of the wiring failed");
      return GKR_ENOMEM;
    }
    if (hipMemcpy(c->dev_block, host.data(), total, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      hipFree(c->dev_block);
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

void gkr_circuit_destroy(gkr_circuit* c) {
  if (!c) return;
  if (c->dev_block) hipFree(c->dev_block);
  delete c;
}

size_t gkr_workspace_bytes(const gkr_circuit* c) { return c ? c->plan.total : 0; }

size_t gkr_layer_proof_bytes(const gkr_circuit* c, uint32_t layer) {
  if (!c || layer >= c->depth) return 0;
  return layer_proof_words(*c, layer) * 4;
}

size_t gkr_proof_bytes(const gkr_circuit* c) {
  if (!c) return 0;
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
                            const gkr_fr* d_outputs, uint8_t* d_state, void* d_ws, size_t ws_bytes,
                            void* stream) {
  if (!c || !d_inputs || !d_outputs || !d_state || !aligned16(d_inputs) || !aligned16(d_outputs)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = bind_workspace(*c, d_ws);
  Words8 circ;
  memcpy(circ.w, c->digest, 32);
  run_digest(d_inputs, 1ull << c->s(c->depth), w.dig_in, w, s);
  run_digest(d_outputs, 1ull << c->s(0), w.dig_out, w, s);
  launch_transcript_begin(w.state, seed_state(seed), circ, w.dig_in, w.dig_out, s);
  launch_state_export(w.state, d_state, s);
  return check_launch();
}

int32_t gkr_output_claim(const gkr_circuit* c, const gkr_fr* d_outputs, uint8_t* d_state,
                         gkr_fr* d_g, gkr_fr* d_claim, void* d_ws, size_t ws_bytes, void* stream) {
  if (!c || !d_outputs || !d_state || !d_claim || (!d_g && c->s(0) > 0) || !aligned16(d_outputs) ||
      (d_g && !aligned16(d_g)) || !aligned16(d_claim)) {
    set_error("null or misaligned argument");
    return GKR_EINVAL;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = bind_workspace(*c, d_ws);
  launch_state_import(w.state, d_state, s);
  launch_to_mont(d_outputs, w.layer[0], 1ull << c->s(0), s);
  run_output_claim(*c, w, s);
  if (c->s(0) > 0) launch_from_mont(w.chal, d_g, c->s(0), s);
  launch_from_mont(&w.state->scratch[0], d_claim, 1, s);
  launch_state_export(w.state, d_state, s);
  return check_launch();
}

int32_t gkr_prove_layer(const gkr_circuit* c, uint32_t layer, const gkr_fr* d_next,
                        const gkr_fr* d_u, const gkr_fr* d_v, const gkr_fr* d_claim_u,
                        const gkr_fr* d_claim_v, uint8_t* d_state, gkr_fr* d_rx, gkr_fr* d_ry,
                        gkr_fr* d_vx, gkr_fr* d_vy, uint8_t* d_layer_proof, void* d_ws,
                        size_t ws_bytes, void* stream) {
  if (!c || layer >= c->depth) {
    set_error("bad circuit or layer");
    return GKR_EINVAL;
  }
  const bool first = layer == 0;
  const uint32_t si = c->s(layer), s1 = c->s(layer + 1);
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
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = bind_workspace(*c, d_ws);
  const uint32_t sc = chal_index_scratch(*c);
  const uint32_t smax = s_max_of(*c);
  Fr* u = w.chal + sc;
  Fr* v = u + smax;
  Fr* cl = v + smax;  // cl[0] = claim_u, cl[1] = claim_v
  launch_state_import(w.state, d_state, s);
  launch_to_mont(d_next, w.layer[layer + 1], 1ull << s1, s);
  if (si > 0) {
    launch_to_mont(d_u, u, si, s);
    launch_to_mont(first ? d_u : d_v, v, si, s);
  }
  launch_to_mont(d_claim_u, cl, 1, s);
  launch_to_mont(first ? d_claim_u : d_claim_v, cl + 1, 1, s);
  Fr* rx = w.chal + host_chal_index_rx(*c, layer);
  Fr* ry = w.chal + host_chal_index_ry(*c, layer);
  run_layer(*c, layer, w, w.layer[layer + 1], u, v, cl, cl + 1, rx, ry,
            reinterpret_cast<uint32_t*>(d_layer_proof), current_tuning(), s);
  if (s1 > 0) {
    launch_from_mont(rx, d_rx, s1, s);
    launch_from_mont(ry, d_ry, s1, s);
  }
  launch_from_mont(&w.state->vx, d_vx, 1, s);
  launch_from_mont(&w.state->vy, d_vy, 1, s);
  launch_state_export(w.state, d_state, s);
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
  const size_t need = gkr_proof_bytes(c);
  if (proof_len) *proof_len = need;
  if (proof_cap < need) {
    set_error("proof buffer too small: " + std::to_string(proof_cap) + " < " + std::to_string(need));
    return GKR_EBUFSZ;
  }
  int32_t rc = check_ws(c, d_ws, ws_bytes);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace w = bind_workspace(*c, d_ws);
  const Tuning tun = current_tuning();
  launch_to_mont(d_inputs, w.layer[c->depth], 1ull << c->s(c->depth), s);
  run_forward(*c, w, s);
  launch_from_mont(w.layer[0], d_outputs, 1ull << c->s(0), s);
  Words8 circ;
  memcpy(circ.w, c->digest, 32);
  run_digest(d_inputs, 1ull << c->s(c->depth), w.dig_in, w, s);
  run_digest(d_outputs, 1ull << c->s(0), w.dig_out, w, s);
  launch_transcript_begin(w.state, seed_state(seed), circ, w.dig_in, w.dig_out, s);
  run_output_claim(*c, w, s);
  uint32_t* proof = reinterpret_cast<uint32_t*>(d_proof);
  DevState* S = w.state;
  for (uint32_t i = 0; i < c->depth; ++i) {
    const Fr* u = (i == 0) ? w.chal : w.chal + host_chal_index_rx(*c, i - 1);
    const Fr* v = (i == 0) ? w.chal : w.chal + host_chal_index_ry(*c, i - 1);
    const Fr* vu = (i == 0) ? &S->scratch[0] : &S->vx;
    run_layer(*c, i, w, w.layer[i + 1], u, v, vu, &S->vy, w.chal + host_chal_index_rx(*c, i),
              w.chal + host_chal_index_ry(*c, i), proof, tun, s);
    proof += layer_proof_words(*c, i);
  }
  return check_launch();
}

}  // extern "C"
