// Host verifier of the GKR proofs (synchronous, no device work).
//
// Replays the transcript, checks g_j(0) + g_j(1) = claim for every round
// (Section 3.2.1), checks each layer's final claim against the wiring
// predicates, and finally evaluates the input MLE at both points itself.
//
// The predicates use the data-parallel structure: with
// T[z,c] = alpha eq(u,(z,c)) + beta eq(v,(z,c)),
//   mult~(rx, ry) = sum_{MUL z} sum_c T[z,c] eq(rx,(x_z,c)) eq(ry,(y_z,c))
//                 = sum_{MUL z} (alpha eqL(u,z) Cu + beta eqL(v,z) Cv) eqL(rx,x_z) eqL(ry,y_z)
// where Cu = prod_k (u_k rx_k ry_k + (1-u_k)(1-rx_k)(1-ry_k)) over the copy
// variables (and Cv likewise), so a layer costs O(2^sigma + n).
#include <string.h>

#include <algorithm>
#include <array>
#include <string>
#include <thread>
#include <vector>

#include "gkr_general.hpp"
#include "gkr_gl.hpp"
#include "gkr_internal.hpp"
#include "gkr_vpd.hpp"
#include "gl.hpp"

namespace gkr {
namespace {

Fr to_m(const Fr& a) { return fr_to_mont(a); }
Fr from_m(const Fr& a) { return fr_from_mont(a); }

std::vector<Fr> eq_table_host(const Fr* r, uint32_t k) {
  std::vector<Fr> t(1ull << k);
  t[0] = fr_one();
  for (uint32_t i = 0; i < k; ++i) {
    // append variable i as the new least significant bit
    const uint64_t cur = 1ull << i;
    const Fr ri = r[i], ni = fr_one_minus(r[i]);
    for (uint64_t b = cur; b-- > 0;) {
      const Fr v = t[b];
      t[2 * b + 1] = fr_mul(v, ri);
      t[2 * b] = fr_mul(v, ni);
    }
  }
  return t;
}

// V~(r) for V given as canonical host limbs (converted on the fly), by folding.
Fr mle_host(const gkr_fr* V, uint32_t k, const Fr* r) {
  const uint64_t size = 1ull << k;
  if (k == 0) return to_m(*reinterpret_cast<const Fr*>(&V[0]));
  // first fold reads the canonical vector; parallel over a few threads for big inputs
  std::vector<Fr> cur(size / 2);
  const uint64_t half = size / 2;
  const Fr r0 = r[0];
  unsigned nt = std::thread::hardware_concurrency();
  if (nt == 0) nt = 1;
  if (half < (1u << 16)) nt = 1;
  if (nt > 16) nt = 16;
  auto fold_first = [&](uint64_t b0, uint64_t b1) {
    for (uint64_t b = b0; b < b1; ++b) {
      const Fr a = to_m(*reinterpret_cast<const Fr*>(&V[b]));
      const Fr c = to_m(*reinterpret_cast<const Fr*>(&V[b + half]));
      cur[b] = fr_add(a, fr_mul(r0, fr_sub(c, a)));
    }
  };
  auto fold_next = [&](std::vector<Fr>& x, uint64_t h, const Fr& rj, uint64_t b0, uint64_t b1) {
    for (uint64_t b = b0; b < b1; ++b) x[b] = fr_add(x[b], fr_mul(rj, fr_sub(x[b + h], x[b])));
  };
  auto parallel = [&](uint64_t n, auto&& fn) {
    if (nt == 1 || n < (1u << 14)) {
      fn(0, n);
      return;
    }
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nt; ++t) th.emplace_back(fn, n * t / nt, n * (t + 1) / nt);
    for (auto& t : th) t.join();
  };
  parallel(half, fold_first);
  uint64_t m = half;
  for (uint32_t j = 1; j < k; ++j) {
    const uint64_t h = m / 2;
    const Fr rj = r[j];
    parallel(h, [&](uint64_t b0, uint64_t b1) { fold_next(cur, h, rj, b0, b1); });
    m = h;
  }
  return cur[0];
}

// Tree digest of canonical elements (same structure as the device kernels).
void tree_digest_host(const uint8_t* data, uint64_t nbytes, uint32_t out[8]) {
  const uint64_t chunk = (uint64_t)kChunkWords * 4;
  if (nbytes <= chunk) {
    sha256_bytes(data, nbytes, out);
    return;
  }
  const uint64_t nchunks = (nbytes + chunk - 1) / chunk;
  std::vector<uint8_t> level(nchunks * 32);
  for (uint64_t t = 0; t < nchunks; ++t) {
    const uint64_t b = t * chunk, e = (b + chunk < nbytes) ? b + chunk : nbytes;
    uint32_t h[8];
    sha256_bytes(data + b, e - b, h);
    for (int k = 0; k < 8; ++k) {
      level[32 * t + 4 * k + 0] = (uint8_t)(h[k] >> 24);
      level[32 * t + 4 * k + 1] = (uint8_t)(h[k] >> 16);
      level[32 * t + 4 * k + 2] = (uint8_t)(h[k] >> 8);
      level[32 * t + 4 * k + 3] = (uint8_t)h[k];
    }
  }
  tree_digest_host(level.data(), level.size(), out);
}

struct HostTranscript {
  Sha256State st;

  void absorb_words(uint32_t tag, const uint32_t* words, int nw) {
    std::vector<uint8_t> m;
    auto put = [&](uint32_t w) {
      m.push_back((uint8_t)(w >> 24));
      m.push_back((uint8_t)(w >> 16));
      m.push_back((uint8_t)(w >> 8));
      m.push_back((uint8_t)w);
    };
    for (int k = 0; k < 8; ++k) put(st.h[k]);
    put(tag);
    for (int k = 0; k < nw; ++k) put(words[k]);
    sha256_bytes(m.data(), m.size(), st.h);
  }
  void absorb_elements(uint32_t tag, const Fr* canon, int count) {
    std::vector<uint32_t> w;
    for (int i = 0; i < count; ++i)
      for (int k = 0; k < 8; ++k) w.push_back(bswap32(canon[i].v[k]));
    absorb_words(tag, w.data(), (int)w.size());
  }
  // The state as a challenge: rehash with "GKRC" until the 254-bit value v
  // is below p; the challenge is v * 2^-256 mod p (returned canonical).
  Fr accept() {
    Fr c = sha256_to_candidate(st);
    while (!fr_is_canonical(c)) {
      absorb_words(kTagChallenge, nullptr, 0);
      c = sha256_to_candidate(st);
    }
    return fr_from_mont(c);
  }
  Fr squeeze() {
    absorb_words(kTagChallenge, nullptr, 0);
    return accept();
  }
  // A round absorbs the values at t = 0 and t = 2 (e1 is fixed by the claim)
  // with one compression of the block LE(e0 2^256 mod p) || LE(e2 2^256 mod p + 2^254).
  Fr round_challenge(const Fr* e) {
    const Fr m0 = fr_to_mont(e[0]), m2 = fr_to_mont(e[2]);
    Sha256Block blk;
    for (int k = 0; k < 8; ++k) {
      blk.w[k] = bswap32(m0.v[k]);
      blk.w[8 + k] = bswap32(k == 7 ? (m2.v[k] | kRoundMark) : m2.v[k]);
    }
    st = sha256_compress_v(st, blk);
    return accept();
  }
};

Fr triple_eq(const Fr* a, const Fr* b, const Fr* c, uint32_t k) {
  Fr acc = fr_one();
  for (uint32_t i = 0; i < k; ++i) {
    const Fr t1 = fr_mul(fr_mul(a[i], b[i]), c[i]);
    const Fr t0 = fr_mul(fr_mul(fr_one_minus(a[i]), fr_one_minus(b[i])), fr_one_minus(c[i]));
    acc = fr_mul(acc, fr_add(t1, t0));
  }
  return acc;
}

bool canonical_all(const void* p, uint64_t count) {
  const Fr* f = static_cast<const Fr*>(p);
  for (uint64_t i = 0; i < count; ++i)
    if (!fr_is_canonical(f[i])) return false;
  return true;
}

}  // namespace

// ---------------------------------------------------------------- general circuits

namespace {

// A claim the verifier holds about a layer (values and points in Montgomery form).
struct HClaim {
  bool subset;
  std::vector<Fr> point;                 // eq: s_j entries; subset: tau + n entries
  Fr value;
  uint32_t tau;                          // subset: bits of the local part
  const std::vector<uint32_t>* used;     // subset: the used gates
};

// Local weights of a claim over a layer's sub-circuit, scaled by `coef`:
// eq: coef eq(point[:sigma], z); subset: coef eq(point[:tau], k) at z = used[k].
std::vector<Fr> claim_local(const HClaim& cl, uint32_t sigma, const Fr& coef) {
  std::vector<Fr> L;
  if (!cl.subset) {
    L = eq_table_host(cl.point.data(), sigma);
    for (Fr& v : L) v = fr_mul(v, coef);
  } else {
    L.assign(1ull << sigma, fr_zero());
    const std::vector<Fr> e = eq_table_host(cl.point.data(), cl.tau);
    for (size_t k = 0; k < cl.used->size(); ++k) L[(*cl.used)[k]] = fr_mul(e[k], coef);
  }
  return L;
}

const Fr* claim_copy_point(const HClaim& cl, uint32_t sigma) {
  return cl.point.data() + (cl.subset ? cl.tau : sigma);
}

}  // namespace

// The general-circuit verifier: the layered checks (rounds, final predicate,
// inputs) plus, per layer, the concatenation identity vy = sum_b eq(r_y[:beta],
// b) v_b, with every block value becoming a claim on its source layer. The
// predicates factor the copy bits as in the layered verifier: with local
// weights L_k and copy point c_k of claim k,
//   mult~ = sum_k triple(c_k, rx_copy, ry_copy) sum_{MUL} L_k[z] eqL(rx, x) eqL(ry, y').
int32_t general_verify(const gkr_circuit& c, const gkr_fr* inputs, const gkr_fr* outputs, uint64_t seed,
                       const uint8_t* proof, size_t proof_len) {
  const GeneralInfo& g = *c.general;
  const uint32_t d = c.depth, n = c.n;
  const size_t need = general_proof_bytes(c);
  if (proof_len != need) {
    set_error("proof length " + std::to_string(proof_len) + ", expected " + std::to_string(need));
    return GKR_EINVAL;
  }
  const uint64_t nin = 1ull << c.s(d), nout = 1ull << c.s(0);
  if (!canonical_all(inputs, nin) || !canonical_all(outputs, nout) || !canonical_all(proof, need / 32)) {
    set_error("element not canonical");
    return GKR_EINVAL;
  }
  const Fr* pf = reinterpret_cast<const Fr*>(proof);
  uint64_t pos = 0;
  HostTranscript tr;
  {
    uint8_t msg[19];
    memcpy(msg, "SISU-GKR-v1", 11);
    for (int k = 0; k < 8; ++k) msg[11 + k] = (uint8_t)(seed >> (8 * k));
    sha256_bytes(msg, sizeof(msg), tr.st.h);
  }
  uint32_t dig[8];
  tr.absorb_words(kTagDigest, c.digest, 8);
  tree_digest_host(reinterpret_cast<const uint8_t*>(inputs), nin * 32, dig);
  tr.absorb_words(kTagDigest, dig, 8);
  tree_digest_host(reinterpret_cast<const uint8_t*>(outputs), nout * 32, dig);
  tr.absorb_words(kTagDigest, dig, 8);

  std::vector<std::vector<HClaim>> pending(d + 1);
  {
    HClaim cl{false, std::vector<Fr>(c.s(0)), fr_zero(), 0, nullptr};
    for (auto& x : cl.point) x = to_m(tr.squeeze());
    cl.value = mle_host(outputs, c.s(0), cl.point.data());
    pending[0].push_back(cl);
  }
  bool accept = true;
  auto phase = [&](uint32_t rounds, Fr& claim, std::vector<Fr>& rs) {
    for (uint32_t j = 0; j < rounds; ++j) {
      const Fr* e = pf + pos;
      pos += 3;
      const Fr e0 = to_m(e[0]), e1 = to_m(e[1]), e2 = to_m(e[2]);
      if (!fr_eq(fr_add(e0, e1), claim)) accept = false;
      const Fr r = to_m(tr.round_challenge(e));
      rs.push_back(r);
      claim = fr_interp3(e0, e1, e2, r);
    }
  };
  for (uint32_t i = 0; i < d; ++i) {
    const GeneralLayer& L = g.layers[i];
    const std::vector<HClaim>& claims = pending[i];
    std::vector<Fr> coef(claims.size(), fr_one());
    if (i > 0)
      for (auto& a : coef) a = to_m(tr.squeeze());
    Fr claim = fr_zero();
    for (size_t k = 0; k < claims.size(); ++k) claim = fr_add(claim, fr_mul(coef[k], claims[k].value));
    const uint32_t s1 = c.s(i + 1), rho = g.rho(i), sg = c.sigma[i], sg1 = c.sigma[i + 1];
    std::vector<Fr> rx, ry;
    phase(s1, claim, rx);
    const Fr vx = to_m(pf[pos]);
    tr.absorb_elements(kTagValue, pf + pos, 1);
    ++pos;
    phase(rho, claim, ry);
    const Fr vy = to_m(pf[pos]);
    tr.absorb_elements(kTagValue, pf + pos, 1);
    ++pos;
    std::vector<Fr> vals;
    for (size_t b = 0; b < L.sources.size(); ++b) {
      vals.push_back(to_m(pf[pos]));
      tr.absorb_elements(kTagValue, pf + pos, 1);
      ++pos;
    }
    // concatenation identity
    {
      const std::vector<Fr> eb = eq_table_host(ry.data(), L.beta);
      Fr s = fr_zero();
      for (size_t b = 0; b < vals.size(); ++b) s = fr_add(s, fr_mul(eb[b], vals[b]));
      if (!fr_eq(s, vy)) accept = false;
    }
    // predicates: per-gate weight W[z] = sum_k triple_k L_k[z]
    std::vector<Fr> W(1ull << sg, fr_zero());
    for (size_t k = 0; k < claims.size(); ++k) {
      const std::vector<Fr> Lk = claim_local(claims[k], sg, coef[k]);
      const Fr t = triple_eq(claim_copy_point(claims[k], sg), rx.data() + sg1, ry.data() + rho - n, n);
      for (size_t z = 0; z < W.size(); ++z) W[z] = fr_add(W[z], fr_mul(t, Lk[z]));
    }
    const std::vector<Fr> elx = eq_table_host(rx.data(), sg1), ely = eq_table_host(ry.data(), rho - n);
    Fr add_v = fr_zero(), mul_v = fr_zero();
    for (const gkr_nested_gate& r : L.recs) {
      const size_t b = std::find(L.sources.begin(), L.sources.end(), r.src) - L.sources.begin();
      const std::vector<uint32_t>& u = L.used[b];
      const uint32_t k = (uint32_t)(std::lower_bound(u.begin(), u.end(), r.y) - u.begin());
      const uint32_t yl = ((uint32_t)b << L.tau) | k;
      const Fr term = fr_mul(fr_mul(W[r.z], elx[r.x]), ely[yl]);
      if (r.type == GKR_GATE_MUL) mul_v = fr_add(mul_v, term);
      else add_v = fr_add(add_v, term);
    }
    const Fr fin = fr_add(fr_mul(fr_mul(mul_v, vx), vy), fr_mul(add_v, fr_add(vx, vy)));
    if (!fr_eq(fin, claim)) accept = false;
    pending[i + 1].push_back(HClaim{false, rx, vx, 0, nullptr});
    for (size_t b = 0; b < L.sources.size(); ++b)
      pending[L.sources[b]].push_back(
          HClaim{true, std::vector<Fr>(ry.begin() + L.beta, ry.end()), vals[b], L.tau, &L.used[b]});
  }
  // the input layer: every claim straight from the inputs
  for (const HClaim& cl : pending[d]) {
    if (!accept) break;
    Fr want;
    if (!cl.subset) {
      want = mle_host(inputs, c.s(d), cl.point.data());
    } else {
      const std::vector<Fr> el = eq_table_host(cl.point.data(), cl.tau);
      const std::vector<Fr> ec = eq_table_host(cl.point.data() + cl.tau, n);
      want = fr_zero();
      for (size_t k = 0; k < cl.used->size(); ++k) {
        Fr s = fr_zero();
        for (uint64_t cp = 0; cp < (1ull << n); ++cp)
          s = fr_add(s, fr_mul(ec[cp], to_m(*reinterpret_cast<const Fr*>(&inputs[((uint64_t)(*cl.used)[k] << n) | cp]))));
        want = fr_add(want, fr_mul(el[k], s));
      }
    }
    if (!fr_eq(want, cl.value)) accept = false;
  }
  return accept ? 1 : 0;
}

// ---------------------------------------------------------------- Goldilocks

namespace {

std::vector<uint64_t> gl_eq_table_host(const uint64_t* r, uint32_t k) {
  std::vector<uint64_t> t(1ull << k);
  t[0] = 1;
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t cur = 1ull << i, ri = r[i], ni = gl_one_minus(r[i]);
    for (uint64_t b = cur; b-- > 0;) {
      const uint64_t v = t[b];
      t[2 * b + 1] = gl_mul(v, ri);
      t[2 * b] = gl_mul(v, ni);
    }
  }
  return t;
}

uint64_t gl_mle_host(const uint64_t* V, uint32_t k, const uint64_t* r) {
  if (k == 0) return V[0];
  std::vector<uint64_t> cur(V, V + (1ull << k));
  uint64_t m = 1ull << k;
  for (uint32_t j = 0; j < k; ++j) {
    const uint64_t h = m / 2;
    for (uint64_t b = 0; b < h; ++b) cur[b] = gl_add(cur[b], gl_mul(r[j], gl_sub(cur[b + h], cur[b])));
    m = h;
  }
  return cur[0];
}

uint64_t gl_triple_eq(const uint64_t* a, const uint64_t* b, const uint64_t* c, uint32_t k) {
  uint64_t acc = 1;
  for (uint32_t i = 0; i < k; ++i) {
    const uint64_t t1 = gl_mul(gl_mul(a[i], b[i]), c[i]);
    const uint64_t t0 = gl_mul(gl_mul(gl_one_minus(a[i]), gl_one_minus(b[i])), gl_one_minus(c[i]));
    acc = gl_mul(acc, gl_add(t1, t0));
  }
  return acc;
}

struct GlHostTranscript {
  HostTranscript t;
  uint64_t accept() {
    uint64_t v = (uint64_t)bswap32(t.st.h[0]) | ((uint64_t)bswap32(t.st.h[1]) << 32);
    while (v >= kGlP) {
      t.absorb_words(kTagChallenge, nullptr, 0);
      v = (uint64_t)bswap32(t.st.h[0]) | ((uint64_t)bswap32(t.st.h[1]) << 32);
    }
    return v;
  }
  uint64_t squeeze() {
    t.absorb_words(kTagChallenge, nullptr, 0);
    return accept();
  }
  void absorb_value(uint64_t v) {
    const uint32_t w[2] = {bswap32((uint32_t)v), bswap32((uint32_t)(v >> 32))};
    t.absorb_words(kTagValue, w, 2);
  }
  uint64_t round(uint64_t e0, uint64_t e2) {
    Sha256Block blk;
    for (int k = 0; k < 16; ++k) blk.w[k] = 0;
    blk.w[0] = bswap32((uint32_t)e0);
    blk.w[1] = bswap32((uint32_t)(e0 >> 32));
    blk.w[2] = bswap32((uint32_t)e2);
    blk.w[3] = bswap32((uint32_t)(e2 >> 32));
    blk.w[15] = 1u;
    t.st = sha256_compress_v(t.st, blk);
    return accept();
  }
};

}  // namespace
}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_gl_verify(const gkr_circuit* c, const uint64_t* inputs, const uint64_t* outputs,
                                 uint64_t seed, const uint8_t* proof, size_t proof_len) {
  try {
    if (!c || !inputs || !outputs || !proof) {
      set_error("null argument");
      return GKR_EINVAL;
    }
    if (c->field != GKR_FIELD_GOLDILOCKS) {
      set_error("gkr_gl_verify takes circuits created for the Goldilocks field");
      return GKR_EINVAL;
    }
    const uint32_t d = c->depth, n = c->n;
    const size_t need = gl_proof_bytes(*c);
    if (proof_len != need) {
      set_error("proof length " + std::to_string(proof_len) + ", expected " + std::to_string(need));
      return GKR_EINVAL;
    }
    const uint64_t nin = 1ull << c->s(d), nout = 1ull << c->s(0);
    const uint64_t* pf = reinterpret_cast<const uint64_t*>(proof);
    for (uint64_t i = 0; i < nin; ++i)
      if (inputs[i] >= kGlP) { set_error("element not canonical"); return GKR_EINVAL; }
    for (uint64_t i = 0; i < nout; ++i)
      if (outputs[i] >= kGlP) { set_error("element not canonical"); return GKR_EINVAL; }
    for (uint64_t i = 0; i < need / 8; ++i) {
      uint64_t v;
      memcpy(&v, proof + 8 * i, 8);
      if (v >= kGlP) { set_error("element not canonical"); return GKR_EINVAL; }
    }
    std::vector<uint64_t> pv(need / 8);
    memcpy(pv.data(), pf, need);
    uint64_t pos = 0;
    GlHostTranscript tr;
    {
      uint8_t msg[22];
      memcpy(msg, "SISU-GKR-GL-v1", 14);
      for (int k = 0; k < 8; ++k) msg[14 + k] = (uint8_t)(seed >> (8 * k));
      sha256_bytes(msg, sizeof(msg), tr.t.st.h);
    }
    uint32_t dig[8];
    tr.t.absorb_words(kTagDigest, c->digest, 8);
    tree_digest_host(reinterpret_cast<const uint8_t*>(inputs), nin * 8, dig);
    tr.t.absorb_words(kTagDigest, dig, 8);
    tree_digest_host(reinterpret_cast<const uint8_t*>(outputs), nout * 8, dig);
    tr.t.absorb_words(kTagDigest, dig, 8);
    std::vector<uint64_t> u(c->s(0)), v;
    for (auto& x : u) x = tr.squeeze();
    uint64_t vu = gl_mle_host(outputs, c->s(0), u.data()), vv = 0;
    bool accept = true;
    for (uint32_t i = 0; i < d; ++i) {
      uint64_t alpha = 1, beta = 0;
      if (i > 0) {
        alpha = tr.squeeze();
        beta = tr.squeeze();
      }
      uint64_t claim = gl_add(gl_mul(alpha, vu), gl_mul(beta, vv));
      const uint32_t s1 = c->s(i + 1), sg = c->sigma[i], sg1 = c->sigma[i + 1];
      std::vector<uint64_t> rxy[2];
      uint64_t vals[2];
      for (int ph = 0; ph < 2; ++ph) {
        for (uint32_t j = 0; j < s1; ++j) {
          const uint64_t e0 = pv[pos], e1 = pv[pos + 1], e2 = pv[pos + 2];
          pos += 3;
          if (gl_add(e0, e1) != claim) accept = false;
          const uint64_t r = tr.round(e0, e2);
          rxy[ph].push_back(r);
          claim = gl_interp3(e0, e1, e2, r);
        }
        vals[ph] = pv[pos++];
        tr.absorb_value(vals[ph]);
      }
      const std::vector<uint64_t>& rx = rxy[0];
      const std::vector<uint64_t>& ry = rxy[1];
      const std::vector<uint64_t> elx = gl_eq_table_host(rx.data(), sg1), ely = gl_eq_table_host(ry.data(), sg1);
      const std::vector<uint64_t> wu = gl_eq_table_host(u.data(), sg);
      const uint64_t cu = gl_triple_eq(u.data() + sg, rx.data() + sg1, ry.data() + sg1, n);
      std::vector<uint64_t> wv;
      uint64_t cv = 0;
      if (i > 0) {
        wv = gl_eq_table_host(v.data(), sg);
        cv = gl_triple_eq(v.data() + sg, rx.data() + sg1, ry.data() + sg1, n);
      }
      uint64_t add_v = 0, mul_v = 0;
      const std::vector<gkr_gate>& gl_ = c->gates[i];
      for (size_t z = 0; z < gl_.size(); ++z) {
        uint64_t wgt = gl_mul(gl_mul(alpha, wu[z]), cu);
        if (i > 0) wgt = gl_add(wgt, gl_mul(gl_mul(beta, wv[z]), cv));
        const uint64_t term = gl_mul(gl_mul(wgt, elx[gl_[z].x]), ely[gl_[z].y]);
        if (gl_[z].type == GKR_GATE_MUL) mul_v = gl_add(mul_v, term);
        else add_v = gl_add(add_v, term);
      }
      const uint64_t vx = vals[0], vy = vals[1];
      const uint64_t fin = gl_add(gl_mul(gl_mul(mul_v, vx), vy), gl_mul(add_v, gl_add(vx, vy)));
      if (fin != claim) accept = false;
      u = rx;
      v = ry;
      vu = vx;
      vv = vy;
    }
    if (accept) {
      if (vu != gl_mle_host(inputs, c->s(d), u.data())) accept = false;
      if (accept && vv != gl_mle_host(inputs, c->s(d), v.data())) accept = false;
    }
    return accept ? 1 : 0;
  } catch (...) {
    set_error("verifier failure (allocation)");
    return GKR_ENOMEM;
  }
}

namespace gkr {
namespace {

HostTranscript layered_statement(const gkr_circuit* c, uint64_t seed, const uint32_t input_digest[8],
                                 const gkr_fr* outputs) {
  HostTranscript tr;
  uint8_t msg[19];
  memcpy(msg, "SISU-GKR-v1", 11);
  for (int k = 0; k < 8; ++k) msg[11 + k] = (uint8_t)(seed >> (8 * k));
  sha256_bytes(msg, sizeof(msg), tr.st.h);
  uint32_t dig[8];
  tr.absorb_words(kTagDigest, c->digest, 8);
  tr.absorb_words(kTagDigest, input_digest, 8);
  tree_digest_host(reinterpret_cast<const uint8_t*>(outputs), (1ull << c->s(0)) * 32, dig);
  tr.absorb_words(kTagDigest, dig, 8);
  return tr;
}

// The layer-by-layer checks of a layered proof (pf: canonical elements),
// from the output claim down to the two claims on the input layer: false if
// a round check or a layer's final check fails. Leaves the input layer's
// points (Montgomery) in u, v and their claimed values in vu, vv.
bool verify_layers(const gkr_circuit* c, HostTranscript& tr, const gkr_fr* outputs, const Fr* pf,
                   std::vector<Fr>& u, std::vector<Fr>& v, Fr& vu, Fr& vv) {
  const uint32_t d = c->depth, n = c->n;
  uint64_t pos = 0;
  u.assign(c->s(0), fr_zero());
  v.clear();
  for (auto& x : u) x = to_m(tr.squeeze());
  vu = mle_host(outputs, c->s(0), u.data());
  vv = fr_zero();
  bool accept = true;
  for (uint32_t i = 0; i < d; ++i) {
    Fr alpha = fr_one(), beta = fr_zero();
    if (i > 0) {
      alpha = to_m(tr.squeeze());
      beta = to_m(tr.squeeze());
    }
    Fr claim = fr_add(fr_mul(alpha, vu), fr_mul(beta, vv));
    const uint32_t s1 = c->s(i + 1), sg = c->sigma[i], sg1 = c->sigma[i + 1];
    std::vector<Fr> rxy[2];
    Fr vals[2];
    for (int phase = 0; phase < 2; ++phase) {
      for (uint32_t j = 0; j < s1; ++j) {
        const Fr* e = pf + pos;
        pos += 3;
        const Fr e0 = to_m(e[0]), e1 = to_m(e[1]), e2 = to_m(e[2]);
        if (!fr_eq(fr_add(e0, e1), claim)) accept = false;
        const Fr r = to_m(tr.round_challenge(e));
        rxy[phase].push_back(r);
        claim = fr_interp3(e0, e1, e2, r);
      }
      vals[phase] = to_m(pf[pos]);
      tr.absorb_elements(kTagValue, pf + pos, 1);
      pos += 1;
    }
    const std::vector<Fr>& rx = rxy[0];
    const std::vector<Fr>& ry = rxy[1];
    // predicates
    const std::vector<Fr> elx = eq_table_host(rx.data(), sg1), ely = eq_table_host(ry.data(), sg1);
    const std::vector<Fr> wu = eq_table_host(u.data(), sg);
    const Fr cu = triple_eq(u.data() + sg, rx.data() + sg1, ry.data() + sg1, n);
    std::vector<Fr> wv;
    Fr cv = fr_zero();
    if (i > 0) {
      wv = eq_table_host(v.data(), sg);
      cv = triple_eq(v.data() + sg, rx.data() + sg1, ry.data() + sg1, n);
    }
    Fr add_v = fr_zero(), mul_v = fr_zero();
    const std::vector<gkr_gate>& gl = c->gates[i];
    for (size_t z = 0; z < gl.size(); ++z) {
      Fr wgt = fr_mul(fr_mul(alpha, wu[z]), cu);
      if (i > 0) wgt = fr_add(wgt, fr_mul(fr_mul(beta, wv[z]), cv));
      const Fr term = fr_mul(fr_mul(wgt, elx[gl[z].x]), ely[gl[z].y]);
      if (gl[z].type == GKR_GATE_MUL) mul_v = fr_add(mul_v, term);
      else add_v = fr_add(add_v, term);
    }
    const Fr vx = vals[0], vy = vals[1];
    const Fr fin = fr_add(fr_mul(fr_mul(mul_v, vx), vy), fr_mul(add_v, fr_add(vx, vy)));
    if (!fr_eq(fin, claim)) accept = false;
    u = rx;
    v = ry;
    vu = vx;
    vv = vy;
  }
  return accept;
}

// ---------------------------------------------------------------- committed inputs

Fr q_weight_tensor(const std::vector<Fr>& r, const std::vector<Fr>& ypow) {
  // prod_j ((1 - r_j) + r_j y^(2^(s-1-j)))
  const size_t s = r.size();
  Fr acc = fr_one();
  for (size_t j = 0; j < s; ++j) acc = fr_mul(acc, fr_add(fr_one_minus(r[j]), fr_mul(r[j], ypow[s - 1 - j])));
  return acc;
}

// q(x) = x^N Q(1/x) + (1 - x^N) Q(0), Q = Q_r1 + lam Q_r2 (Montgomery in and out).
Fr q_at_host(const std::vector<Fr>& r1, const std::vector<Fr>& r2, const Fr& lam, const Fr& x, Fr& xN) {
  const size_t s = r1.size();
  std::vector<Fr> ypow(s + 1), xpow(s + 1);
  ypow[0] = fr_inverse(x);
  xpow[0] = x;
  for (size_t k = 1; k <= s; ++k) {
    ypow[k] = fr_mul(ypow[k - 1], ypow[k - 1]);
    xpow[k] = fr_mul(xpow[k - 1], xpow[k - 1]);
  }
  xN = xpow[s];
  std::vector<Fr> zero(s + 1, fr_zero());
  const Fr qinv = fr_add(q_weight_tensor(r1, ypow), fr_mul(lam, q_weight_tensor(r2, ypow)));
  const Fr q0 = fr_add(q_weight_tensor(r1, zero), fr_mul(lam, q_weight_tensor(r2, zero)));
  return fr_add(fr_mul(xN, qinv), fr_mul(fr_one_minus(xN), q0));
}

uint32_t bitrev_host(uint64_t v, uint32_t bits) {
  uint64_t r = 0;
  for (uint32_t i = 0; i < bits; ++i) r |= ((v >> i) & 1) << (bits - 1 - i);
  return (uint32_t)r;
}

// The domain point at position t of a bit-reversed table over shift <w_m>.
Fr point_of_position(uint64_t t, uint32_t log_m, const Fr& shift) {
  return fr_mul(shift, fr_pow_u64(vpd_root_of_unity(log_m), bitrev_host(t, log_m)));
}

struct ByteReader {
  const uint8_t* p;
  size_t len, pos = 0;
  bool ok = true;
  void raw(uint8_t* out, size_t k) {
    if (pos + k > len) {
      ok = false;
      memset(out, 0, k);
      return;
    }
    memcpy(out, p + pos, k);
    pos += k;
  }
  // A canonical element (returned in Montgomery form); a non-canonical one fails the read.
  Fr element() {
    Fr a;
    raw(reinterpret_cast<uint8_t*>(a.v), 32);
    if (!fr_is_canonical(a)) {
      ok = false;
      return fr_zero();
    }
    return to_m(a);
  }
  // A digest as SHA-256 words (the bytes are big-endian words).
  void digest(uint32_t w[8]) {
    uint8_t b[32];
    raw(b, 32);
    for (int k = 0; k < 8; ++k)
      w[k] = ((uint32_t)b[4 * k] << 24) | ((uint32_t)b[4 * k + 1] << 16) | ((uint32_t)b[4 * k + 2] << 8) | b[4 * k + 3];
  }
};

Sha256Block pair_block_host(const Fr& a, const Fr& b) {
  Sha256Block blk;
  for (int k = 0; k < 8; ++k) {
    blk.w[k] = bswap32(a.v[k]);
    blk.w[8 + k] = bswap32(b.v[k]);
  }
  return blk;
}

// Root from a leaf digest and its bottom-up path.
void root_from_path(Sha256State h, uint64_t u, ByteReader& rd, uint32_t depth, uint32_t out[8]) {
  for (uint32_t lv = 0; lv < depth; ++lv) {
    uint32_t sib[8];
    rd.digest(sib);
    Sha256Block blk;
    for (int k = 0; k < 8; ++k) {
      blk.w[k] = (u & 1) ? sib[k] : h.h[k];
      blk.w[8 + k] = (u & 1) ? h.h[k] : sib[k];
    }
    h = sha256_compress_v(sha256_iv(), blk);
    u >>= 1;
  }
  for (int k = 0; k < 8; ++k) out[k] = h.h[k];
}

bool same_words(const uint32_t* a, const uint32_t* b) {
  for (int k = 0; k < 8; ++k)
    if (a[k] != b[k]) return false;
  return true;
}

// Fold of a pair (R(x), R(-x)) by beta: (a + b) / 2 + beta (a - b) / (2x).
Fr fold_pair(const Fr& a, const Fr& b, const Fr& beta, const Fr& x) {
  const Fr inv2 = fr_inv2();
  return fr_add(fr_mul(fr_add(a, b), inv2), fr_mul(fr_mul(fr_mul(beta, fr_sub(a, b)), inv2), fr_inverse(x)));
}

// The opening of the commitment root_f at (r1, r2) with claims (c1, c2), all
// Montgomery; continues the transcript.
bool verify_opening(const uint32_t root_f[8], uint32_t s, const std::vector<Fr>& r1, const std::vector<Fr>& r2,
                    const Fr& c1, const Fr& c2, HostTranscript& tr, ByteReader& rd, uint32_t queries) {
  const uint32_t logM = s + kVpdLogBlowup, d0 = logM - 1;
  const uint64_t M = 1ull << logM;
  const Fr lam = to_m(tr.squeeze());
  const Fr c = fr_add(c1, fr_mul(lam, c2));
  uint32_t root_hg[8];
  rd.digest(root_hg);
  tr.absorb_words(kTagCommit, root_hg, 8);
  Fr a[4];
  for (auto& x : a) x = to_m(tr.squeeze());
  std::vector<Fr> betas(s);
  std::vector<std::array<uint32_t, 8>> roots(s > 0 ? s - 1 : 0);
  for (uint32_t i = 0; i < s; ++i) {
    betas[i] = to_m(tr.squeeze());
    if (i + 1 < s) {
      rd.digest(roots[i].data());
      tr.absorb_words(kTagCommit, roots[i].data(), 8);
    }
  }
  const Fr fin = rd.element();
  {
    const Fr canon = from_m(fin);
    tr.absorb_elements(kTagValue, &canon, 1);
  }
  bool ok = rd.ok;
  const Fr shift = vpd_shift();
  for (uint32_t q = 0; q < queries && ok; ++q) {
    const uint64_t u = tr.squeeze().v[0] & (M / 2 - 1);  // the canonical challenge mod M / 2
    const Fr f0 = rd.element(), f1 = rd.element();
    uint32_t rt[8];
    root_from_path(sha256_compress_v(sha256_iv(), pair_block_host(f0, f1)), u, rd, d0, rt);
    ok = ok && same_words(rt, root_f);
    Fr hg[4];
    for (auto& x : hg) x = rd.element();
    Sha256State lh = sha256_compress_v(sha256_iv(), pair_block_host(hg[0], hg[1]));
    lh = sha256_compress_v(lh, pair_block_host(hg[2], hg[3]));
    root_from_path(lh, u, rd, d0, rt);
    ok = ok && same_words(rt, root_hg);
    const Fr x = point_of_position(2 * u, logM, shift);
    Fr pair[2];
    for (int side = 0; side < 2; ++side) {
      const Fr xx = side ? fr_neg(x) : x;
      const Fr fx = side ? f1 : f0, hx = hg[side], gx = hg[2 + side];
      Fr xN;
      const Fr qx = q_at_host(r1, r2, lam, xx, xN);
      const Fr lhs = fr_mul(fx, qx);
      const Fr rhs = fr_add(fr_add(c, fr_mul(xx, gx)), fr_mul(fr_sub(xN, fr_one()), hx));
      ok = ok && fr_eq(lhs, rhs);
      pair[side] = fr_add(fr_add(fr_mul(a[0], fx), fr_mul(a[1], hx)),
                          fr_mul(side ? fr_sub(a[2], fr_mul(a[3], x)) : fr_add(a[2], fr_mul(a[3], x)), gx));
    }
    Fr cur = fold_pair(pair[0], pair[1], betas[0], x);
    uint64_t pos = u;
    Fr sh = fr_mul(shift, shift);
    for (uint32_t i = 1; i < s; ++i) {
      const Fr v0 = rd.element(), v1 = rd.element();
      const uint64_t leaf = pos >> 1;
      root_from_path(sha256_compress_v(sha256_iv(), pair_block_host(v0, v1)), leaf, rd, d0 - i, rt);
      ok = ok && same_words(rt, roots[i - 1].data());
      ok = ok && fr_eq((pos & 1) ? v1 : v0, cur);
      cur = fold_pair(v0, v1, betas[i], point_of_position(2 * leaf, logM - i, sh));
      pos = leaf;
      sh = fr_mul(sh, sh);
    }
    ok = ok && fr_eq(cur, fin) && rd.ok;
  }
  return ok && rd.ok && rd.pos == rd.len;
}

}  // namespace
}  // namespace gkr

extern "C" int32_t gkr_verify(const gkr_circuit* c, const gkr_fr* inputs, const gkr_fr* outputs,
                              uint64_t seed, const uint8_t* proof, size_t proof_len) {
  try {
    if (!c || !inputs || !outputs || !proof) {
      set_error("null argument");
      return GKR_EINVAL;
    }
    if (c->general) return general_verify(*c, inputs, outputs, seed, proof, proof_len);
    if (c->field != GKR_FIELD_BN254) {
      set_error("this circuit is over the Goldilocks field: use gkr_gl_verify");
      return GKR_EINVAL;
    }
    const uint32_t d = c->depth;
    size_t need = 0;
    for (uint32_t i = 0; i < d; ++i) need += (6ull * c->s(i + 1) + 2) * 32;
    if (proof_len != need) {
      set_error("proof length " + std::to_string(proof_len) + ", expected " + std::to_string(need));
      return GKR_EINVAL;
    }
    const uint64_t nin = 1ull << c->s(d), nout = 1ull << c->s(0);
    if (!canonical_all(inputs, nin) || !canonical_all(outputs, nout) || !canonical_all(proof, need / 32)) {
      set_error("element not canonical");
      return GKR_EINVAL;
    }
    uint32_t dig[8];
    tree_digest_host(reinterpret_cast<const uint8_t*>(inputs), nin * 32, dig);
    HostTranscript tr = layered_statement(c, seed, dig, outputs);
    std::vector<Fr> u, v;
    Fr vu, vv;
    bool accept = verify_layers(c, tr, outputs, reinterpret_cast<const Fr*>(proof), u, v, vu, vv);
    if (accept) {
      if (!fr_eq(vu, mle_host(inputs, c->s(d), u.data()))) accept = false;
      if (accept && !fr_eq(vv, mle_host(inputs, c->s(d), v.data()))) accept = false;
    }
    return accept ? 1 : 0;
  } catch (...) {
    set_error("verifier failure (allocation)");
    return GKR_ENOMEM;
  }
}

extern "C" int32_t gkr_verify_committed(const gkr_circuit* c, const gkr_fr* outputs, uint64_t seed, uint32_t queries,
                                        const uint8_t* proof, size_t proof_len) {
  try {
    if (!c || !outputs || !proof) {
      set_error("null argument");
      return GKR_EINVAL;
    }
    size_t need = 0;
    if (int32_t rc = gkr_committed_sizes(c, queries, nullptr, &need)) return rc;
    if (proof_len != need) {
      set_error("proof length " + std::to_string(proof_len) + ", expected " + std::to_string(need));
      return GKR_EINVAL;
    }
    const uint32_t d = c->depth;
    size_t gkr_len = 0;
    for (uint32_t i = 0; i < d; ++i) gkr_len += (6ull * c->s(i + 1) + 2) * 32;
    if (!canonical_all(outputs, 1ull << c->s(0)) || !canonical_all(proof + 32, gkr_len / 32)) {
      set_error("element not canonical");
      return GKR_EINVAL;
    }
    ByteReader head{proof, 32};
    uint32_t root[8];
    head.digest(root);
    HostTranscript tr = layered_statement(c, seed, root, outputs);
    std::vector<Fr> u, v;
    Fr vu, vv;
    const bool layers_ok = verify_layers(c, tr, outputs, reinterpret_cast<const Fr*>(proof + 32), u, v, vu, vv);
    ByteReader rd{proof + 32 + gkr_len, proof_len - 32 - gkr_len};
    const bool open_ok = verify_opening(root, c->s(d), u, v, vu, vv, tr, rd, queries);
    return (layers_ok && open_ok) ? 1 : 0;
  } catch (...) {
    set_error("verifier failure (allocation)");
    return GKR_ENOMEM;
  }
}

