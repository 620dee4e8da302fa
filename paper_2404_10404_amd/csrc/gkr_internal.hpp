// Internal declarations shared by the device kernels, the host driver and the
// host verifier of the GKR prover library.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gkr.h"
#include "fr.hpp"
#include "sha256.hpp"

namespace gkr {

constexpr int kBlock = 256;             // threads per workgroup (grid-wide kernels, batch kernel)
constexpr int kTailBlock = 512;         // threads of the single-workgroup tail kernels
constexpr uint32_t kMaxRoundBlocks = 4096;  // cap on workgroups of a reduction launch
constexpr int kMaxPartialValues = 2;    // reduced values per workgroup
constexpr uint32_t kChunkWords = 256;   // 1 KiB SHA-256 leaf chunk of a tree digest

// Transcript tags as big-endian words ("GKRD", "GKRV", "GKRC").
constexpr uint32_t kTagDigest = 0x474B5244u;
constexpr uint32_t kTagValue = 0x474B5256u;
constexpr uint32_t kTagChallenge = 0x474B5243u;
// A round message is absorbed as one compression block holding the
// Montgomery forms of e0 and e2 (little-endian), with bit 254 of the second
// (bit 30 of its top limb) set; both are below p < 2^254.
constexpr uint32_t kRoundMark = 1u << 30;

// Gate-layer wiring on the device. Gate records pack the type into bit 31.
struct LayerWiring {
  const uint2* gates;   // [2^{sigma_i}]      .x = x | type<<31, .y = y
  const uint32_t* xrow; // [2^{sigma_{i+1}}+1] CSR of gates by x
  const uint2* xent;    // [2^{sigma_i}]      .x = z, .y = y | type<<31
  const uint32_t* yrow; // [2^{sigma_{i+1}}+1] CSR of gates by y
  const uint2* yent;    // [2^{sigma_i}]      .x = z, .y = x | type<<31
};

// Scalars of one proof in device memory (all field values in Montgomery form).
struct DevState {
  uint32_t st[8];   // transcript chaining value, SHA-256 words h[0..7]
  uint32_t counter; // last-workgroup counter of grid reductions (returns to 0)
  uint32_t pending; // 1: the claim has not yet moved through the last round
  uint32_t pad1;
  uint32_t* pend_msg;  // where that round's message goes
  uint32_t pad[3];
  Fr claim;         // running sumcheck claim (before the pending round, if any)
  Fr pend_e0, pend_e2, pend_r;  // the pending round: its sums at t = 0, 2 and its challenge
  Fr alpha, beta;
  Fr vx, vy;
  Fr su, sv;        // sum_c U[c], sum_c V[c]
  Fr ka_f, kb_f;    // Ka~, Kb~ at the phase-2 local point
  Fr scratch[4];
};

// One step of a proof program: a kernel body over `ntiles` workgroups.
// The host driver records a proof as a sequence of steps; the plain executor
// launches one kernel per step and the persistent batch kernel runs the steps
// of many proofs. Parameters are typed by `type` (see gkr_kernels.hip).
enum StepType : uint32_t {
  ST_TO_MONT = 0,
  ST_FROM_MONT,
  ST_FORWARD,
  ST_DIGEST,
  ST_TRANSCRIPT_BEGIN,
  ST_SQUEEZE,
  ST_LAYER_BEGIN,
  ST_EQ,
  ST_WSUM,
  ST_P1_INIT,
  ST_P1_INIT_ROUND,
  ST_ROUND_A,
  ST_ROUND_B,
  ST_TAIL_A,
  ST_TAIL_B,
  ST_COPY_WEIGHTS,
  ST_P2_TABLES,
  ST_COPY_CONTRACT,
  ST_LOCAL_CONTRACT,
  ST_COPY_TABLES,
  ST_LOCAL_VALUES,
  ST_STATE_EXPORT,
  ST_STATE_IMPORT,
  ST_COUNT,
  // General circuits (accumulation gates, right inputs from any later layer):
  // launched by launch_general_step, plain path only.
  ST_G_GATHER = 64,
  ST_G_FORWARD,
  ST_G_SCATTER,
  ST_G_TTABLE,
  ST_G_P1,
  ST_G_P2,
  ST_G_LAYER_BEGIN,
  ST_G_VALUES,
  ST_G_END,
  // The Goldilocks-field prover: launched by launch_gl_step, plain path only.
  ST_GL_FORWARD = 96,
  ST_GL_DIGEST,
  ST_GL_BEGIN,
  ST_GL_SQUEEZE,
  ST_GL_LAYER_BEGIN,
  ST_GL_EQ,
  ST_GL_WSUM,
  ST_GL_P1,
  ST_GL_ROUND,
  ST_GL_TAIL,
  ST_GL_ROUND5,
  ST_GL_TAIL5,
  ST_GL_COPY_WEIGHTS,
  ST_GL_P2T,
  ST_GL_COPY_CONTRACT,
  ST_GL_LOCAL_VALUES,
  ST_GL_LOCAL_CONTRACT,
  ST_GL_COPY_TABLES,
  ST_GL_END,
  // The commitment to the input layer and its opening: launched by
  // launch_vpd_step, plain path only.
  ST_VPD_POWERS = 128,
  ST_VPD_TWIDDLES,
  ST_VPD_SCALE,
  ST_VPD_NTT,
  ST_VPD_MUL,
  ST_VPD_LEAVES,
  ST_VPD_NODES,
  ST_VPD_TREE_TOP,
  ST_VPD_BEGIN,
  ST_VPD_ABSORB,
  ST_VPD_ROOT_OUT,
  ST_VPD_FOLD0,
  ST_VPD_FOLD,
  ST_VPD_FINAL,
  ST_VPD_QUERIES,
  ST_VPD_END,
  // The copy contraction on the matrix cores: launched by launch_cc_step,
  // plain path only.
  ST_CC_BUILD = 192,
  ST_CC_BSUM,
  ST_CC_GEMM,
  ST_CC_EPILOGUE
};

struct Step {
  uint32_t type;
  uint32_t ntiles;   // workgroups
  uint32_t u[6];     // small integers
  uint64_t q[4];     // sizes
  const void* p[16]; // device pointers
  uint32_t w[16];    // host words (seed state, circuit digest)
  double bytes;      // algorithmic HBM bytes (timing reports only)
  double mulmods;    // field products (timing reports only)
};

// Tunables of the round schedule (autotuned; see gkr_tuning.*).
struct Tuning {
  uint32_t tail_log;          // single-workgroup tail once a table has <= 2^tail_log entries
  uint32_t max_round_blocks;  // cap on the workgroups of a grid-wide round
  uint32_t pairs_per_thread;  // a grid-wide round gives each thread at least this many pairs
  uint32_t matrix_cores;      // 1: the phase-2 copy contraction on the int8 matrix cores where it applies
};

// Device buffers of one proof, carved out of the caller's workspace.
struct Workspace {
  Fr* layer[GKR_MAX_DEPTH + 1];  // only [0..d] used
  Fr *G, *H, *Wf;
  Fr *aU, *bV, *Cu, *Cv, *U, *V, *EC, *EL, *EqR;
  Fr *P, *Q, *Fa, *Fb, *Ks, *Ka, *Kb;
  Fr *Wc, *Fc, *Kc, *wpart;
  Fr* partials;
  void* cc;                 // matrix-core contraction scratch (null if no layer uses it)
  uint32_t *dig_a, *dig_b;  // tree-digest levels (8 words per digest)
  uint32_t* dig_in;         // final digests (8 words each)
  uint32_t* dig_out;
  Fr* chal;                 // g, then rx/ry of every layer
  DevState* state;
  size_t bytes;
};

// Host-side description of the workspace layout of a circuit.
struct Plan {
  size_t off_layer[GKR_MAX_DEPTH + 1];
  size_t off_G, off_H, off_Wf, off_aU, off_bV, off_Cu, off_Cv, off_U, off_V, off_EC, off_EL,
      off_EqR, off_P, off_Q, off_Fa, off_Fb, off_Ks, off_Ka, off_Kb, off_Wc, off_Fc, off_Kc,
      off_wpart, off_partials, off_dig_a, off_dig_b, off_dig_in, off_dig_out, off_chal, off_state, off_cc;
  size_t cc_bytes;
  size_t total;
  uint32_t ychunks;  // y-range split of the phase-2 copy-table pass
  size_t dig_level_words;
};

}  // namespace gkr

namespace gkr {
struct GeneralInfo;  // general circuits only (gkr_general.hip)

// Scalars of one Goldilocks proof in device memory (canonical 64-bit elements).
struct GlState {
  uint32_t st[8];   // transcript chaining value, SHA-256 words h[0..7]
  uint32_t counter; // last-workgroup counter of grid reductions (returns to 0)
  uint32_t pad;
  uint64_t claim, alpha, beta, vx, vy;
  uint64_t su, sv;      // sum_c U[c], sum_c V[c] (phase 2)
  uint64_t ka_f, kb_f;  // Ka~, Kb~ at the phase-2 local point
  uint64_t scratch[4];  // [0] the output claim V_0~(g)
};

// Workspace layout of a Goldilocks proof: layers 1..d-1 (layer d is the
// caller's inputs, layer 0 the caller's outputs), tables, state.
struct GlPlan {
  size_t off_layer[GKR_MAX_DEPTH + 1];
  size_t off_G, off_H, off_Wf, off_aU, off_bV, off_Cu, off_Cv, off_EL, off_EC, off_partials, off_dig_a,
      off_dig_b, off_dig_in, off_dig_out, off_chal, off_state;
  // phase 2 with the copy factors contracted
  size_t off_U, off_V, off_P, off_Q, off_Fa, off_Fb, off_Ka, off_Kb, off_Ks, off_EqR, off_Wc, off_Fc, off_Kc,
      off_wpart;
};
}  // namespace gkr

struct gkr_circuit {
  uint32_t depth = 0, n = 0;
  gkr::GeneralInfo* general = nullptr;        // non-null for a general circuit
  uint32_t field = GKR_FIELD_BN254;           // GKR_FIELD_GOLDILOCKS: proved by gkr_gl_prove_circuit
  gkr::GlPlan gl;                             // Goldilocks workspace layout
  ~gkr_circuit();                             // frees the device block and the general description
  std::vector<uint32_t> sigma;                // [depth+1]
  std::vector<std::vector<gkr_gate>> gates;   // host copy of each layer's sub-circuit
  std::vector<uint64_t> mul_gates;            // MUL gates of each layer's sub-circuit
  uint32_t digest[8];                         // circuit digest, SHA-256 words
  int device = 0;
  void* dev_block = nullptr;
  std::vector<gkr::LayerWiring> wiring;       // device pointers into dev_block
  gkr::Plan plan;
  uint32_t s(uint32_t i) const { return sigma[i] + n; }
};

namespace gkr {

void set_error(const std::string& msg);
size_t plan_workspace(const gkr_circuit& c, Plan& p);
// General circuits (gkr_general.hip, gkr_general_verify.cpp).
void general_destroy(GeneralInfo* g);
size_t general_proof_bytes(const gkr_circuit& c);
size_t general_layer_proof_bytes(const gkr_circuit& c, uint32_t layer);
Workspace bind_workspace(const gkr_circuit& c, void* base);
uint32_t host_chal_index_rx(const gkr_circuit& c, uint32_t layer);  // index of rx[0] of a layer in chal
uint32_t host_chal_index_ry(const gkr_circuit& c, uint32_t layer);

// Host SHA-256 of a byte string (used for the transcript seed and the circuit digest).
void sha256_bytes(const uint8_t* data, size_t len, uint32_t out_words[8]);

}  // namespace gkr
