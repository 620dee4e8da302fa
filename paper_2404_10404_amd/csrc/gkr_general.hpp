// Host-side description of general circuits (accumulation gates, right inputs
// from any later layer) and the entry points of their proof program
// (gkr_general.hip) and verifier (gkr_verify.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "gkr_internal.hpp"

namespace gkr {

// A gate layer receives at most this many claims (the eq claim of the layer
// above and one claim per earlier layer that reads it).
constexpr uint32_t kGeneralMaxClaims = 14;

struct GeneralLayer {
  std::vector<gkr_nested_gate> recs;         // the nested gates, as given
  std::vector<uint32_t> sources;             // right-input layers, increasing (block b = sources[b])
  std::vector<std::vector<uint32_t>> used;   // per block: the used gates of that layer, increasing
  uint32_t beta = 0, tau = 0;                // block bits, bits of the largest used set
  uint64_t mul_recs = 0;
  // device indexes (inside the circuit's device block)
  const uint32_t* zrow = nullptr;  // CSR by output gate z: (x | type << 31, y')
  const uint2* zent = nullptr;
  const uint32_t* xrow = nullptr;  // CSR by left input x: (z, y' | type << 31)
  const uint2* xent = nullptr;
  const uint32_t* yrow = nullptr;  // CSR by right index y': (z, x | type << 31)
  const uint2* yent = nullptr;
  std::vector<const uint32_t*> used_dev;  // per block: the used gates
  std::vector<const uint32_t*> pos_dev;   // per block: position in the used set of each gate of the
                                          // source layer's sub-circuit (~0 when unused)
};

// A claim on a layer: made by layer h (h = -1: the output claim V_0~(g)); b = -1
// for the eq claim of h's phase 1 (point r_x of h), else the value of h's
// source block b (point: the local part of r_y of h, weights on the used set).
struct ClaimRef {
  int h, b;
};

struct GeneralInfo {
  uint32_t n = 0;
  std::vector<GeneralLayer> layers;
  std::vector<std::vector<ClaimRef>> claims;  // [layer], in the order they were produced
  // workspace layout (offsets in bytes) and index tables into the challenge,
  // coefficient and value areas
  std::vector<size_t> off_R;
  size_t off_T = 0, off_L = 0, off_C = 0, off_EqL = 0, off_EqC = 0, off_EL = 0, off_EC = 0;
  size_t off_coef = 0, off_vals = 0;
  std::vector<size_t> coef_index, val_index, rx_index, ry_index;
  uint32_t kmax = 1;
  uint32_t rho(uint32_t i) const { return layers[i].beta + layers[i].tau + n; }
};

struct Program;
struct Tuning;

// Shared emission (gkr_api.hip): one FormA phase (rounds, then the tail), and
// the statement binding followed by the output point and claim.
void emit_phase_a(Program& pg, const Fr* const* src0, Fr* const* dst, uint32_t nrounds, DevState* S, Fr* partials,
                  Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value, const Tuning& tun);
void emit_statement_and_output_claim(Program& pg, const gkr_circuit& c, const Workspace& w, const gkr_fr* d_inputs,
                                     const gkr_fr* d_outputs, uint64_t seed, const Tuning& tun);

// The proof of a general circuit (forward evaluation, statement, every layer).
void emit_prove_general(Program& pg, const gkr_circuit& c, void* d_ws, const gkr_fr* d_inputs, uint64_t seed,
                        gkr_fr* d_outputs, uint8_t* d_proof, const Tuning& tun);
void launch_general_step(const Step& st, hipStream_t s);

// Host verifier of a general circuit's proof (1 accept, 0 reject, < 0 error).
int32_t general_verify(const gkr_circuit& c, const gkr_fr* inputs, const gkr_fr* outputs, uint64_t seed,
                       const uint8_t* proof, size_t proof_len);

}  // namespace gkr
