// Proof programs: the host records a proof as a sequence of steps, which the
// plain path launches one kernel per step and the batch kernel runs for many
// proofs at once.
#pragma once

#include <vector>

#include "gkr_internal.hpp"
#include "gkr_kernels.hpp"

namespace gkr {

struct Program {
  std::vector<Step> steps;
  // Steps that only the plain launcher runs (the matrix-core contraction) are
  // allowed; the batch kernel's programs switch this off.
  bool matrix_cores = true;

  void to_mont(const gkr_fr* in, Fr* out, uint64_t n);
  void from_mont(const Fr* in, gkr_fr* out, uint64_t n);
  void forward(const Fr* W, Fr* V, const uint2* gates, uint32_t n, uint64_t count, uint64_t mul_gates);
  void digest(const gkr_fr* vec, uint64_t nelem, uint32_t* final_out, const Workspace& w);
  void transcript_begin(DevState* S, const Words8& seed_state, const uint32_t* circ, const uint32_t* din,
                        const uint32_t* dout);
  void squeeze(DevState* S, Fr* out, uint32_t count);
  void layer_begin(DevState* S, bool first, const Fr* vu, const Fr* vv);
  void eq(int count, const uint32_t* bits, const Fr* const* points, const Fr* const* scales, Fr* const* outs);
  void wsum(const Fr* V, const Fr* A, const Fr* B, uint32_t n, uint64_t count, Fr* partials, DevState* S,
            Fr* dst, const Tuning& tun);
  void p1_init(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU, const Fr* bV, const Fr* Cu,
               const Fr* Cv, uint32_t n, uint64_t count, uint64_t gates);
  void p1_init_round(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU, const Fr* bV,
                     const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t half, uint64_t gates, DevState* S,
                     Fr* partials, Fr* r_out, uint32_t* msg, const Tuning& tun);
  template <int NT>
  void round(const Fr* const* src, Fr* const* dst, uint64_t half, const Fr* rprev, DevState* S, Fr* partials,
             Fr* r_out, uint32_t* msg, const Tuning& tun);
  template <int NT>
  void tail(const Fr* const* src, Fr* const* dst, uint64_t size, const Fr* rpending, uint32_t rounds,
            DevState* S, Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value);
  void copy_weights(const Fr* Cu, const Fr* Cv, const Fr* EC, Fr* U, Fr* V, uint64_t ncop, DevState* S);
  void p2_tables(const LayerWiring& lw, const Fr* aU, const Fr* bV, const Fr* EL, const DevState* S, Fr* Fa,
                 Fr* Fb, Fr* Ka, Fr* Kb, Fr* Ks, uint64_t count, uint64_t gates);
  void copy_contract(const Fr* W, const Fr* U, const Fr* V, Fr* Pt, Fr* Qt, uint32_t n, uint64_t rows);
  void local_contract(const Fr* W, const Fr* EqR, Fr* part, uint32_t n, uint64_t rows, uint32_t R);
  void copy_tables(const Fr* part, uint32_t R, const Fr* U, const Fr* V, const Fr* fa_f, const Fr* fb_f,
                   const DevState* S, Fr* Wc, Fr* Fc, Fr* Kc, uint64_t ncop);
  void local_values(const Fr* EqR, const Fr* Ka, const Fr* Kb, uint64_t rows, DevState* S, Fr* partials);
  void state_export(const DevState* S, uint8_t* out);
  void state_import(DevState* S, const uint8_t* in);

  // Launch every step as its own kernel, in order, on stream s.
  void run(hipStream_t s) const;
};

void emit_layer(Program& pg, const gkr_circuit& c, uint32_t i, const Workspace& w, const Fr* W, const Fr* u,
                const Fr* v, const Fr* vu, const Fr* vv, Fr* rx, Fr* ry, uint32_t* proof, const Tuning& tun);
void emit_prove_circuit(Program& pg, const gkr_circuit& c, const Workspace& w, const gkr_fr* d_inputs,
                        uint64_t seed, gkr_fr* d_outputs, uint8_t* d_proof, const Tuning& tun);
int32_t check_ws(const gkr_circuit* c, const void* ws, size_t ws_bytes);

}  // namespace gkr
