// Launchers of the GKR kernels (implemented in gkr_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "gkr_internal.hpp"

namespace gkr {

struct Words8 {
  uint32_t w[8];
};

template <int NT>
struct Tabs {
  const Fr* src[NT];
  Fr* dst[NT];
};

// Phase 1 and the copy rounds of phase 2: sum_b W[b] G[b] + H[b]; tables (W, G, H).
struct FormA {
  static constexpr int NT = 3;
  __device__ static inline void eval(const Fr* x, Fr& acc) {
    acc = fr_add(acc, fr_add(fr_mul(x[0], x[1]), x[2]));
  }
};

// Sub-circuit rounds of phase 2 with the copy factors contracted:
// sum_b P[b] Fa[b] + Q[b] Fb[b] + Ks[b]; tables (P, Fa, Q, Fb, Ks).
struct FormB {
  static constexpr int NT = 5;
  __device__ static inline void eval(const Fr* x, Fr& acc) {
    acc = fr_add(acc, fr_add(fr_add(fr_mul(x[0], x[1]), fr_mul(x[2], x[3])), x[4]));
  }
};

struct EqJobs {
  int count;
  int bits[4];
  const Fr* point[4];
  const Fr* scale[4];  // nullptr = 1
  Fr* out[4];
};

void launch_to_mont(const gkr_fr* in, Fr* out, uint64_t n, hipStream_t s);
void launch_from_mont(const Fr* in, gkr_fr* out, uint64_t n, hipStream_t s);
void launch_forward(const Fr* W, Fr* V, const uint2* gates, uint32_t n, uint64_t count,
                    uint64_t mul_gates, hipStream_t s);
void launch_digest_level(const uint32_t* in, uint64_t nwords, int swap, uint32_t* out, uint64_t nchunks,
                         hipStream_t s);
void launch_transcript_begin(DevState* S, const Words8& seed_state, const Words8& circ,
                             const uint32_t* din, const uint32_t* dout, hipStream_t s);
void launch_squeeze(DevState* S, Fr* out, uint32_t count, hipStream_t s);
void launch_layer_begin(DevState* S, int first, const Fr* vu, const Fr* vv, hipStream_t s);
void launch_eq_tables(const EqJobs& jobs, hipStream_t s);
void launch_weighted_sum(const Fr* V, const Fr* A, const Fr* B, uint32_t n, uint64_t count,
                         Fr* partials, uint32_t* counter, Fr* dst, uint32_t max_blocks, hipStream_t s);
void launch_phase1_init(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU,
                        const Fr* bV, const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t count,
                        uint64_t gates, hipStream_t s);
void launch_phase1_init_round(const Fr* W, Fr* G, Fr* H, const LayerWiring& lw, const Fr* aU,
                              const Fr* bV, const Fr* Cu, const Fr* Cv, uint32_t n, uint64_t half,
                              uint64_t gates, DevState* S, Fr* partials, Fr* r_out, uint32_t* msg,
                              uint32_t max_blocks, hipStream_t s);
template <class Form>
void launch_round(const Tabs<Form::NT>& t, uint64_t half, const Fr* rprev, DevState* S,
                  Fr* partials, Fr* r_out, uint32_t* msg, uint32_t max_blocks, hipStream_t s);
template <class Form>
void launch_tail(const Tabs<Form::NT>& t, uint64_t size, const Fr* rpending, uint32_t rounds,
                 DevState* S, Fr* r_out, uint32_t* msg, Fr* final_out, uint32_t* proof_value,
                 hipStream_t s);
void launch_copy_weights(const Fr* Cu, const Fr* Cv, const Fr* EC, Fr* U, Fr* V, uint64_t ncop,
                         DevState* S, hipStream_t s);
void launch_phase2_tables(const LayerWiring& lw, const Fr* aU, const Fr* bV, const Fr* EL,
                          const DevState* S, Fr* Fa, Fr* Fb, Fr* Ka, Fr* Kb, Fr* Ks, uint64_t count,
                          uint64_t gates, hipStream_t s);
void launch_copy_contract(const Fr* W, const Fr* U, const Fr* V, Fr* P, Fr* Q, uint32_t n,
                          uint64_t rows, hipStream_t s);
void launch_local_contract(const Fr* W, const Fr* EqR, Fr* part, uint32_t n, uint64_t rows,
                           uint32_t ychunks, hipStream_t s);
void launch_copy_tables(const Fr* part, uint32_t ychunks, const Fr* U, const Fr* V, const Fr* fa_f,
                        const Fr* fb_f, const DevState* S, Fr* Wc, Fr* Fc, Fr* Kc, uint64_t ncop,
                        hipStream_t s);
void launch_local_values(const Fr* EqR, const Fr* Ka, const Fr* Kb, uint64_t rows, DevState* S,
                         hipStream_t s);
void launch_state_export(const DevState* S, uint8_t* out, hipStream_t s);
void launch_state_import(DevState* S, const uint8_t* in, hipStream_t s);

}  // namespace gkr
