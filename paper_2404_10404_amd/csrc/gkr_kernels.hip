// Plain kernels of the GKR prover for gfx950: one kernel per step type,
// launched with grid = the step's tile count (the bodies are in gkr_bodies.hpp).
#include "gkr_bodies.hpp"
#include "gkr_profile.hpp"

namespace gkr {

// ------------------------------------------------------------ plain kernels

// One kernel per step type, so each is compiled with only the registers its
// own body needs. The counter of a reduction step lives in the proof's state.
#define GKR_PLAIN_KERNEL(NAME, TYPE)                                              \
  __global__ void __launch_bounds__(kBlock) NAME(Step st) {                       \
    run_step_tile_##TYPE(st, blockIdx.x, gridDim.x);                              \
  }
// Grid-wide sweeps whose speed depends on latency hiding: at least 3 waves
// per SIMD (at most 168 VGPRs).
#define GKR_PLAIN_KERNEL_OCC3(NAME, TYPE)                                         \
  __global__ void __launch_bounds__(kBlock, 3) NAME(Step st) {                    \
    run_step_tile_##TYPE(st, blockIdx.x, gridDim.x);                              \
  }

#define GKR_SIMPLE(TYPE, BODY) \
  __device__ __forceinline__ void run_step_tile_##TYPE(const Step& st, uint32_t t, uint32_t n) { BODY(st, t, n); }

GKR_SIMPLE(to_mont, body_to_mont)
GKR_SIMPLE(from_mont, body_from_mont)
GKR_SIMPLE(forward, body_forward)
GKR_SIMPLE(digest, body_digest)
GKR_SIMPLE(transcript_begin, body_transcript_begin)
GKR_SIMPLE(squeeze, body_squeeze)
GKR_SIMPLE(layer_begin, body_layer_begin)
GKR_SIMPLE(eq, body_eq)
GKR_SIMPLE(p1_init, body_p1_init)
GKR_SIMPLE(tail_a, body_tail_pipe<FormA>)
GKR_SIMPLE(tail_b, body_tail_pipe<FormB>)
GKR_SIMPLE(copy_weights, body_copy_weights)
GKR_SIMPLE(p2_tables, body_p2_tables)
GKR_SIMPLE(copy_contract, body_copy_contract)
GKR_SIMPLE(local_contract, body_local_contract)
GKR_SIMPLE(copy_tables, body_copy_tables)
GKR_SIMPLE(state_export, body_state_export)
GKR_SIMPLE(state_import, body_state_import)

__device__ __forceinline__ void run_step_tile_wsum(const Step& st, uint32_t t, uint32_t n) {
  body_wsum(st, t, n);
  if (last_tile(&P<DevState*>(st, 4)->counter, n)) finish_wsum(st, n);
}
__device__ __forceinline__ void run_step_tile_p1_init_round(const Step& st, uint32_t t, uint32_t n) {
  body_p1_init_round<true>(st, t, n);
  if (last_tile(&P<DevState*>(st, 9)->counter, n)) finish_p1_init_round(st, n);
}
__device__ __forceinline__ void run_step_tile_round_a(const Step& st, uint32_t t, uint32_t n) {
  body_round<FormA>(st, t, n);
  if (last_tile(&P<DevState*>(st, RoundPtrs<3>::kS)->counter, n)) finish_round_step<FormA>(st, n);
}
__device__ __forceinline__ void run_step_tile_local_values(const Step& st, uint32_t t, uint32_t n) {
  body_local_values(st, t, n);
  if (last_tile(&P<DevState*>(st, 3)->counter, n)) finish_local_values(st, n);
}
__device__ __forceinline__ void run_step_tile_round_b(const Step& st, uint32_t t, uint32_t n) {
  body_round<FormB>(st, t, n);
  if (last_tile(&P<DevState*>(st, RoundPtrs<5>::kS)->counter, n)) finish_round_step<FormB>(st, n);
}

GKR_PLAIN_KERNEL(k_to_mont, to_mont)
GKR_PLAIN_KERNEL(k_from_mont, from_mont)
GKR_PLAIN_KERNEL(k_forward, forward)
GKR_PLAIN_KERNEL(k_digest, digest)
GKR_PLAIN_KERNEL(k_transcript_begin, transcript_begin)
GKR_PLAIN_KERNEL(k_squeeze, squeeze)
GKR_PLAIN_KERNEL(k_layer_begin, layer_begin)
GKR_PLAIN_KERNEL(k_eq, eq)
GKR_PLAIN_KERNEL(k_wsum, wsum)
GKR_PLAIN_KERNEL(k_p1_init, p1_init)
#define GKR_PLAIN_KERNEL_OCC4(NAME, TYPE)                                         \
  __global__ void __launch_bounds__(kBlock, 4) NAME(Step st) {                    \
    run_step_tile_##TYPE(st, blockIdx.x, gridDim.x);                              \
  }
GKR_PLAIN_KERNEL_OCC4(k_p1_init_round, p1_init_round)
GKR_PLAIN_KERNEL_OCC3(k_round_a, round_a)
GKR_PLAIN_KERNEL_OCC3(k_round_b, round_b)
// The single-workgroup tails run with kTailBlock threads (two waves per SIMD).
#define GKR_TAIL_KERNEL(NAME, TYPE)                                               \
  __global__ void __launch_bounds__(kTailBlock) NAME(Step st) {                   \
    run_step_tile_##TYPE(st, blockIdx.x, gridDim.x);                              \
  }
GKR_TAIL_KERNEL(k_tail_a, tail_a)
GKR_TAIL_KERNEL(k_tail_b, tail_b)
GKR_PLAIN_KERNEL(k_copy_weights, copy_weights)
GKR_PLAIN_KERNEL(k_p2_tables, p2_tables)
GKR_PLAIN_KERNEL(k_copy_contract, copy_contract)
GKR_PLAIN_KERNEL(k_local_contract, local_contract)
GKR_PLAIN_KERNEL(k_copy_tables, copy_tables)
GKR_PLAIN_KERNEL(k_local_values, local_values)
GKR_PLAIN_KERNEL(k_state_export, state_export)
GKR_PLAIN_KERNEL(k_state_import, state_import)

static const ProfClass kStepClass[ST_COUNT] = {
    PC_CONVERT,        PC_CONVERT, PC_FORWARD, PC_DIGEST,        PC_TRANSCRIPT,    PC_TRANSCRIPT,
    PC_TRANSCRIPT,     PC_EQ,      PC_CLAIM,   PC_PHASE1_INIT,   PC_PHASE1_INIT,   PC_ROUND_A,
    PC_ROUND_B,        PC_TAIL_A,  PC_TAIL_B,  PC_SMALL,         PC_PHASE2_TABLES, PC_COPY_CONTRACT,
    PC_LOCAL_CONTRACT, PC_SMALL,   PC_SMALL,   PC_SMALL,         PC_SMALL};

void launch_step(const Step& st, hipStream_t s) {
  const int tok = prof_begin(s);
  const dim3 grid(st.ntiles), block(kBlock);
  switch (st.type) {
    case ST_TO_MONT: k_to_mont<<<grid, block, 0, s>>>(st); break;
    case ST_FROM_MONT: k_from_mont<<<grid, block, 0, s>>>(st); break;
    case ST_FORWARD: k_forward<<<grid, block, 0, s>>>(st); break;
    case ST_DIGEST: k_digest<<<grid, block, 0, s>>>(st); break;
    case ST_TRANSCRIPT_BEGIN: k_transcript_begin<<<grid, block, 0, s>>>(st); break;
    case ST_SQUEEZE: k_squeeze<<<grid, block, 0, s>>>(st); break;
    case ST_LAYER_BEGIN: k_layer_begin<<<grid, block, 0, s>>>(st); break;
    case ST_EQ: k_eq<<<grid, block, 0, s>>>(st); break;
    case ST_WSUM: k_wsum<<<grid, block, 0, s>>>(st); break;
    case ST_P1_INIT: k_p1_init<<<grid, block, 0, s>>>(st); break;
    case ST_P1_INIT_ROUND: k_p1_init_round<<<grid, block, 0, s>>>(st); break;
    case ST_ROUND_A: k_round_a<<<grid, block, 0, s>>>(st); break;
    case ST_ROUND_B: k_round_b<<<grid, block, 0, s>>>(st); break;
    case ST_TAIL_A: k_tail_a<<<grid, dim3(kTailBlock), 0, s>>>(st); break;
    case ST_TAIL_B: k_tail_b<<<grid, dim3(kTailBlock), 0, s>>>(st); break;
    case ST_COPY_WEIGHTS: k_copy_weights<<<grid, block, 0, s>>>(st); break;
    case ST_P2_TABLES: k_p2_tables<<<grid, block, 0, s>>>(st); break;
    case ST_COPY_CONTRACT: k_copy_contract<<<grid, block, 0, s>>>(st); break;
    case ST_LOCAL_CONTRACT: k_local_contract<<<grid, block, 0, s>>>(st); break;
    case ST_COPY_TABLES: k_copy_tables<<<grid, block, 0, s>>>(st); break;
    case ST_LOCAL_VALUES: k_local_values<<<grid, block, 0, s>>>(st); break;
    case ST_STATE_EXPORT: k_state_export<<<grid, block, 0, s>>>(st); break;
    case ST_STATE_IMPORT: k_state_import<<<grid, block, 0, s>>>(st); break;
    default: break;
  }
  if (tok >= 0) prof_end(tok, s, kStepClass[st.type], st.bytes, st.mulmods);
}

}  // namespace gkr
