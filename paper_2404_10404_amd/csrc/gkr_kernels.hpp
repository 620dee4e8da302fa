// Step forms and launchers of the GKR kernels (implemented in gkr_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "gkr_internal.hpp"

namespace gkr {

struct Words8 {
  uint32_t w[8];
};

// Phase 1 and the copy rounds of phase 2: sum_b W[b] G[b] + H[b]; tables (W, G, H).
struct FormA {
  static constexpr int NT = 3;
};

// Sub-circuit rounds of phase 2 with the copy factors contracted:
// sum_b P[b] Fa[b] + Q[b] Fb[b] + Ks[b]; tables (P, Fa, Q, Fb, Ks).
struct FormB {
  static constexpr int NT = 5;
};

// Pointer slots of round steps over NT tables: src[0..NT), dst[NT..2NT), then
// the previous challenge (null: no fold), the proof state, the partials, the
// challenge output and the message output.
template <int NT>
struct RoundPtrs {
  static constexpr int kR = 2 * NT, kS = kR + 1, kPart = kR + 2, kROut = kR + 3, kMsg = kR + 4;
};

// Launch one step as its own kernel (grid = st.ntiles workgroups).
void launch_step(const Step& st, hipStream_t s);

// One job of the persistent batch kernel: its step program and counters
// (ctr[0] current step, ctr[1..nsteps] claimed tiles, ctr[1+nsteps..] done tiles).
struct BatchJobDev {
  const Step* steps;
  uint32_t* ctr;
  uint32_t nsteps;
  uint32_t pad;
};

constexpr uint32_t kMaxBatchJobs = 64;

struct BatchArgs {
  BatchJobDev jobs[kMaxBatchJobs];
  uint32_t njobs;
  uint32_t step_budget;     // 0 = no budget
  uint32_t stop_on_finish;  // stop the launch when any job finishes
  uint32_t pad;
  uint32_t* ctl;            // [0] jobs finished, [1] stop, [2] steps completed, [3] spare
};

void launch_batch(const BatchArgs& a, uint32_t workgroups, hipStream_t s);
void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s);
uint32_t batch_kernel_max_workgroups_per_cu();

}  // namespace gkr
