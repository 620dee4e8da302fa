// The persistent batch kernel of the GKR prover (many proofs' step programs
// in one launch); the step bodies are in gkr_bodies.hpp.
#include "gkr_bodies.hpp"
#include "gkr_profile.hpp"

namespace gkr {

// ------------------------------------------------------------ batch kernel

// Persistent kernel over up to kMaxBatchJobs step programs. Job j's counters
// (device memory) are ctr[0] = current step, ctr[1 + s] = tiles of step s
// claimed, ctr[1 + nsteps + s] = tiles of step s done. A workgroup claims a
// tile of some job's current step, runs it, and counts it done; the tile that
// completes a step publishes the next one (release fence, then the store), and
// the tile that completes a job's last step counts the job finished. Tiles
// never wait on other tiles, so the kernel always drains: a workgroup leaves
// when a scan finds no unfinished job, or once ctl[1] (stop) is set - when the
// step budget is reached or, with stop_on_finish, when any job finishes. A
// workgroup with no claimable tile while jobs are unfinished sleeps and scans
// again; the tiles it waits for are running and never wait themselves. A
// claimed tile is always run to the end, so a later launch continues exactly
// where this one stopped. ctl[0] = jobs finished in this launch, ctl[2] =
// steps completed.
// The launch bound (two workgroups per CU, up to 256 vector registers per
// lane) keeps every value of this large kernel in registers; the build
// refuses kernels that spill, which guards the occupancy target (a spilled
// build once gave wrong proofs in stop/resume runs, when the end-of-tile
// release relied on an s_waitcnt builtin; see the release below).
__global__ void __launch_bounds__(kBlock, 2) k_batch(BatchArgs a) {
  __shared__ uint32_t sh_job, sh_step, sh_tile, sh_state;  // state: 0 work, 1 none, 2 exit
  __shared__ uint32_t sh_acquire;  // 1: the claimed tile's (job, step) needs an acquire
  __shared__ Step sh_st;
  uint32_t* ctl = a.ctl;
  const uint32_t njobs = a.njobs;
  uint32_t start = (blockIdx.x * 2654435761u) % njobs;
  // The (job, step) this workgroup last acquired for (thread 0). Further tiles
  // of the same step need no new acquire: their inputs are outputs of earlier
  // steps, all published before that acquire, and nothing rewrites a step's
  // inputs while the step runs, so no stale line can have entered the caches.
  uint32_t acq_job = ~0u, acq_step = ~0u;
  for (;;) {
    if (threadIdx.x == 0) {
      uint32_t state = 1;
      if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        state = 2;
      } else {
        bool unfinished = false;
        for (uint32_t scan = 0; scan < njobs && state == 1; ++scan) {
          const uint32_t j = (start + scan) % njobs;
          const BatchJobDev& jb = a.jobs[j];
          uint32_t* ctr = jb.ctr;
          // relaxed: the acquire fence below runs once a tile is claimed
          const uint32_t s = __hip_atomic_load(&ctr[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (s >= jb.nsteps) continue;
          unfinished = true;
          const uint32_t nt = jb.steps[s].ntiles;
          if (__hip_atomic_load(&ctr[1 + s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= nt) continue;
          const uint32_t t = atomicAdd(&ctr[1 + s], 1u);
          if (t < nt) {
            sh_job = j;
            sh_step = s;
            sh_tile = t;
            sh_acquire = (j != acq_job || s != acq_step) ? 1u : 0u;
            acq_job = j;
            acq_step = s;
            state = 0;
            start = j;  // stay with this job while it has tiles
          }
        }
        if (!unfinished) state = 2;  // every job is finished
      }
      sh_state = state;
    }
    __syncthreads();
    const uint32_t state = sh_state;
    if (state == 2) break;
    if (state == 1) {
      if (threadIdx.x == 0) __builtin_amdgcn_s_sleep(8);
      __syncthreads();
      continue;
    }
    const uint32_t j = sh_job, s = sh_step, tile = sh_tile;
    const BatchJobDev& jb = a.jobs[j];
    // copy the step record to LDS (256-byte record, 4-byte words)
    {
      const uint32_t* src = reinterpret_cast<const uint32_t*>(&jb.steps[s]);
      uint32_t* dst = reinterpret_cast<uint32_t*>(&sh_st);
      for (uint32_t k = threadIdx.x; k < sizeof(Step) / 4; k += kBlock) dst[k] = src[k];
    }
    // Acquire the writes of the previous steps (published by the release store
    // of ctr[0] the scan read): one wave invalidates (the CU's L1 and this
    // XCD's L2 copies of lines other XCDs write) and waits for the
    // invalidation to complete before the barrier, so no wave of the workgroup
    // loads before it is done. (Without the wait the barrier does not hold the
    // other waves back, and their loads could hit stale lines while the
    // invalidation is in flight.)
    if (threadIdx.x < 64 && sh_acquire) acquire_agent_wait();
    __syncthreads();
    run_step_tile(sh_st, tile, sh_st.ntiles);
    // Release this tile's writes before it is counted done (workgroups on
    // other XCDs read these tables in the next step): every wave waits until
    // its stores have reached the L2 (the compiler moves no store below the
    // wait), then, after the barrier, one wave writes the L2 back and waits for
    // the write-back before it counts the tile. A workgroup-scope barrier
    // alone does not wait for global stores on this chip, and an s_waitcnt
    // builtin is no compiler memory barrier, so neither orders another wave's
    // stores before the counter update.
    wait_vmem();
    __syncthreads();
    if (threadIdx.x < 64) release_agent_wait();
    if (threadIdx.x == 0) {
      uint32_t* ctr = jb.ctr;
      const uint32_t d = __hip_atomic_fetch_add(&ctr[1 + jb.nsteps + s], 1u, __ATOMIC_RELEASE,
                                                __HIP_MEMORY_SCOPE_AGENT);
      if (d == sh_st.ntiles - 1) {
        __threadfence();
        const uint32_t done_steps = atomicAdd(&ctl[2], 1u) + 1;
        __hip_atomic_store(&ctr[0], s + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        if (s + 1 == jb.nsteps) {
          atomicAdd(&ctl[0], 1u);
          if (a.stop_on_finish) atomicExch(&ctl[1], 1u);
        }
        if (a.step_budget && done_steps >= a.step_budget) atomicExch(&ctl[1], 1u);
      }
    }
    __syncthreads();
  }
}

// Zero a job's counters (n words) so its program runs from the start.
__global__ void __launch_bounds__(kBlock) k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kBlock) p[i] = v;
}

void launch_batch(const BatchArgs& a, uint32_t workgroups, hipStream_t s) {
  const int tok = prof_begin(s);
  k_batch<<<workgroups, kBlock, 0, s>>>(a);
  if (tok >= 0) prof_end(tok, s, PC_BATCH, 0.0, 0.0);
}

void launch_fill_u32(uint32_t* p, uint64_t n, uint32_t v, hipStream_t s) {
  uint64_t g = (n + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  k_fill_u32<<<(uint32_t)g, kBlock, 0, s>>>(p, n, v);
}

uint32_t batch_kernel_max_workgroups_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_batch, kBlock, 0) != hipSuccess) {
    (void)hipGetLastError();
    return 1;
  }
  return nb < 1 ? 1 : (uint32_t)nb;
}

}  // namespace gkr
