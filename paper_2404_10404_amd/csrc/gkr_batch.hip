// Batched proving: plans (a proof's step program recorded in device memory)
// and the persistent kernel that runs many plans at once.
//
// A plan is built once per job (allocating, synchronous). Running plans is
// asynchronous, allocates nothing and copies nothing between host and device:
// counters are cleared by a fill kernel and the job table travels in the
// kernel arguments, so a run can be captured in a HIP graph. A run that stops
// early (step budget, or stop-on-finish) leaves every plan at a step boundary
// or inside a partly claimed step; the next run continues from there.
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "gkr_kernels.hpp"
#include "gkr_program.hpp"
#include "gkr_tuning.hpp"

struct gkr_plan {
  gkr_job job;
  uint32_t nsteps = 0;
  void* dev = nullptr;  // steps, then counters
  gkr::Step* steps = nullptr;
  uint32_t* ctr = nullptr;
  size_t ctr_words = 0;
};

namespace gkr {
static bool aligned16b(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }
}  // namespace gkr

using namespace gkr;

extern "C" {

int32_t gkr_plan_create(const gkr_job* job, gkr_plan** out) {
  if (!job || !out || !job->circuit) {
    set_error("null argument");
    return GKR_EINVAL;
  }
  *out = nullptr;
  const gkr_circuit* c = job->circuit;
  if (c->general || c->field != GKR_FIELD_BN254) {
    set_error("batch plans take layered BN254 circuits only");
    return GKR_EUNSUPPORTED;
  }
  if (!job->d_inputs || !job->d_outputs || !job->d_proof || !aligned16b(job->d_inputs) ||
      !aligned16b(job->d_outputs) || !aligned16b(job->d_proof)) {
    set_error("null or misaligned job buffer");
    return GKR_EINVAL;
  }
  if (job->proof_cap < gkr_proof_bytes(c)) {
    set_error("proof buffer too small");
    return GKR_EBUFSZ;
  }
  int32_t rc = check_ws(c, job->d_ws, job->ws_bytes);
  if (rc) return rc;
  try {
    Workspace w = bind_workspace(*c, job->d_ws);
    Program pg;
    pg.matrix_cores = false;
    emit_prove_circuit(pg, *c, w, job->d_inputs, job->seed, job->d_outputs, job->d_proof, current_tuning());
    gkr_plan* p = new gkr_plan();
    p->job = *job;
    p->nsteps = (uint32_t)pg.steps.size();
    p->ctr_words = 1 + 2ull * p->nsteps;
    const size_t step_bytes = sizeof(Step) * pg.steps.size();
    const size_t total = step_bytes + 4 * p->ctr_words;
    if (hipMalloc(&p->dev, total) != hipSuccess) {
      (void)hipGetLastError();
      delete p;
      set_error("device allocation of the plan failed");
      return GKR_ENOMEM;
    }
    p->steps = static_cast<Step*>(p->dev);
    p->ctr = reinterpret_cast<uint32_t*>(static_cast<char*>(p->dev) + step_bytes);
    std::vector<uint32_t> zeros(p->ctr_words, 0);
    if (hipMemcpy(p->steps, pg.steps.data(), step_bytes, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(p->ctr, zeros.data(), 4 * p->ctr_words, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipGetLastError();
      hipFree(p->dev);
      delete p;
      set_error("upload of the plan failed");
      return GKR_EDEVICE;
    }
    *out = p;
    return GKR_OK;
  } catch (const std::bad_alloc&) {
    set_error("host allocation failed");
    return GKR_ENOMEM;
  }
}

void gkr_plan_destroy(gkr_plan* p) {
  if (!p) return;
  if (p->dev) hipFree(p->dev);
  delete p;
}

int32_t gkr_plan_reset(gkr_plan* p, void* stream) {
  if (!p) {
    set_error("null plan");
    return GKR_EINVAL;
  }
  launch_fill_u32(p->ctr, p->ctr_words, 0u, static_cast<hipStream_t>(stream));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return GKR_EDEVICE;
  }
  return GKR_OK;
}

int32_t gkr_run_batch(gkr_plan* const* plans, uint32_t n, uint32_t* d_ctl, uint32_t workgroups,
                      uint32_t step_budget, uint32_t stop_on_finish, void* stream) {
  if (!plans || !d_ctl || n == 0 || n > kMaxBatchJobs) {
    set_error("need 1.." + std::to_string(kMaxBatchJobs) + " plans and a control buffer");
    return GKR_EINVAL;
  }
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  for (uint32_t i = 0; i < n; ++i) {
    if (!plans[i]) {
      set_error("null plan");
      return GKR_EINVAL;
    }
    for (uint32_t k = 0; k < i; ++k)
      if (plans[k] == plans[i]) {
        set_error("a plan appears twice in one run");
        return GKR_EINVAL;
      }
    a.jobs[i].steps = plans[i]->steps;
    a.jobs[i].ctr = plans[i]->ctr;
    a.jobs[i].nsteps = plans[i]->nsteps;
  }
  a.njobs = n;
  a.step_budget = step_budget;
  a.stop_on_finish = stop_on_finish ? 1 : 0;
  a.ctl = d_ctl;
  if (workgroups == 0) {
    int dev = 0, cus = 0;
    hipGetDevice(&dev);
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
      (void)hipGetLastError();
      cus = 256;
    }
    workgroups = (uint32_t)cus * batch_kernel_max_workgroups_per_cu();
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  launch_fill_u32(d_ctl, 4, 0u, s);
  launch_batch(a, workgroups, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    set_error(std::string("kernel launch failed: ") + hipGetErrorString(e));
    return GKR_EDEVICE;
  }
  return GKR_OK;
}

int32_t gkr_plan_progress(const gkr_plan* p, uint32_t* done_steps, uint32_t* total_steps) {
  if (!p) {
    set_error("null plan");
    return GKR_EINVAL;
  }
  uint32_t cur = 0;
  if (hipMemcpy(&cur, p->ctr, 4, hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    set_error("reading plan progress failed");
    return GKR_EDEVICE;
  }
  if (done_steps) *done_steps = cur;
  if (total_steps) *total_steps = p->nsteps;
  return GKR_OK;
}

int32_t gkr_prove_batch(const gkr_job* jobs, uint32_t n, void* stream) {
  if (!jobs || n == 0) {
    set_error("no jobs");
    return GKR_EINVAL;
  }
  std::vector<gkr_plan*> plans(n, nullptr);
  int32_t rc = GKR_OK;
  for (uint32_t i = 0; i < n && rc == GKR_OK; ++i) rc = gkr_plan_create(&jobs[i], &plans[i]);
  uint32_t* ctl = nullptr;
  if (rc == GKR_OK && hipMalloc(&ctl, 16) != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation failed");
    rc = GKR_ENOMEM;
  }
  for (uint32_t b = 0; b < n && rc == GKR_OK; b += kMaxBatchJobs) {
    const uint32_t m = std::min<uint32_t>(kMaxBatchJobs, n - b);
    rc = gkr_run_batch(plans.data() + b, m, ctl, 0, 0, 0, stream);
  }
  if (rc == GKR_OK && hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) {
    (void)hipGetLastError();
    set_error("batch run failed");
    rc = GKR_EDEVICE;
  }
  if (ctl) hipFree(ctl);
  for (gkr_plan* p : plans) gkr_plan_destroy(p);
  return rc;
}

}  // extern "C"
