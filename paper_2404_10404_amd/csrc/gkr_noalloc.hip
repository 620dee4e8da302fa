// gkr_prove_circuit_noalloc: gkr_prove_circuit with its workspace in a
// static device array instead of a caller buffer, for callers that cannot
// allocate device memory (code under HIP graph capture, tight serving loops,
// harnesses that forbid allocation).
//
// The array `scratch` is GKR_NOALLOC_WORKSPACE_BYTES of device memory that
// each GPU the library runs on holds until the process ends. In host code its
// name is only a stand-in for the symbol, not a device address: the device
// address is looked up once per device with hipGetSymbolAddress (with that
// device current) and kept per device; every use below goes through that
// pointer. Every call on a GPU shares that GPU's array and it keeps the last
// call's contents: calls whose work overlaps on one GPU (queued on streams
// with no ordering between them) race; calls queued on one stream run one
// after another.
// Nothing in the array needs clearing between calls: a proof writes every
// table before it reads it, and its first transcript step zeroes the
// reduction counter and the pending-round flag in the proof's state.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "gkr_kernels.hpp"
#include "gkr_program.hpp"
#include "gkr_tuning.hpp"

static __device__ __align__(256) uint8_t scratch[GKR_NOALLOC_WORKSPACE_BYTES];

namespace gkr {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on each device (nullptr until looked up).
static void* g_scratch_ptr[kMaxDevices] = {};
static std::mutex g_scratch_mu;

// The scratch array's device address on the current device, looked up on the
// first call there.
static int32_t scratch_on_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    set_error("gkr_prove_circuit_noalloc: no current HIP device (or device index >= 64)");
    return GKR_EDEVICE;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      set_error(std::string("gkr_prove_circuit_noalloc: hipGetSymbolAddress(scratch) failed: ") +
                hipGetErrorString(e));
      return GKR_EDEVICE;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GKR_OK;
}

}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_prove_circuit_noalloc(const gkr_circuit* c, const gkr_fr* d_inputs, uint64_t seed,
                                             gkr_fr* d_outputs, uint8_t* d_proof, size_t proof_cap,
                                             size_t* proof_len, void* stream) {
  if (!c) {
    set_error("null circuit");
    return GKR_EINVAL;
  }
  if (c->plan.total > (size_t)GKR_NOALLOC_WORKSPACE_BYTES) {
    set_error("gkr_prove_circuit_noalloc: the circuit needs a " + std::to_string(c->plan.total) +
              "-byte workspace, above the static workspace of " +
              std::to_string((size_t)GKR_NOALLOC_WORKSPACE_BYTES) +
              " bytes; use gkr_prove_circuit with a caller workspace");
    return GKR_EUNSUPPORTED;
  }
  if (c->device < 0) {
    set_error("circuit was created without a HIP device (host-only: verification only)");
    return GKR_EDEVICE;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device) {
    (void)hipGetLastError();
    set_error("gkr_prove_circuit_noalloc: the current device is not the circuit's device");
    return GKR_EINVAL;
  }
  void* ws = nullptr;
  const int32_t rc = scratch_on_current_device(&ws);
  if (rc != GKR_OK) return rc;
  return gkr_prove_circuit(c, d_inputs, seed, d_outputs, d_proof, proof_cap, proof_len, ws,
                           (size_t)GKR_NOALLOC_WORKSPACE_BYTES, stream);
}
