// Integer-multiply microbenchmarks of the VALU, and the HBM stream of a
// folding round: the measured ceilings the roofline of the prover's kernels
// is read against (beside the datasheet peaks).
//
// Each kernel runs `iters` iterations of independent dependency chains per
// thread (enough chains that the issue rate, not the latency, bounds them)
// over a grid that fills every SIMD several times; the rate is operations per
// second over the whole grid, timed with HIP events around one launch.
#include <hip/hip_runtime.h>

#include <string>

#include "fr.hpp"
#include "gkr_kernels.hpp"

namespace gkr {

constexpr int kUbBlock = 256;
constexpr int kUbChains = 8;
constexpr int kUbUnroll = 16;

// v_mad_u64_u32: 32 x 32 -> 64-bit product plus a 64-bit addend.
__global__ void __launch_bounds__(kUbBlock) k_ub_mad64(uint32_t iters, uint32_t* out) {
  uint64_t a[kUbChains];
  const uint32_t x = threadIdx.x * 2654435761u + blockIdx.x, y = x ^ 0x9e3779b9u;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) a[k] = (uint64_t)(x + k) << 7;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUbUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kUbChains; ++k)
        asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(a[k]) : "v"(x), "v"(y) : "vcc");
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) s ^= a[k];
  out[blockIdx.x * kUbBlock + threadIdx.x] = (uint32_t)s ^ (uint32_t)(s >> 32);
}

// The multiply-accumulate of the device field product: v_mad_u64_u32 with its
// carry into an overflow word (v_addc). Counted as one operation per pair.
__global__ void __launch_bounds__(kUbBlock) k_ub_mac_pair(uint32_t iters, uint32_t* out) {
  uint64_t a[kUbChains];
  uint32_t o[kUbChains];
  const uint32_t x = threadIdx.x * 2654435761u + blockIdx.x, y = x ^ 0x9e3779b9u;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) {
    a[k] = (uint64_t)(x + k) << 7;
    o[k] = 0;
  }
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUbUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kUbChains; ++k)
        asm volatile("v_mad_u64_u32 %0, vcc, %2, %3, %0\n\tv_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
                     : "+v"(a[k]), "+v"(o[k])
                     : "v"(x), "v"(y)
                     : "vcc");
    }
  }
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) s ^= a[k] ^ o[k];
  out[blockIdx.x * kUbBlock + threadIdx.x] = (uint32_t)s ^ (uint32_t)(s >> 32);
}

// A full-rate reference: v_add_u32.
__global__ void __launch_bounds__(kUbBlock) k_ub_add32(uint32_t iters, uint32_t* out) {
  uint32_t a[kUbChains];
  const uint32_t x = threadIdx.x * 2654435761u + blockIdx.x;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) a[k] = x + k;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUbUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kUbChains; ++k) asm volatile("v_add_u32_e32 %0, %0, %1" : "+v"(a[k]) : "v"(x));
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) s ^= a[k];
  out[blockIdx.x * kUbBlock + threadIdx.x] = s;
}

// v_mul_lo_u32 and v_mul_hi_u32 (the two halves of a 32 x 32 product).
__global__ void __launch_bounds__(kUbBlock) k_ub_mul32(uint32_t iters, uint32_t* out) {
  uint32_t a[kUbChains];
  const uint32_t x = threadIdx.x * 2654435761u + blockIdx.x;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) a[k] = x + k;
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < kUbUnroll; ++u) {
#pragma unroll
      for (int k = 0; k < kUbChains; ++k) {
        if (k & 1) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(a[k]) : "v"(x));
        else asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(a[k]) : "v"(x));
      }
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kUbChains; ++k) s ^= a[k];
  out[blockIdx.x * kUbBlock + threadIdx.x] = s;
}

// Montgomery products of the prover (fr_mul, the device product-scanning
// form): four independent chains x <- x * y per thread.
__global__ void __launch_bounds__(kUbBlock) k_ub_frmul(uint32_t iters, uint32_t* out) {
  constexpr int kChains = 4;
  const uint32_t t = blockIdx.x * kUbBlock + threadIdx.x;
  Fr x[kChains];
  const Fr y = fr_make(t * 2654435761u, t, 0x12345678u, t ^ 0xabcdefu, 7u, t * 3u, 0x2468aceu, 0x0e0a77c1u);
#pragma unroll
  for (int k = 0; k < kChains; ++k) x[k] = fr_make(t + k, k, t, 1u, 2u, 3u, t ^ k, 0x01234567u);
  for (uint32_t i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < kChains; ++k) x[k] = fr_mul(x[k], y);
  }
  uint32_t s = 0;
#pragma unroll
  for (int k = 0; k < kChains; ++k)
#pragma unroll
    for (int j = 0; j < 8; ++j) s ^= x[k].v[j];
  out[t] = s;
}

// The HBM access pattern of a folding round, without its arithmetic: for
// each b < h, the 32-byte entries b, b + 2h, b + h and b + 3h of a 4h-entry
// table are read and two 32-byte entries b and b + h of a 2h-entry table
// written (as 16-byte global loads and stores, one pair per thread). The rate
// it reaches is the practical ceiling of the round kernels' traffic.
typedef uint32_t UbU4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) UbU4 UbGlobalU4;
__global__ void __launch_bounds__(kUbBlock) k_ub_stream(const UbU4* src_g, UbU4* dst_g, uint64_t h) {
  const uint64_t b = (uint64_t)blockIdx.x * kUbBlock + threadIdx.x;
  if (b >= h) return;
  const UbGlobalU4* src = (const UbGlobalU4*)src_g;
  UbGlobalU4* dst = (UbGlobalU4*)dst_g;
  const UbU4 a0 = src[2 * b], a1 = src[2 * b + 1];
  const UbU4 c0 = src[2 * (b + 2 * h)], c1 = src[2 * (b + 2 * h) + 1];
  const UbU4 e0 = src[2 * (b + h)], e1 = src[2 * (b + h) + 1];
  const UbU4 f0 = src[2 * (b + 3 * h)], f1 = src[2 * (b + 3 * h) + 1];
  dst[2 * b] = a0 ^ c0;
  dst[2 * b + 1] = a1 ^ c1;
  dst[2 * (b + h)] = e0 ^ f0;
  dst[2 * (b + h) + 1] = e1 ^ f1;
}
constexpr uint64_t kUbStreamPairs = 1ull << 24;  // h: a 2 GiB source, a 1 GiB destination

// Passes of the stream pattern: bytes moved per second (reads + writes).
static int32_t ubench_stream(uint32_t passes, double* bytes_per_s, double* ms_out) {
  const uint64_t h = kUbStreamPairs;
  void *src = nullptr, *dst = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int32_t rc = GKR_OK;
  if (hipMalloc(&src, 4 * h * 32) != hipSuccess || hipMalloc(&dst, 2 * h * 32) != hipSuccess) {
    (void)hipGetLastError();
    set_error("gkr_ubench: allocation failed");
    rc = GKR_ENOMEM;
  }
  float ms = 0.f;
  if (rc == GKR_OK && (hipMemset(src, 0x5a, 4 * h * 32) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
                       hipEventCreate(&e1) != hipSuccess))
    rc = GKR_EDEVICE;
  const uint32_t blocks = (uint32_t)(h / kUbBlock);
  if (rc == GKR_OK) {
    const UbU4* s = static_cast<const UbU4*>(src);
    UbU4* d = static_cast<UbU4*>(dst);
    k_ub_stream<<<blocks, kUbBlock>>>(s, d, h);  // warm-up
    hipEventRecord(e0, nullptr);
    for (uint32_t i = 0; i < passes; ++i) k_ub_stream<<<blocks, kUbBlock>>>(s, d, h);
    hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = GKR_EDEVICE;
  }
  if (rc == GKR_EDEVICE) {
    (void)hipGetLastError();
    set_error("gkr_ubench: launch or timing failed");
  } else if (rc == GKR_OK) {
    *bytes_per_s = 6.0 * h * 32 * passes / (ms * 1e-3);
    if (ms_out) *ms_out = ms;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  if (src) hipFree(src);
  if (dst) hipFree(dst);
  return rc;
}

}  // namespace gkr

using namespace gkr;

extern "C" int32_t gkr_ubench(uint32_t kind, uint32_t iters, double* ops_per_s, double* ms_out) {
  if (!ops_per_s || iters == 0 || kind > 5) {
    set_error("gkr_ubench: kind must be 0..5, iters > 0, ops_per_s non-null");
    return GKR_EINVAL;
  }
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) {
    (void)hipGetLastError();
    set_error("gkr_ubench: no HIP device");
    return GKR_EDEVICE;
  }
  if (kind == 5) return ubench_stream(iters, ops_per_s, ms_out);
  const uint32_t blocks = (uint32_t)cus * 16;  // 16 waves per SIMD-quad: four per SIMD
  uint32_t* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipMalloc(&out, sizeof(uint32_t) * blocks * kUbBlock) != hipSuccess) {
    (void)hipGetLastError();
    set_error("gkr_ubench: allocation failed");
    return GKR_ENOMEM;
  }
  int32_t rc = GKR_OK;
  float ms = 0.f;
  double ops_per_thread = 0;
  auto launch = [&](uint32_t it) {
    switch (kind) {
      case 0: k_ub_mad64<<<blocks, kUbBlock>>>(it, out); break;
      case 1: k_ub_mac_pair<<<blocks, kUbBlock>>>(it, out); break;
      case 2: k_ub_add32<<<blocks, kUbBlock>>>(it, out); break;
      case 3: k_ub_mul32<<<blocks, kUbBlock>>>(it, out); break;
      default: k_ub_frmul<<<blocks, kUbBlock>>>(it, out); break;
    }
  };
  ops_per_thread = (kind == 4) ? 4.0 * iters : (double)kUbChains * kUbUnroll * iters;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = GKR_EDEVICE;
  if (rc == GKR_OK) {
    launch(iters < 4 ? iters : 4);  // warm-up (code load, clocks)
    hipEventRecord(e0, nullptr);
    launch(iters);
    hipEventRecord(e1, nullptr);
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = GKR_EDEVICE;
  }
  if (rc != GKR_OK) {
    (void)hipGetLastError();
    set_error("gkr_ubench: launch or timing failed");
  } else {
    *ops_per_s = ops_per_thread * blocks * kUbBlock / (ms * 1e-3);
    if (ms_out) *ms_out = ms;
  }
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  hipFree(out);
  return rc;
}
