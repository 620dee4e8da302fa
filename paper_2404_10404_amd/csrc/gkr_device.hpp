// Device helpers of the GKR kernels: element loads/stores, wave shuffles,
// workgroup reductions and the last-tile protocol of grid-wide reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "gkr_internal.hpp"
#include "gkr_kernels.hpp"

namespace gkr {

// Table elements live in device (global) memory: the loads and stores go
// through address-space-1 pointers so that they compile to global (not flat)
// memory instructions.
typedef uint32_t U32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) U32x4 GlobalU4;

__device__ __forceinline__ Fr ldf(const Fr* p, uint64_t i) {
  const GlobalU4* q = (const GlobalU4*)(p + i);
  const U32x4 a = q[0], b = q[1];
  return fr_make(a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w);
}

__device__ __forceinline__ void stf(Fr* p, uint64_t i, const Fr& v) {
  GlobalU4* q = (GlobalU4*)(p + i);
  q[0] = U32x4{v.v[0], v.v[1], v.v[2], v.v[3]};
  q[1] = U32x4{v.v[4], v.v[5], v.v[6], v.v[7]};
}

__device__ __forceinline__ Fr shfl_xor_fr(const Fr& a, int mask) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = (uint32_t)__shfl_xor((int)a.v[k], mask, 64);
  return r;
}

// The value of lane `src` in every lane of the wave.
__device__ __forceinline__ Fr shfl_fr(const Fr& a, int src) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = (uint32_t)__shfl((int)a.v[k], src, 64);
  return r;
}

// A DPP move of every limb (lanes of rows outside RowMask read zero).
template <int Ctrl, int RowMask>
__device__ __forceinline__ Fr dpp_fr(const Fr& a) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)a.v[k], Ctrl, RowMask, 0xF, false);
  return r;
}

// Sum over the 64 lanes of a wave (all lanes active) into lane 63: DPP steps
// within quads (quad_perm), half-rows and rows (mirrors), then across rows
// (row_bcast15, row_bcast31). Other lanes hold partial sums.
__device__ __forceinline__ Fr wave_sum_to_lane63(Fr v) {
  v = fr_add(v, dpp_fr<0xB1, 0xF>(v));   // quad_perm [1,0,3,2]
  v = fr_add(v, dpp_fr<0x4E, 0xF>(v));   // quad_perm [2,3,0,1]
  v = fr_add(v, dpp_fr<0x141, 0xF>(v));  // row_half_mirror
  v = fr_add(v, dpp_fr<0x140, 0xF>(v));  // row_mirror
  v = fr_add(v, dpp_fr<0x142, 0xA>(v));  // row_bcast15 into rows 1 and 3
  v = fr_add(v, dpp_fr<0x143, 0xC>(v));  // row_bcast31 into rows 2 and 3
  return v;
}

// Waits until every vector memory operation this wave has issued is
// complete (a store has reached the L2; a cache write-back or invalidation
// has finished). An asm statement with a memory clobber: the compiler moves no
// memory operation across it and does not drop it, unlike the s_waitcnt
// builtin, which it treats as touching no memory.
__device__ __forceinline__ void wait_vmem() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Agent-scope fences that also wait for their cache maintenance: the fence
// builtin orders the compiler and emits the L2 write-back (release) or the
// L1/L2 invalidation (acquire); the wait makes it complete before this wave's
// next instruction, so a workgroup barrier after it orders every wave of the
// workgroup behind it.
__device__ __forceinline__ void release_agent_wait() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  wait_vmem();
}
__device__ __forceinline__ void acquire_agent_wait() {
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  wait_vmem();
}

// A value in registers the compiler cannot trace back to its load: a kernel
// that never writes a field may otherwise load it again at every use (in the
// middle of a product's chain of multiply-adds) instead of keeping it live.
__device__ __forceinline__ Fr opaque(Fr x) {
#pragma unroll
  for (int k = 0; k < 8; ++k) asm volatile("" : "+v"(x.v[k]));
  return x;
}

template <class T>
__device__ __forceinline__ T P(const Step& st, int i) {
  return reinterpret_cast<T>(const_cast<void*>(st.p[i]));
}

// Sum of NV values over the workgroup; the totals are valid in thread 0.
template <int NV>
__device__ void block_reduce(Fr (&v)[NV]) {
  __shared__ Fr red[NV][kBlock / 64];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = fr_add(v[k], shfl_xor_fr(v[k], off));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      Fr acc = red[k][0];
#pragma unroll
      for (int w = 1; w < kBlock / 64; ++w) acc = fr_add(acc, red[k][w]);
      v[k] = acc;
    }
  }
  __syncthreads();
}

// Copies thread 0's values to every thread of the workgroup.
template <int NV>
__device__ void broadcast_from_thread0(Fr (&v)[NV]) {
  __shared__ Fr bc[NV];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) bc[k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = bc[k];
  __syncthreads();
}

// Workgroup sum of NV values, stored as the tile's partials.
// Sum of NV values over the workgroup (any multiple of 64 threads, at most
// 1024); the totals are valid in every lane of wave 0.
template <int NV>
__device__ __forceinline__ void block_sum_to_wave0(Fr (&v)[NV]) {
  __shared__ Fr red[NV][16];
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum_to_lane63(v[k]);
  const uint32_t lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 63) {
#pragma unroll
    for (int k = 0; k < NV; ++k) red[k][wid] = v[k];
  }
  __syncthreads();
  if (wid == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      Fr acc = red[k][0];
      for (uint32_t w = 1; w < nw; ++w) acc = fr_add(acc, red[k][w]);
      v[k] = acc;
    }
  }
}
// Per-tile partial sums of a grid-wide reduction (written by thread 0).
template <int NV>
__device__ void write_partial(Fr (&v)[NV], Fr* partials, uint32_t tile) {
  block_sum_to_wave0<NV>(v);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) stf(partials, (uint64_t)tile * NV + k, v[k]);
  }
}
// Publishes this tile's writes and counts it; true (in every thread) for the
// last of ntiles tiles, which then sees all tiles' writes. The counter is back
// at zero afterwards.
// Only the partial sums (written by thread 0) cross tiles here, so thread 0
// counts the tile with a release read-modify-write (an L2 write-back of its
// own earlier stores, no invalidation) and only the last tile pays for an
// acquire (L2 invalidation on this chip's per-XCD caches), in every one of
// its waves (each wave's own loads are ordered after its own invalidation).
__device__ __forceinline__ bool last_tile(uint32_t* counter, uint32_t ntiles) {
  __shared__ int is_last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == ntiles - 1);
    if (is_last) __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  const bool last = is_last;
  if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return last;
}

// Sum of the ntiles partials of a grid-wide reduction; valid in every lane of wave 0.
template <int NV>
__device__ void sum_partials(const Fr* partials, uint32_t ntiles, Fr (&out)[NV]) {
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = fr_zero();
  for (uint32_t b = threadIdx.x; b < ntiles; b += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NV; ++k) out[k] = fr_add(out[k], ldf(partials, (uint64_t)b * NV + k));
  }
  block_sum_to_wave0<NV>(out);
}

}  // namespace gkr
