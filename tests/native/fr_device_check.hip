// Device check of the prover's field code (test helper, built by build()).
//
// frcheck_run runs one operation of paper_2404_10404_amd/csrc/fr.hpp on the
// GPU, one thread per case, on limbs the test supplies, so the device paths
// the kernels use (inline-asm multiply-accumulates, the product-scanning
// Montgomery product, lazy accumulators and their reductions) are compared
// with Python integers. Case i reads a[i*terms + k], b[i*terms + k] for
// k < terms and writes out[i] (eight 32-bit limbs per element).
//   op 0  fr_mul(a0, b0)                          = a0 b0 R^-1 mod p
//   op 1  fr_mul_add2(a0, b0, a1, b1)             = (a0 b0 + a1 b1) R^-1
//   op 2  frw_mac over k < terms, frw_reduce<terms>   = sum a_k b_k R^-1
//   op 3  frc_mac over k < terms, frc_wide, frw_reduce<terms>
//   op 4  fr_sub(a0, b0)      op 5  fr_add(a0, b0)      op 6  fr_half(a0)
//   op 7  fr_double(a0)       op 8  fr_to_mont(a0)      op 9  fr_from_mont(a0)
#include <hip/hip_runtime.h>

#include "../../paper_2404_10404_amd/csrc/fr.hpp"

using namespace gkr;

namespace {

__device__ Fr ld(const uint32_t* p, uint64_t i) {
  Fr r;
#pragma unroll
  for (int k = 0; k < 8; ++k) r.v[k] = p[8 * i + k];
  return r;
}

template <int T>
__device__ Fr reduce_terms(const FrWide& A) { return frw_reduce<T>(A); }

__device__ Fr reduce_dyn(const FrWide& A, int terms) {
  switch (terms) {
#define C(n) case n: return reduce_terms<n>(A);
    C(1) C(2) C(3) C(4) C(5) C(6) C(7) C(8) C(9) C(10) C(11) C(12) C(13) C(14) C(15) C(16)
#undef C
    default: return fr_zero();
  }
}

__global__ void k_frcheck(int op, int terms, const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t n) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint64_t base = (uint64_t)i * terms;
  const Fr a0 = ld(a, base), b0 = ld(b, base);
  Fr r = fr_zero();
  switch (op) {
    case 0: r = fr_mul(a0, b0); break;
    case 1: r = fr_mul_add2(a0, b0, ld(a, base + 1), ld(b, base + 1)); break;
    case 2: {
      FrWide A = frw_zero();
      for (int k = 0; k < terms; ++k) frw_mac(A, ld(a, base + k), ld(b, base + k));
      r = reduce_dyn(A, terms);
      break;
    }
    case 3: {
      FrCols C = frc_zero();
      for (int k = 0; k < terms; ++k) frc_mac(C, ld(a, base + k), ld(b, base + k));
      r = reduce_dyn(frc_wide(C), terms);
      break;
    }
    case 4: r = fr_sub(a0, b0); break;
    case 5: r = fr_add(a0, b0); break;
    case 6: r = fr_half(a0); break;
    case 7: r = fr_double(a0); break;
    case 8: r = fr_to_mont(a0); break;
    case 9: r = fr_from_mont(a0); break;
    default: break;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) out[8ull * i + k] = r.v[k];
}

}  // namespace

// Returns 0, or -1 for bad arguments, -3 when the launch fails. Synchronous.
extern "C" int frcheck_run(int op, int terms, const void* d_a, const void* d_b, void* d_out, uint32_t n) {
  if (op < 0 || op > 9 || terms < 1 || terms > 16 || ((op == 1) && terms < 2) || !d_a || !d_b || !d_out)
    return -1;
  if (n == 0) return 0;
  const uint32_t block = 64;
  k_frcheck<<<(n + block - 1) / block, block>>>(op, terms, static_cast<const uint32_t*>(d_a),
                                                static_cast<const uint32_t*>(d_b), static_cast<uint32_t*>(d_out), n);
  if (hipGetLastError() != hipSuccess) return -3;
  if (hipDeviceSynchronize() != hipSuccess) return -3;
  return 0;
}
