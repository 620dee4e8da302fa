// The phase-2 copy contraction on the matrix cores (gkr_contract.hip): plan,
// step emission and launcher. Used by the plain path for layers with at least
// 2^kCcMinLogRows sub-circuit wires and 2^kCcMinLogCopies copies; the scalar
// contraction (ST_COPY_CONTRACT) takes every other layer and the batch kernel.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "gkr_internal.hpp"

namespace gkr {

constexpr uint32_t kCcMinLogCopies = 10;  // rows of at least 32 KiB
constexpr uint32_t kCcMinLogRows = 8;     // at least one 256-row tile
constexpr uint64_t kCcTargetGroups = 256; // workgroups of the product (row tiles x K chunks), one per CU

struct CcPlan {
  uint32_t chunks = 0, row_tiles = 0;
  uint64_t chunk_bytes = 0;
  size_t bt_bytes = 0, part_bytes = 0, bs_bytes = 0;
};

bool cc_applies(uint32_t n, uint32_t sigma);
CcPlan cc_plan(uint32_t n, uint32_t sigma);
// Scratch bytes of one contraction (banded matrix, partial columns, byte sums); 0 if it does not apply.
size_t cc_scratch_bytes(uint32_t n, uint32_t sigma);

struct Program;
// P[y], Q[y] for y < 2^sigma from W (2^sigma rows of 2^n elements), U, V (2^n
// each); scratch holds cc_scratch_bytes(n, sigma) bytes, 256-byte aligned.
void emit_copy_contract_mfma(Program& pg, const Fr* W, const Fr* U, const Fr* V, Fr* Pt, Fr* Qt, uint32_t n,
                             uint32_t sigma, void* scratch);
void launch_cc_step(const Step& st, hipStream_t s);

}  // namespace gkr
