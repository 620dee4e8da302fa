// Entry points of the Goldilocks-field prover (gkr_gl.hip) shared with the
// host driver.
#pragma once

#include <hip/hip_runtime.h>

#include "gkr_internal.hpp"

namespace gkr {

void launch_gl_step(const Step& st, hipStream_t s);
// Workspace layout of a Goldilocks circuit (fills c.gl and c.plan.total).
void plan_gl_workspace(gkr_circuit& c);
size_t gl_proof_bytes(const gkr_circuit& c);

}  // namespace gkr
