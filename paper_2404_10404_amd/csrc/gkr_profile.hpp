// Optional per-kernel-class timing with HIP events (off unless enabled).
#pragma once

#include <hip/hip_runtime.h>

namespace gkr {

enum ProfClass {
  PC_FORWARD = 0,
  PC_DIGEST,
  PC_TRANSCRIPT,
  PC_EQ,
  PC_CLAIM,
  PC_PHASE1_INIT,
  PC_ROUND_A,
  PC_ROUND_B,
  PC_TAIL_A,
  PC_TAIL_B,
  PC_PHASE2_TABLES,
  PC_COPY_CONTRACT,
  PC_LOCAL_CONTRACT,
  PC_SMALL,
  PC_CONVERT,
  PC_BATCH,
  PC_G_GATHER,
  PC_G_FORWARD,
  PC_G_CLAIMS,
  PC_G_PHASE1_INIT,
  PC_G_PHASE2_TABLES,
  PC_VPD_NTT,
  PC_VPD_MERKLE,
  PC_VPD_FRI,
  PC_VPD_OTHER,
  PC_COUNT
};

bool prof_on();
// Bracket one launch: prof_begin returns a token (-1 when off).
int prof_begin(hipStream_t s);
// bytes: algorithmic HBM bytes of the launch; mulmods: field products it needs.
void prof_end(int token, hipStream_t s, ProfClass cls, double bytes, double mulmods);

}  // namespace gkr
