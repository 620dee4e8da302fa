// The commitment to the input layer and its opening at the last layer's two
// points (Section 2.4, Virgo's polynomial delegation): shared declarations of
// the device program (gkr_vpd.hip), the launcher and the host verifier.
//
// The inputs V (N = 2^s values) are the coefficients of f(X) = sum_b V[b] X^b.
// f is committed by a Merkle tree over its values on the coset L = 5 <w_M>,
// M = 4N, stored in bit-reversed order; the two claims are combined with a
// squeezed lam and opened by a univariate sumcheck (p = f q = c + X g' +
// (X^N - 1) h) whose low-degree test is FRI on R = a0 f + a1 h + a2 g' + a3 X g'.
#pragma once

#include <stdint.h>

#include <vector>

#include "fr.hpp"
#include "gkr_internal.hpp"

namespace gkr {

constexpr uint32_t kVpdLogBlowup = 2;
constexpr uint32_t kVpdMaxLogN = 26;         // M = 4N <= 2^28, the 2-adicity of p - 1
constexpr uint32_t kVpdMaxQueries = GKR_MAX_QUERIES;
constexpr uint32_t kVpdLoBits = 13;          // split of the exponent in the two-level power tables
constexpr uint32_t kTagCommit = 0x474B524Du; // "GKRM"

// Device scalars of an opening (Montgomery form).
struct VpdState {
  Fr lam;
  Fr a[4];
  Fr beta[kVpdMaxLogN];
  uint32_t idx[kVpdMaxQueries];  // query leaves of the first layer
};

// Workspace layout of a commitment and an opening for s = log2 N (offsets in bytes).
struct VpdPlan {
  uint32_t s = 0, queries = 0;
  uint64_t N = 0, M = 0;
  size_t off_T, off_wlo, off_whi, off_wilo, off_wihi, off_glo, off_ghi;
  size_t off_fL, off_hL, off_gL, off_fri, off_treeF, off_treeHG, off_treeFri;
  size_t off_EA, off_EB, off_EC, off_ED, off_state;
  size_t total;
};

// Plan of the commitment region for 2^s values and `queries` queries.
VpdPlan plan_vpd(uint32_t s, uint32_t queries, uint32_t n_copy_bits);
// Bytes of an opening (after the GKR layers of a committed proof).
size_t vpd_opening_bytes(uint32_t s, uint32_t queries);

// Host constants (Montgomery form).
Fr vpd_root_of_unity(uint32_t log_m);  // generator of the order-2^log_m subgroup
Fr vpd_shift();                        // the coset shift 5
Fr fr_pow_u64(const Fr& base, uint64_t e);
Fr fr_inverse(const Fr& a);

struct Program;

// Commitment of the Montgomery-form values d_vals (2^s of them) into the
// region `base` planned by plan_vpd: twiddles, f on L, its Merkle tree; the
// root's 8 words land at the top of the tree (vpd_root_words).
void emit_vpd_commit(Program& pg, const VpdPlan& vp, void* base, const Fr* d_vals);
const uint32_t* vpd_root_words(const VpdPlan& vp, const void* base);
// Opening at the points rx, ry (device arrays of s Montgomery elements) on
// the transcript in S; the claims themselves are the verifier's business.
// proof_out receives vpd_opening_bytes(s, queries) bytes. sigma, n: the split
// of the s variables into sub-circuit and copy bits (local bits first).
void emit_vpd_open(Program& pg, const VpdPlan& vp, void* base, const Fr* d_vals, DevState* S, const Fr* rx,
                   const Fr* ry, uint32_t sigma, uint32_t n, uint8_t* proof_out);
// Writes the commitment root (32 bytes) to proof_out.
void emit_vpd_root_out(Program& pg, const VpdPlan& vp, void* base, uint8_t* proof_out);

void launch_vpd_step(const Step& st, hipStream_t s);

}  // namespace gkr
