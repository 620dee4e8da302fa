/*
 * gkr.h - C ABI of the MI355X data-parallel GKR prover.
 *
 * The library proves that `outputs = C(inputs)` for a layered arithmetic
 * circuit C made of 2^n identical copies of one sub-circuit of fan-in-2 ADD
 * and MUL gates, over the BN254 scalar field. Layer 0 is the output layer and
 * layer d the input layer; gate layer i reads layer i+1 (GKR section of the
 * paper: the layer relation V_i(g) = sum add_i(g,x,y)(V(x)+V(y)) +
 * mult_i(g,x,y) V(x)V(y)). Each layer is reduced with the two-phase
 * linear-time product sumcheck (Libra section) over bookkeeping tables; the
 * copy bits are bound after the sub-circuit bits, the order of the
 * distributed multilinear-product sumcheck (Section 3.2.1) on one worker.
 *
 * Conventions shared by every entry point
 *   - Field elements at the boundary are gkr_fr: the canonical value (< p)
 *     as 8 little-endian 32-bit limbs. Montgomery form never crosses the ABI.
 *   - Gate g = z * 2^n + c is gate z of copy c (copy index in the low bits).
 *     A gate of layer i reads gates x*2^n + c and y*2^n + c of layer i+1.
 *   - Points are given with variable 1 first; variable 1 is the most
 *     significant index bit, so the sub-circuit bits come before the copy bits.
 *   - Pointers named d_* are device pointers (memory from hipMalloc or a torch
 *     CUDA tensor); all other pointers are host pointers. The caller owns every
 *     buffer; the library never frees caller memory and keeps no pointer to a
 *     caller buffer after a call returns.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is queued asynchronously on that stream; the host
 *     returns as soon as it is queued. The proving entry points
 *     (gkr_prove_circuit, gkr_transcript_init, gkr_output_claim,
 *     gkr_prove_layer, gkr_plan_reset, gkr_run_batch) allocate no device
 *     memory, do not synchronise the stream and copy nothing between host and
 *     device, so a whole proof can be captured in a HIP graph. The set-up and
 *     convenience calls that do (gkr_circuit_create, gkr_plan_create,
 *     gkr_plan_progress, gkr_prove_batch) say so below.
 *   - Every entry point returns GKR_OK (0) or a negative status; on failure
 *     gkr_last_error() returns a message for the calling thread. No C++
 *     exception crosses the ABI. Entry points that fail leave caller buffers
 *     unspecified but never write outside them.
 *
 * Fiat-Shamir transcript (non-interactive form of the verifier's challenges):
 *   init           st = SHA256("SISU-GKR-v1" || LE64(seed))
 *   absorb(t, m)   st = SHA256(st || t || m), t a four-byte tag
 *   accept         v = LE(st) mod 2^254; while v >= p: st = SHA256(st || "GKRC"), recompute v;
 *                  the challenge is v * 2^-256 mod p
 *   squeeze        st = SHA256(st || "GKRC"), then accept
 *   round(e0, e2)  st = C(st, LE(e0 * 2^256 mod p) || LE((e2 * 2^256 mod p) + 2^254)), then accept
 * C is the SHA-256 compression function with st as chaining value and one
 * 64-byte block (bit 254 of the second value, free since values are below p,
 * marks a round block). Statement: absorb("GKRD", circuit digest),
 * absorb("GKRD", tree digest of the inputs), absorb("GKRD", tree digest of the
 * outputs); tree digests hash 1 KiB chunks and then the concatenated chunk
 * digests, recursively. The round challenge is that of round(e0, e2) (e1 is
 * fixed by the running claim, e1 = claim - e0); a phase's final value is
 * absorbed with "GKRV". Challenges alpha, beta and the output point come from
 * squeeze.
 *
 * Proof layout: for each gate layer i = 0..d-1 with s' = s_{i+1}:
 *   s' phase-1 messages (e0, e1, e2: the round polynomial at t = 0, 1, 2),
 *   vx, s' phase-2 messages, vy  -- (6 s' + 2) * 32 bytes, canonical elements.
 */
#ifndef GKR_H
#define GKR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GKR_OK 0
#define GKR_EINVAL (-1)       /* bad argument, shape or buffer size          */
#define GKR_ENOMEM (-2)       /* host or device allocation failed            */
#define GKR_EDEVICE (-3)      /* a HIP call or kernel launch failed          */
#define GKR_EBUFSZ (-4)       /* an output or workspace buffer is too small  */
#define GKR_EUNSUPPORTED (-5) /* shape beyond the supported limits           */

#define GKR_GATE_ADD 0u
#define GKR_GATE_MUL 1u

/* Fields (Section 4.1, choice of the finite field: BN254, or Goldilocks
 * p = 2^64 - 2^32 + 1, faster for the prover but without pairings). */
#define GKR_FIELD_BN254 0u
#define GKR_FIELD_GOLDILOCKS 1u

/* Largest supported log2 layer width s_i = sigma_i + n, and copy count n. */
#define GKR_MAX_LOG_WIDTH 30u
#define GKR_MAX_LOG_COPIES 24u
#define GKR_MAX_DEPTH 4096u

/* An element of the BN254 scalar field Fr, the field the paper proves over
 * (Section 4.1, choice of the finite field): the canonical value (< p) as
 * eight little-endian 32-bit limbs. */
typedef struct {
  uint32_t limb[8];
} gkr_fr;

/* One gate of a sub-circuit (Section 2.2: a gate of layer i adds or
 * multiplies two values of layer i+1, which the wiring predicates add_i and
 * mult_i encode): inputs x, y index the next layer of the same copy; type is
 * GKR_GATE_ADD or GKR_GATE_MUL. `reserved` is ignored. 12 bytes. */
typedef struct {
  uint32_t x, y;
  uint8_t type;
  uint8_t reserved[3];
} gkr_gate;

/* The Fiat-Shamir transcript state: the SHA-256 chaining value as 32 bytes
 * (eight big-endian words). The paper's protocol is interactive (the
 * verifier sends a random challenge after every round, Section 3.2.1); this
 * state carries the non-interactive form of those challenges described at the
 * top of this file. The entry points below take it in device memory. */
typedef struct {
  uint8_t state[32];
} gkr_transcript;

/* One nested gate of a general circuit (Section 2.7, general arithmetic
 * circuit: a gate may read any later layer as long as one input is in the
 * next layer; Section 3.4.3, accumulation gate: a gate holds a list of nested
 * fan-in-2 gates, possibly of different types and reading different layers,
 * and its value is their sum). In gate layer i: output gate z, left input x
 * in layer i+1, right input y in layer src (i < src <= depth); type
 * GKR_GATE_ADD or GKR_GATE_MUL; `reserved` is ignored. 20 bytes. Copies as
 * for gkr_gate: gate z of copy c reads x*2^n + c and y*2^n + c. */
typedef struct {
  uint32_t z, x, src, y;
  uint8_t type;
  uint8_t reserved[3];
} gkr_nested_gate;

typedef struct gkr_circuit gkr_circuit;

/* Message describing the last failure on the calling thread ("" if none). */
const char* gkr_last_error(void);

/*
 * Create a circuit (Section 2.2: a layered circuit, layer 0 the output and
 * layer d the input; Section 3.2: 2^n identical sub-circuits, one per worker
 * share, here one copy index): `depth` gate layers (1..GKR_MAX_DEPTH),
 * 2^log_copies copies, log_sub_width[0..depth] = sigma_i (layer 0 = output,
 * [depth] = input), gates[i] = 2^{sigma_i} gates of layer i's sub-circuit
 * (host memory, copied). Validates every index, builds the wiring indexes by x and by y,
 * uploads them to the current device and computes the circuit digest. The
 * circuit is immutable and may be used from several streams at once. When no
 * HIP device is present the circuit is created host-only: gkr_verify works
 * and every proving call returns GKR_EDEVICE.
 * Errors: GKR_EINVAL (bad shape or gate), GKR_EUNSUPPORTED (too large),
 * GKR_ENOMEM, GKR_EDEVICE.
 */
int32_t gkr_circuit_create(uint32_t depth, uint32_t log_copies, const uint32_t* log_sub_width,
                           const gkr_gate* const* gates, gkr_circuit** out);
void gkr_circuit_destroy(gkr_circuit* circuit);

/*
 * Create a layered circuit over a chosen field (Section 4.1, choice of the
 * finite field). GKR_FIELD_BN254 is gkr_circuit_create. GKR_FIELD_GOLDILOCKS
 * gives a circuit proved by gkr_gl_prove_circuit and verified by
 * gkr_gl_verify over p = 2^64 - 2^32 + 1, with canonical uint64_t elements
 * (8 bytes; the same wiring, circuit digest and protocol steps) and the
 * transcript rules of that field:
 *   init           st = SHA256("SISU-GKR-GL-v1" || LE64(seed))
 *   accept         v = LE64(st[0..7]); while v >= p: st = SHA256(st || "GKRC"), recompute;
 *                  the challenge is v
 *   squeeze        st = SHA256(st || "GKRC"), then accept
 *   round(e0, e2)  st = C(st, LE64(e0) || LE64(e2) || 47 zero bytes || 0x01), then accept
 *   values         vx, vy absorbed with "GKRV" as 8 bytes; statement as for BN254 with
 *                  8-byte elements in the tree digests.
 * Proof layout as for BN254 with 8-byte elements: (6 s_{i+1} + 2) * 8 bytes
 * per layer. gkr_workspace_bytes and gkr_proof_bytes report the Goldilocks
 * sizes; the BN254 proving calls and gkr_verify refuse such a circuit.
 * Errors: as gkr_circuit_create, and GKR_EINVAL for an unknown field.
 */
int32_t gkr_circuit_create_field(uint32_t field, uint32_t depth, uint32_t log_copies,
                                 const uint32_t* log_sub_width, const gkr_gate* const* gates,
                                 gkr_circuit** out);

/*
 * Whole proof of a Goldilocks circuit (Section 2.2 as for gkr_prove_circuit):
 * d_inputs 2^{s_d} canonical uint64_t (< p; device, 16-byte aligned: the
 * rounds read it in 16-byte pairs), d_outputs receives 2^{s_0} elements,
 * d_proof gkr_proof_bytes() bytes (device, 8-byte aligned). The workspace,
 * stream and error conventions are gkr_prove_circuit's.
 */
int32_t gkr_gl_prove_circuit(const gkr_circuit* circuit, const uint64_t* d_inputs, uint64_t seed,
                             uint64_t* d_outputs, uint8_t* d_proof, size_t proof_cap, size_t* proof_len,
                             void* d_ws, size_t ws_bytes, void* stream);

/*
 * Verifier of a Goldilocks proof (Section 2.2 and the round check of Section
 * 3.2.1, as gkr_verify): host buffers, synchronous; 1 accept, 0 reject,
 * GKR_EINVAL for a proof of the wrong length or a non-canonical element.
 */
int32_t gkr_gl_verify(const gkr_circuit* circuit, const uint64_t* inputs, const uint64_t* outputs,
                      uint64_t seed, const uint8_t* proof, size_t proof_len);

/*
 * Create a general circuit (Sections 2.7 and 3.4.3, see gkr_nested_gate):
 * `depth` gate layers, 2^log_copies copies, log_sub_width[0..depth] = sigma_i,
 * counts[i] >= 1 nested gates of gate layer i at gates[i] (host memory,
 * copied; any order). Gate z of layer i is the sum of its nested gates (0 if
 * it has none). For a pair of layers only the gates the reading layer uses
 * are indexed: layer i's right inputs are proved over the concatenation of
 * the used gates of each source layer (increasing source layer, each block
 * 2^tau_i entries, zero padded), and the prover then sends every block's
 * value at the local part of the phase-2 point; those values are claims on
 * the source layers, combined at the start of each layer with squeezed
 * coefficients. Proof of layer i: s_{i+1} phase-1 messages, vx, rho_i
 * phase-2 messages (rho_i = block bits + tau_i + n), vy, then one value per
 * source layer; the circuit digest is SHA256("GKR-GENERAL-v1" || LE32 depth,
 * log_copies, sigma_0..sigma_depth || per gate layer LE32 count || per nested
 * gate LE32 z, x, src, y || u8 type). gkr_prove_circuit, the no-allocation
 * variant, gkr_transcript_init, gkr_output_claim and gkr_verify accept the
 * result; gkr_prove_layer and the batch calls return GKR_EUNSUPPORTED for it.
 * A gate layer may be read by at most 13 earlier layers. Errors: GKR_EINVAL
 * (bad shape or nested gate), GKR_EUNSUPPORTED (too large), GKR_ENOMEM,
 * GKR_EDEVICE.
 */
int32_t gkr_general_circuit_create(uint32_t depth, uint32_t log_copies, const uint32_t* log_sub_width,
                                   const uint64_t* counts, const gkr_nested_gate* const* gates,
                                   gkr_circuit** out);

/* Device workspace one proof needs (layer store + bookkeeping tables + state). */
size_t gkr_workspace_bytes(const gkr_circuit* circuit);
/* Bytes of a whole proof, and of gate layer `layer`'s part: (6 s_{layer+1} + 2) * 32. */
size_t gkr_proof_bytes(const gkr_circuit* circuit);
size_t gkr_layer_proof_bytes(const gkr_circuit* circuit, uint32_t layer);
/* Field-gate count of one proof: sum over gate layers of 2^{s_i}. */
uint64_t gkr_gate_layers(const gkr_circuit* circuit);

/*
 * Whole proof (Section 2.2: the prover evaluates the circuit, then reduces
 * the claim about the outputs layer by layer to a claim about the inputs;
 * each layer as in gkr_prove_layer): forward evaluation, statement binding,
 * output claim, every layer. d_inputs: 2^{s_d} canonical inputs. Writes d_outputs (2^{s_0}
 * elements) and the proof into d_proof (device, proof_cap bytes);
 * *proof_len (host) receives gkr_proof_bytes(). d_ws: gkr_workspace_bytes()
 * bytes of device memory owned by this call until the stream reaches its end;
 * concurrent proofs need separate workspaces.
 * Inputs must be canonical (< p); non-canonical inputs give an unspecified
 * (but in-bounds) result. Errors: GKR_EINVAL, GKR_EBUFSZ (proof_cap or
 * ws_bytes too small), GKR_EDEVICE.
 */
int32_t gkr_prove_circuit(const gkr_circuit* circuit, const gkr_fr* d_inputs, uint64_t seed,
                          gkr_fr* d_outputs, uint8_t* d_proof, size_t proof_cap, size_t* proof_len,
                          void* d_ws, size_t ws_bytes, void* stream);

/*
 * gkr_prove_circuit without a caller workspace, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). The workspace is a static device array
 * of GKR_NOALLOC_WORKSPACE_BYTES (256 MiB) that every GPU the library runs on
 * holds until the process ends; the call itself allocates nothing, and the
 * caller still passes inputs, outputs and the proof buffer as for
 * gkr_prove_circuit (same bytes, same errors). Circuits whose
 * gkr_workspace_bytes() exceeds GKR_NOALLOC_WORKSPACE_BYTES are rejected with
 * GKR_EUNSUPPORTED; the current device must be the circuit's (GKR_EINVAL).
 * Every call on one GPU shares that GPU's array: calls whose device work
 * overlaps (streams with no ordering between them) race; calls on one stream
 * are ordered. The array needs no clearing between calls.
 */
#define GKR_NOALLOC_WORKSPACE_BYTES (256ull << 20)
int32_t gkr_prove_circuit_noalloc(const gkr_circuit* circuit, const gkr_fr* d_inputs, uint64_t seed,
                                  gkr_fr* d_outputs, uint8_t* d_proof, size_t proof_cap, size_t* proof_len,
                                  void* stream);

/*
 * Bind the statement (Section 2.2: the prover claims that the outputs are the
 * circuit evaluated on the inputs; the challenges that follow must depend on
 * that statement): d_transcript (device) receives the transcript state after
 * init(seed) and the three "GKRD" absorbs. d_inputs / d_outputs are the
 * canonical input (2^{s_d}) and output (2^{s_0}) vectors.
 */
int32_t gkr_transcript_init(const gkr_circuit* circuit, uint64_t seed, const gkr_fr* d_inputs,
                            const gkr_fr* d_outputs, gkr_transcript* d_transcript, void* d_ws,
                            size_t ws_bytes, void* stream);

/*
 * Output claim (Section 2.2: the verifier picks a random point g and the
 * protocol starts from the claim V_0~(g) about the outputs' multilinear
 * extension): squeezes g (s_0 challenges) from d_transcript (updated in
 * place) and evaluates the output MLE there. Writes d_g (s_0 elements,
 * variable 1 first) and d_claim (1 element) = V_0~(g).
 */
int32_t gkr_output_claim(const gkr_circuit* circuit, const gkr_fr* d_outputs, gkr_transcript* d_transcript,
                         gkr_fr* d_g, gkr_fr* d_claim, void* d_ws, size_t ws_bytes, void* stream);

/*
 * One gate layer (Section 2.2: the sumcheck over the layer relation reduces
 * claims about V_layer~ to claims about V_{layer+1}~ at the points r_x, r_y;
 * Section 2.3: Libra's linear-time prover runs it in two phases, x then y,
 * over bookkeeping tables; Section 3.2.1: the copy variables are bound after
 * the sub-circuit variables): reduces claims about V_layer~ to claims about
 * V_{layer+1}~.
 *   d_next      V_{layer+1}, 2^{s_{layer+1}} canonical elements
 *   d_u, d_v    points (s_layer elements each); d_v is ignored for layer 0
 *   d_claim_u/v claimed values V_layer~(u), V_layer~(v); d_claim_v ignored for layer 0
 *   d_transcript transcript state (device), read then updated in place. For
 *               layer 0 it is the state after the output point was squeezed;
 *               for later layers, after the previous layer's last absorb.
 * For layer > 0 the call squeezes alpha, beta and proves alpha*V~(u) + beta*V~(v);
 * layer 0 proves V~(u). Outputs: d_rx, d_ry (s_{layer+1} elements each),
 * d_vx = V_{layer+1}~(rx), d_vy = V_{layer+1}~(ry), and the layer's proof
 * bytes into d_layer_proof (gkr_layer_proof_bytes()). The claims must be the
 * true MLE values: the prover derives e1 of each round from the running claim.
 */
int32_t gkr_prove_layer(const gkr_circuit* circuit, uint32_t layer, const gkr_fr* d_next,
                        const gkr_fr* d_u, const gkr_fr* d_v, const gkr_fr* d_claim_u,
                        const gkr_fr* d_claim_v, gkr_transcript* d_transcript, gkr_fr* d_rx, gkr_fr* d_ry,
                        gkr_fr* d_vx, gkr_fr* d_vy, uint8_t* d_layer_proof, void* d_ws,
                        size_t ws_bytes, void* stream);

/*
 * Batched proving (many proofs at once in one persistent kernel). The paper
 * runs one prover per worker; batching many proofs in one launch is this
 * library's own (no passage defines it).
 *
 * A job names a circuit, its inputs, seed and output/proof/workspace buffers
 * (the buffers gkr_prove_circuit takes). gkr_plan_create records the job's
 * proof as a step program in device memory (allocates and copies: call it
 * outside any timed or captured region). gkr_run_batch then runs 1..64 plans
 * together: resident workgroups take tiles of whichever plan has work, so the
 * serial Fiat-Shamir steps of one proof overlap the table sweeps of the
 * others. A run allocates nothing and copies nothing between host and device
 * (graph-capturable). Each plan's proof bytes are identical to its
 * gkr_prove_circuit bytes. Buffers of different jobs must not overlap.
 */
typedef struct {
  const gkr_circuit* circuit;
  const gkr_fr* d_inputs;
  uint64_t seed;
  gkr_fr* d_outputs;
  uint8_t* d_proof;
  size_t proof_cap;
  void* d_ws;
  size_t ws_bytes;
} gkr_job;

typedef struct gkr_plan gkr_plan;

/* Record a job's proof program (GKR_EINVAL, GKR_EBUFSZ, GKR_ENOMEM, GKR_EDEVICE). */
int32_t gkr_plan_create(const gkr_job* job, gkr_plan** out);
void gkr_plan_destroy(gkr_plan* plan);
/* Queue a reset of the plan's progress so its next run proves from the start. */
int32_t gkr_plan_reset(gkr_plan* plan, void* stream);
/*
 * Queue one persistent launch over `n` (1..64) distinct plans. d_ctl: 4 device
 * words owned by this call until the stream reaches its end ([0] plans
 * finished in this launch, [1] stop flag, [2] steps completed). workgroups:
 * resident workgroups (0 = fill the device). step_budget > 0 stops the launch
 * after about that many completed steps; stop_on_finish stops it when any plan
 * finishes. A stopped launch leaves every plan resumable: run it again to
 * continue. Plans already finished are skipped.
 */
int32_t gkr_run_batch(gkr_plan* const* plans, uint32_t n, uint32_t* d_ctl, uint32_t workgroups,
                      uint32_t step_budget, uint32_t stop_on_finish, void* stream);
/* Steps completed so far and the plan's step count (synchronous device read). */
int32_t gkr_plan_progress(const gkr_plan* plan, uint32_t* done_steps, uint32_t* total_steps);
/*
 * Convenience: plans for `n` jobs, persistent runs of up to 64 plans each on
 * `stream`, then a synchronisation and cleanup. Allocates; synchronous.
 */
int32_t gkr_prove_batch(const gkr_job* jobs, uint32_t n, void* stream);

/*
 * Verifier (Section 2.2: the verifier's side of the protocol, ending with
 * the wiring predicates add~, mult~ at (r_x, r_y) and the inputs' MLE;
 * Section 3.2.1: every round's polynomial must satisfy g_j(0) + g_j(1) = the
 * running claim, which then becomes g_j(r_j)). Host only, synchronous.
 * inputs / outputs / proof are host buffers. Returns 1 (accept), 0 (reject) or a negative status for malformed
 * arguments: GKR_EINVAL for a proof of the wrong length or any element >= p.
 */
int32_t gkr_verify(const gkr_circuit* circuit, const gkr_fr* inputs, const gkr_fr* outputs,
                   uint64_t seed, const uint8_t* proof, size_t proof_len);

/*
 * Round-schedule tuning (process-wide; used by the autotuner; this library's
 * own, no passage). Proof bytes
 * never depend on it. tail_log: tables of at most 2^tail_log entries finish
 * their phase in one workgroup (1..20); max_round_blocks: cap on the
 * workgroups of one grid-wide round (1..4096); pairs_per_thread: a grid-wide
 * round gets ceil(pairs / (256 * pairs_per_thread)) workgroups, capped
 * (1..1024). Proofs read the tuning when they are queued. Errors: GKR_EINVAL
 * for a value out of range (nothing is changed). gkr_get_tuning writes the
 * current values to the non-null pointers.
 */
int32_t gkr_set_tuning(uint32_t tail_log, uint32_t max_round_blocks, uint32_t pairs_per_thread);
int32_t gkr_get_tuning(uint32_t* tail_log, uint32_t* max_round_blocks, uint32_t* pairs_per_thread);

/*
 * How plain proofs contract phase 2's copy factors (process-wide; this
 * library's own, no passage; proof bytes never depend on it): 1 (the
 * default) runs the contraction on the int8 matrix cores for layers with at
 * least 2^10 copies and 2^8 sub-circuit wires, 0 always runs the scalar
 * lazy-product pass. Proofs read it when they are queued. Errors: GKR_EINVAL
 * for a mode above 1 (nothing is changed). gkr_get_contraction writes the
 * current mode to a non-null pointer.
 */
int32_t gkr_set_contraction(uint32_t matrix_cores);
int32_t gkr_get_contraction(uint32_t* matrix_cores);

/*
 * Kernel timing for measurement (this library's own, no passage). While enabled, every launch is bracketed by
 * two HIP events on its own stream (do not enable it while capturing a HIP
 * graph). gkr_profile_read waits for the recorded events and returns, per
 * kernel class, the launch count, the summed event time, and the algorithmic
 * HBM bytes and field products the host attributed to those launches
 * (see the kernel descriptions in the design notes). Enabling resets the sums.
 */
typedef struct {
  char name[32];
  uint64_t launches;
  double ms;
  double bytes;
  double mulmods;
} gkr_profile_entry;

int32_t gkr_profile_enable(int32_t on);
int32_t gkr_profile_read(gkr_profile_entry* out, uint32_t cap, uint32_t* count);

/*
 * Microbenchmarks of the device's vector ALU and HBM (this library's own,
 * for the roofline of the prover's kernels; no passage). Runs
 * one timed launch of `iters` iterations over every compute unit on the
 * current device and writes the grid-wide rate to *ops_per_s (and the
 * launch time to *ms, if not null). kind: 0 = v_mad_u64_u32 (32x32+64 ->
 * 64), 1 = v_mad_u64_u32 with its carry into an overflow word (the
 * multiply-accumulate of the field product, one operation per pair),
 * 2 = v_add_u32 (full-rate reference), 3 = v_mul_lo_u32 / v_mul_hi_u32,
 * 4 = Montgomery field products (the prover's device product), 5 = the HBM
 * access pattern of a folding round without its arithmetic (per pair b < h =
 * 2^24: read 32-byte entries b, b+h, b+2h, b+3h of a 2 GiB table, write
 * entries b, b+h of a 1 GiB one; `iters` passes; *ops_per_s is then bytes
 * moved per second, reads plus writes). Allocates (kind 5: 3 GiB) and
 * synchronises (not for timed or captured regions). Errors: GKR_EINVAL,
 * GKR_ENOMEM, GKR_EDEVICE.
 */
int32_t gkr_ubench(uint32_t kind, uint32_t iters, double* ops_per_s, double* ms);

/*
 * Committed inputs (Section 2.4, the Virgo protocol: the prover commits to
 * the input layer's multilinear extension before the GKR protocol runs and
 * opens it at the last layer's two points, so the verifier never reads the
 * inputs; the commitment is transparent and built on a univariate sumcheck).
 * This library's construction, for N = 2^s inputs V:
 *   - f(X) = sum_b V[b] X^b; f is evaluated on the coset L = 5 <w_M>, M = 4N
 *     (w_M = 5^((p-1)/M); so s <= 26), and a table over a coset is stored in
 *     bit-reversed order: position t holds the value at 5 w_M^bitrev(t).
 *   - Merkle trees: leaf u covers positions 2u, 2u + 1 of a table (64 bytes:
 *     the Montgomery forms e 2^256 mod p, 32 bytes little-endian each) or of
 *     two tables (128 bytes, h then g'); a leaf digest is the SHA-256
 *     compression function chained from the initial hash value over its
 *     64-byte blocks (no padding), a node the compression of left || right.
 *   - The statement absorbs ("GKRD", root of f) in place of the input
 *     digest. After the last layer, with points rx, ry and claims vx, vy:
 *     lam = squeeze, c = vx + lam vy = sum_b V[b] w[b], w = eq(rx, .) +
 *     lam eq(ry, .); q(X) = sum_b w[b] X^((N - b) mod N) (the verifier
 *     evaluates it in O(s): q(x) = x^N Q(1/x) + (1 - x^N) Q(0), Q(Y) =
 *     prod_j ((1 - rx_j) + rx_j Y^(2^(s-j))) + lam prod_j (same with ry));
 *     the prover splits f q = c + X g' + (X^N - 1) h (deg g', h < N - 1),
 *     absorbs ("GKRM", root of (h, g')), squeezes a0..a3, and runs FRI on
 *     R = a0 f + a1 h + a2 g' + a3 X g' (degree < N): for i < s, beta_i =
 *     squeeze, fold R_{i+1}(x^2) = (R_i(x) + R_i(-x)) / 2 + beta_i (R_i(x) -
 *     R_i(-x)) / (2x), and for i + 1 < s absorb ("GKRM", root of R_{i+1});
 *     the constant R_s is absorbed with "GKRV"; then `queries` leaves u_j =
 *     squeeze mod (M / 2) of the first layer.
 *   - Proof: root of f || the layered proof (layout above) || root of (h, g')
 *     || roots of R_1..R_{s-1} || R_s || per query: f leaf (2 elements) and
 *     its path (s + 1 digests), (h, g') leaf (4 elements) and path, and for
 *     i = 1..s-1 the leaf u_j >> i of R_i (2 elements) and its path (s + 1 - i
 *     digests); paths bottom-up, elements canonical, digests as SHA-256 bytes.
 *
 * gkr_committed_sizes: workspace and proof bytes of a committed proof of a
 * layered BN254 circuit with depth >= 1 and 2^1 .. 2^26 inputs, for 1 ..
 * GKR_MAX_QUERIES queries (either output may be NULL). Errors:
 * GKR_EUNSUPPORTED (general or Goldilocks circuit, input count out of range),
 * GKR_EINVAL.
 */
#define GKR_MAX_QUERIES 256u
int32_t gkr_committed_sizes(const gkr_circuit* circuit, uint32_t queries, size_t* ws_bytes,
                            size_t* proof_bytes);

/*
 * The committed-input proof of outputs = C(inputs) (Section 2.4 with the
 * layered proof of gkr_prove_circuit between commitment and opening).
 * d_inputs, d_outputs, d_proof, d_ws as for gkr_prove_circuit (16-byte
 * aligned device buffers; the workspace of gkr_committed_sizes, 16-byte
 * aligned); proof_cap >= the proof bytes. Queued on `stream`; allocates
 * nothing. Errors: GKR_EINVAL, GKR_EBUFSZ, GKR_EUNSUPPORTED, GKR_EDEVICE.
 */
int32_t gkr_prove_circuit_committed(const gkr_circuit* circuit, const gkr_fr* d_inputs, uint64_t seed,
                                    uint32_t queries, gkr_fr* d_outputs, uint8_t* d_proof, size_t proof_cap,
                                    void* d_ws, size_t ws_bytes, void* stream);

/*
 * Verifier of a committed-input proof (the GKR round and layer checks of
 * gkr_verify, then the opening: Merkle paths, the identity
 * f(x) q(x) = c + x g'(x) + (x^N - 1) h(x) at each queried x and -x, and the
 * FRI folds down to R_s). It reads the outputs but not the inputs: host
 * buffers, synchronous; 1 accept, 0 reject, GKR_EINVAL for a proof of the
 * wrong length or a non-canonical element in the layered part.
 */
int32_t gkr_verify_committed(const gkr_circuit* circuit, const gkr_fr* outputs, uint64_t seed, uint32_t queries,
                             const uint8_t* proof, size_t proof_len);

/*
 * The commitment alone (Section 2.4's commit step) to 2^log_n canonical
 * values d_values (device, 1 <= log_n <= 26): writes the 32-byte root to
 * d_root (device). gkr_vpd_workspace_bytes gives the workspace size (device,
 * 16-byte aligned). Queued on `stream`; allocates nothing. Errors:
 * GKR_EUNSUPPORTED, GKR_EINVAL, GKR_EBUFSZ, GKR_EDEVICE.
 */
int32_t gkr_vpd_workspace_bytes(uint32_t log_n, size_t* bytes);
int32_t gkr_vpd_commit(uint32_t log_n, const gkr_fr* d_values, uint8_t* d_root, void* d_ws, size_t ws_bytes,
                       void* stream);

#ifdef __cplusplus
}
#endif

#endif /* GKR_H */
