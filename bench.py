"""Benchmark: GKR prover field-gates/s, batched vs plain, and serving p50/p99
latency, on one MI355X.

A step is one whole proof (forward evaluation, statement binding, output claim
and every layer's two sumcheck phases) of the workload over inputs already in
HBM. `value` = field gates (sum over gate layers of 2^{s_i}) x steps / wall time.

Default workload (c3): the single-worker share at its real shape, 2^12
identical copies of a depth-24 sub-circuit with 2^14 gates per layer (2^26
gates per layer), 30% MUL gates, seed 3. --workload c2: 2^8 copies x depth 16
x 2^12 gates; c1: one depth-4 circuit of 2^10 gates per layer.

The default line also carries:
  roofline      the dominant kernel class (HIP events around each launch
                during a separate timed pass on the proof's stream) against
                the HBM peak or the integer-multiply peak measured live by
                the library's microbenchmark (gkr_ubench);
  batched       64 uneven jobs: sequential plain proofs, sequential HIP-graph
                replays, one persistent launch (proofs vs the oracle's
                digests);
  serving       a Poisson trace of the serving mix (256 jobs by default):
                plain one-at-a-time loop vs continuous batching, p50/p99;
  cpu_baseline  the oracle on a bounded slice of the same workload.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import gkr_synth as gs  # noqa: E402

HBM_PEAK_GBS = 8000.0
# Full-rate 32-bit VALU issue (theoretical): 256 CUs x 4 SIMDs x 32 lanes x
# 2.4 GHz (the 157.3 TFLOP/s fp32 vector rate counted as single operations).
# The roofline uses the measured v_mad_u64_u32 rate instead.
VALU_PEAK_TOPS = 256 * 4 * 32 * 2.4e9 / 1e12
# 32x32 multiply-accumulates of one schoolbook Montgomery product with 8 limbs
# (64 for the product, 64 + 8 for the reduction).
MACS_PER_MULMOD = 2 * 8 * 8 + 8


def log(msg):
    """Progress on stderr (stdout carries only the JSON line)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


def alu_peaks(gkr):
    """Integer-multiply peaks measured on this device by gkr_ubench."""
    out = {}
    for kind, key in ((0, "mad_u64_u32_per_s"), (1, "mac_pair_per_s"), (2, "add_u32_per_s"),
                      (3, "mul_u32_per_s"), (4, "field_products_per_s")):
        rate, ms = gkr.ubench(kind, 1024 if kind < 4 else 64)
        out[key] = rate
    # the HBM stream of a folding round without its arithmetic (8 passes of 3 GiB)
    out["round_stream_bytes_per_s"] = gkr.ubench(5, 8)[0]
    return out

WORKLOADS = {
    "c1": (gs.plain_c1, "plain circuit: depth 4, 2^10 gates/layer"),
    "c2": (gs.data_parallel_c2, "data-parallel: 2^8 copies x (depth 16, 2^12 gates/layer) = 2^20 gates/layer"),
    "c3": (gs.worker_share_c3, "single-worker share: 2^12 copies x (depth 24, 2^14 gates/layer) = 2^26 gates/layer, 30% MUL"),
}


class ProfEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_uint64), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("mulmods", ctypes.c_double)]


def profile_pass(gkr, prover, d_in, seed, steps):
    import torch
    L = gkr.lib()
    L.gkr_profile_enable.argtypes = [ctypes.c_int32]
    L.gkr_profile_read.argtypes = [ctypes.POINTER(ProfEntry), ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]
    torch.cuda.synchronize()
    L.gkr_profile_enable(1)
    for _ in range(steps):
        prover.prove(d_in, seed)
    torch.cuda.synchronize()
    arr = (ProfEntry * 32)()
    cnt = ctypes.c_uint32(0)
    L.gkr_profile_read(arr, 32, ctypes.byref(cnt))
    L.gkr_profile_enable(0)
    out = {}
    for i in range(cnt.value):
        e = arr[i]
        out[e.name.decode()] = {"launches": e.launches // steps, "ms": e.ms / steps,
                                "bytes": e.bytes / steps, "mulmods": e.mulmods / steps}
    return out


# Profile class -> kernel, for the traffic records taken with rocprofv3 --pmc.
CLASS_KERNEL = {"round": "k_round_a", "round_sub": "k_round_b", "tail": "k_tail_a", "tail_sub": "k_tail_b",
                "phase1_init": "k_p1_init_round", "forward": "k_forward", "copy_contract": "k_cc_gemm",
                "local_contract": "k_local_contract", "digest": "k_digest", "g_gather": "k_g_gather",
                "g_forward": "k_g_forward", "g_claim_tables": "k_g_ttable", "g_phase1_init": "k_g_p1",
                "g_phase2_tables": "k_g_p2"}
KERNEL_SOURCES = ["fr.hpp", "sha256.hpp", "gkr_device.hpp", "gkr_kernels.hpp", "gkr_bodies.hpp", "gkr_kernels.hip"]
# The Goldilocks prover's classes and the sources its kernels are built from.
GL_CLASS_KERNEL = {"round": "k_gl_round<3>", "round_sub": "k_gl_round<5>", "tail": "k_gl_tail<3>",
                   "tail_sub": "k_gl_tail<5>", "phase1_init": "k_gl_p1", "phase2_tables": "k_gl_p2t",
                   "forward": "k_gl_forward", "digest": "k_gl_digest", "copy_contract": "k_gl_copy_contract",
                   "local_contract": "k_gl_local_contract"}
GL_KERNEL_SOURCES = ["fr.hpp", "sha256.hpp", "gkr_device.hpp", "gkr_kernels.hpp", "gkr_bodies.hpp", "gl.hpp", "gkr_gl.hip"]


def kernel_sources_digest(sources=None):
    h = hashlib.sha256()
    for name in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2404_10404_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_record(kernel, workload, sources=None):
    """HBM bytes per launch measured by rocprofv3 (FETCH_SIZE, WRITE_SIZE runs,
    scaled by a plain copy of known size), from the summaries under profiles/;
    None when no record exists or the kernel sources changed since."""
    d = os.path.join(ROOT, "profiles")
    if not os.path.isdir(d):
        return None
    digest = kernel_sources_digest(sources)
    for name in sorted(os.listdir(d)):
        if not name.endswith(".md"):
            continue
        with open(os.path.join(d, name)) as f:
            for line in f:
                if line.startswith("traffic-record:"):
                    rec = json.loads(line[len("traffic-record:"):])
                    if rec.get("kernel") == kernel and rec.get("workload") == workload:
                        if rec.get("sources_sha256") != digest:
                            return None
                        return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
    return None


def roofline(prof, workload=None, mac_peak_tops=None, macs_per_mulmod=MACS_PER_MULMOD, class_kernel=None,
             sources=None, stream_gbs=None):
    """Roofline of the dominant kernel class: t_roof = max(bytes / HBM peak,
    multiply-adds / integer-multiply peak); the bound is the larger term.
    The integer peak is the measured v_mad_u64_u32 rate when given; a field
    product counts macs_per_mulmod 32x32 multiply-adds (136 for BN254's
    8-limb Montgomery product, 4 for a Goldilocks 64 x 64 product). With
    stream_gbs (the measured rate of a folding round's access pattern alone,
    gkr_ubench kind 5) the HBM rate is also given as a fraction of it."""
    name, e = max(prof.items(), key=lambda kv: kv[1]["ms"])
    sec = e["ms"] / 1e3
    gbs = e["bytes"] / sec / 1e9
    tops = e["mulmods"] * macs_per_mulmod / sec / 1e12
    alu_peak = mac_peak_tops if mac_peak_tops else VALU_PEAK_TOPS
    t_hbm = e["bytes"] / (HBM_PEAK_GBS * 1e9)
    t_alu = e["mulmods"] * macs_per_mulmod / (alu_peak * 1e12)
    if t_hbm >= t_alu:
        r = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gbs / HBM_PEAK_GBS, 4)}
    else:
        r = {"bound": "alu", "achieved": round(tops, 3), "peak": round(alu_peak, 3),
             "unit": "TOP/s (32x32 multiply-adds)", "frac": round(tops / alu_peak, 4),
             "peak_source": "measured v_mad_u64_u32 rate (gkr_ubench kind 0)" if mac_peak_tops
             else "theoretical full-rate VALU"}
    r["alu_frac"] = round(tops / alu_peak, 4)
    r["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
    if stream_gbs:
        r["hbm_stream_gbs"] = round(stream_gbs, 1)
        r["hbm_frac_of_stream"] = round(gbs / stream_gbs, 4)
    r.update({"kernel": name, "launches_per_step": e["launches"],
              "avg_launch_us": round(e["ms"] * 1e3 / max(1, e["launches"]), 2),
              "hbm_gbs": round(gbs, 1), "alu_tops": round(tops, 3),
              "algorithmic_bytes_per_launch": round(e["bytes"] / max(1, e["launches"]))})
    kern = (class_kernel or CLASS_KERNEL).get(name)
    t = traffic_record(kern, workload, sources) if kern and workload else None
    r["traffic"] = None if t is None else round(t)
    return r


def class_fractions(prof, mac_peak_tops, product_rate=None, macs_per_mulmod=MACS_PER_MULMOD, top=6):
    """Per kernel class (the longest ones): time, launches and the fractions of
    the HBM peak, of the measured v_mad_u64_u32 rate (products x multiply-adds
    per product) and, when given, of the measured whole field-product rate
    (gkr_ubench kind 4: the product runs at its multiply-add-with-carry pair
    rate, below the bare multiply-add rate)."""
    out = {}
    for name, e in sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:top]:
        sec = e["ms"] / 1e3
        if sec <= 0:
            continue
        d = {"ms": round(e["ms"], 3), "launches": e["launches"],
             "hbm_frac": round(e["bytes"] / sec / 1e9 / HBM_PEAK_GBS, 4)}
        if e["mulmods"] and mac_peak_tops:
            d["alu_frac"] = round(e["mulmods"] * macs_per_mulmod / sec / 1e12 / mac_peak_tops, 4)
        if e["mulmods"] and product_rate:
            d["product_frac"] = round(e["mulmods"] / sec / product_rate, 4)
        out[name] = d
    return out


def cpu_baseline(spec, budget_s=20.0):
    """The oracle (pure Python, one core) on a slice of the workload with fewer
    copies; its rate carries over to the whole workload (the prover is linear
    in the gate count), so a full proof's oracle time is extrapolated."""
    from oracle import circuit as oc
    from oracle import prover as op
    n = 0
    # grow the slice while a proof is expected to stay within the budget
    sample = None
    t_used = 0.0
    while True:
        sl = gs.copy_slice(spec, n)
        wiring = gs.make_wiring(sl)
        inputs = gs.elements_to_ints(gs.make_inputs(sl))
        c = oc.Circuit.from_synth(sl, wiring)
        t0 = time.perf_counter()
        op.prove(c, inputs, sl.seed)
        dt = time.perf_counter() - t0
        sample = (sl, dt)
        t_used += dt
        if n >= spec.log_copies or t_used + 2.2 * dt > budget_s:
            break
        n += 1
    sl, dt = sample
    rate = sl.gate_layers / dt
    out = {"value": round(rate, 1), "unit": "field-gates/s", "cores": 1, "kind": "oracle",
           "sample": "oracle proof of the same sub-circuit with 2^%d of the 2^%d copies (%d gate-layers) in %.1f s"
                     % (sl.log_copies, spec.log_copies, sl.gate_layers, dt)}
    if sl.log_copies < spec.log_copies:
        out["extrapolated_full_proof_s"] = round(spec.gate_layers / rate, 1)
        out["extrapolated"] = True
    return out


def batched_comparison(gkr, steps, warmup):
    """64 uneven jobs: sequential plain proofs, sequential graph replays, one batched launch."""
    import torch
    specs = gs.batch_jobs_c4()
    jobs = []
    for spec in specs:
        c = gkr.Circuit.from_synth(spec, gs.make_wiring(spec))
        d_in = gkr.device_elements(gs.make_inputs(spec))
        out = torch.zeros((1 << c.s(0), 8), dtype=torch.int32, device="cuda")
        proof = gkr.alloc_bytes(c.proof_bytes)
        ws = gkr.alloc_bytes(c.workspace_bytes)
        jobs.append((spec, c, d_in, out, proof, ws))
    gates = sum(c.gate_layers for _, c, *_ in jobs)

    def plain():
        for spec, c, d_in, out, proof, ws in jobs:
            gkr.prove_circuit(c, d_in, spec.seed, out, proof, ws)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    log("batched: plain sequential proofs")
    t_plain = timed(plain)
    log("batched: graph capture and replays")
    # the same sequential proofs captured once per job in HIP graphs, then replayed
    graphs = []
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        for spec, c, d_in, out, proof, ws in jobs:
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                gkr.prove_circuit(c, d_in, spec.seed, out, proof, ws, stream=stream)
            graphs.append(g)
    torch.cuda.synchronize()

    def graph_replay():
        for g in graphs:
            g.replay()

    t_graph = timed(graph_replay)
    plans = [gkr.Plan(gkr.make_job(c, d_in, spec.seed, out, proof, ws)) for spec, c, d_in, out, proof, ws in jobs]
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")

    def batched():
        for p in plans:
            p.reset()
        gkr.run_batch(plans, ctl)

    log("batched: one persistent launch")
    t_batch = timed(batched)
    # the batched proofs are checked against the oracle digests when available
    exact = None
    gp = os.path.join(ROOT, "tests", "golden", "c4_batch.json")
    if os.path.exists(gp):
        with open(gp) as f:
            gold = json.load(f)["jobs"]
        exact = all(hashlib.sha256(bytes(proof[: c.proof_bytes].cpu().numpy().tobytes())).hexdigest()
                    == gold[k]["proof_sha256"] for k, (spec, c, d_in, out, proof, ws) in enumerate(jobs))
    return {
        "workload": "64 uneven jobs: log2 gates/layer in [10,18], depth in [8,32], 2^4..2^10 copies",
        "gate_layers": gates,
        "plain_sequential": {"ms": round(t_plain * 1e3, 3), "field_gates_per_s": round(gates / t_plain, 1)},
        "graph_sequential": {"ms": round(t_graph * 1e3, 3), "field_gates_per_s": round(gates / t_graph, 1)},
        "batched_persistent": {"ms": round(t_batch * 1e3, 3), "field_gates_per_s": round(gates / t_batch, 1)},
        "speedup_vs_plain": round(t_plain / t_batch, 2),
        "bit_exact_vs_oracle_golden": exact,
    }


def serving_comparison(gkr, njobs, max_slots, budget_gib, util=0.8):
    """Poisson trace of the serving mix: plain one-at-a-time loop vs continuous batching."""
    import torch

    from paper_2404_10404_amd import serve
    specs = gs.serving_jobs_c5(njobs)
    reqs = []
    for k, spec in enumerate(specs):
        c = gkr.Circuit.from_synth(spec, gs.make_wiring(spec))
        reqs.append(serve.Request(rid=k, circuit=c, inputs=gs.make_inputs(spec), seed=spec.seed, arrival=0.0,
                                  gate_layers=spec.gate_layers))
    # mean plain service time of the mix (all jobs back to back, after one warm-up job)
    log("serving: %d requests built; mean plain service time" % len(reqs))
    serve.serve_plain(reqs[:1], keep_proofs=False)
    t0 = time.perf_counter()
    serve.serve_plain(reqs, keep_proofs=False)
    mean_service = (time.perf_counter() - t0) / len(reqs)
    rate = util / mean_service
    gaps = gs.poisson_gaps(len(reqs), rate)
    t = 0.0
    for r, g in zip(reqs, gaps):
        t += float(g)
        r.arrival = t
    log("serving: plain loop on the trace (%.3f arrivals/s)" % rate)
    plain = serve.serve_plain(reqs, keep_proofs=True)
    budget = int(budget_gib * (1 << 30))
    log("serving: continuous batching, stream executor")
    mixed = serve.serve(reqs, serve.StreamExecutor(keep_proofs=True), max_slots=max_slots, budget_bytes=budget)
    torch.cuda.synchronize()
    log("serving: continuous batching, persistent-kernel executor")
    persistent = serve.serve(reqs, serve.GpuExecutor(keep_proofs=True), max_slots=max_slots, budget_bytes=budget)
    torch.cuda.synchronize()
    same = all(mixed[r.rid].proof == plain[r.rid].proof == persistent[r.rid].proof and mixed[r.rid].proof is not None
               for r in reqs)
    return {
        "workload": "%d jobs: log2 gates/layer uniform in [12,22], depth in [8,24], Poisson arrivals" % len(reqs),
        "arrival_rate_per_s": round(rate, 3), "mean_plain_service_s": round(mean_service, 5),
        "max_slots": max_slots, "hbm_budget_gib": budget_gib,
        "plain_loop": serve.summary(plain, reqs),
        "continuous_batching": dict(serve.summary(mixed, reqs), executor="4 HIP streams, whole proofs enqueued"),
        "continuous_batching_persistent": dict(serve.summary(persistent, reqs),
                                               executor="persistent batch kernel; an epoch ends when a job "
                                                        "finishes or near the next admissible arrival"),
        "proofs_identical_alone_and_in_mix": same,
    }


def general_leg(gkr, steps, warmup, profile_steps, mac_peak_tops):
    """The general-circuit workload (accumulation gates, right inputs from up to
    four layers back): field-gates/s and nested-gates/s of plain proofs, the
    proof against the oracle's digest, the dominant kernel's roofline."""
    import torch
    spec = gs.general_data_parallel()
    wiring = gs.make_general_wiring(spec)
    inputs = gs.make_general_inputs(spec)
    c = gkr.GeneralCircuit.from_synth(spec, wiring)
    nested = sum(len(w.z) for w in wiring) << spec.log_copies
    prover = gkr.Prover(c)
    d_in = gkr.device_elements(inputs)
    del inputs
    for _ in range(warmup):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "general circuit: 2^8 copies x (depth 8, 2^12 gates/layer), 1..4 nested gates per gate, "
                       "a quarter of the right inputs from 2..4 layers back",
           "gate_layers_per_proof": c.gate_layers, "nested_gates_per_proof": nested,
           "ms_per_proof": round(dt * 1e3, 4), "field_gates_per_s": round(c.gate_layers / dt, 1),
           "nested_gates_per_s": round(nested / dt, 1)}
    gd = golden_digest("g1")
    if gd is not None:
        out["bit_exact_vs_oracle_golden"] = hashlib.sha256(prover.proof_bytes()).hexdigest() == gd
    if profile_steps:
        prof = profile_pass(gkr, prover, d_in, spec.seed, profile_steps)
        out["roofline"] = roofline(prof, "g1", mac_peak_tops)
        out["kernels"] = {k: {"ms": round(v["ms"], 4), "launches": v["launches"]} for k, v in
                          sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:8]}
    del prover, d_in
    return out


def goldilocks_leg(gkr, steps, warmup, profile_steps, mac_peak_tops, bn254_ms=None):
    """The single-worker share (2^12 copies x depth 24 x 2^14 gates/layer) over
    the Goldilocks field (Section 4.1): field-gates/s, the speed-up over the
    BN254 proof, its 2^4-copy slice against the oracle's digest, the dominant
    kernel's roofline."""
    import torch
    spec = gs.worker_share_c3()
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring, field=gkr.FIELD_GOLDILOCKS)
    prover = gkr.GlProver(c)
    d_in = gkr.gl_device_elements(gs.make_goldilocks_inputs(spec))
    for _ in range(warmup):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "Goldilocks field, single-worker share: 2^12 copies x (depth 24, 2^14 gates/layer), 30% MUL",
           "gate_layers_per_proof": c.gate_layers, "ms_per_proof": round(dt * 1e3, 4),
           "field_gates_per_s": round(c.gate_layers / dt, 1)}
    if bn254_ms:
        out["speedup_vs_bn254"] = round(bn254_ms / (dt * 1e3), 2)
    if profile_steps:
        prof = profile_pass(gkr, prover, d_in, spec.seed, profile_steps)
        out["roofline"] = roofline(prof, "gl_c3", mac_peak_tops, macs_per_mulmod=4, class_kernel=GL_CLASS_KERNEL,
                                   sources=GL_KERNEL_SOURCES)
        out["kernels"] = {k: {"ms": round(v["ms"], 4), "launches": v["launches"]} for k, v in
                          sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:8]}
    del prover, d_in
    torch.cuda.empty_cache()
    gd = golden_digest("gl_c3slice")
    if gd is not None:
        sl = gs.copy_slice(spec, 4)
        cs = gkr.Circuit.from_synth(sl, gs.make_wiring(sl), field=gkr.FIELD_GOLDILOCKS)
        ps = gkr.GlProver(cs)
        ps.prove(gkr.gl_device_elements(gs.make_goldilocks_inputs(sl)), sl.seed)
        torch.cuda.synchronize()
        out["slice_2^4_copies_vs_oracle_golden"] = hashlib.sha256(ps.proof_bytes()).hexdigest() == gd
    return out


VPD_CLASS_KERNEL = {"vpd_ntt": "k_vpd_ntt", "vpd_fri": "k_vpd_fold", "vpd_merkle": "k_vpd_leaves"}
VPD_KERNEL_SOURCES = ["fr.hpp", "sha256.hpp", "gkr_device.hpp", "gkr_kernels.hpp", "gkr_bodies.hpp", "gkr_vpd.hpp",
                      "gkr_vpd.hip"]


def committed_leg(gkr, steps, warmup, profile_steps, mac_peak_tops, plain_ms=None):
    """The single-worker share with its 2^26 inputs committed (Section 2.4):
    commitment, the layered proof and the opening at the last layer's two
    points with 64 queries; ms per proof and its cost over the plain proof,
    the commitment kernels by class with the dominant one's roofline, the
    library's verifier (outputs only) on the proof, and the committed proof
    of the 2^20-gate data-parallel circuit against the oracle's digest."""
    import torch
    spec = gs.worker_share_c3()
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    queries = gkr.DEFAULT_QUERIES
    prover = gkr.CommittedProver(c, queries)
    d_in = gkr.device_elements(gs.make_inputs(spec))
    for _ in range(warmup):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    out = {"workload": "single-worker share with committed inputs: 2^12 copies x (depth 24, 2^14 gates/layer), "
                       "2^26 inputs, coset of 2^28, %d queries" % queries,
           "queries": queries, "ms_per_proof": round(dt * 1e3, 4),
           "field_gates_per_s": round(c.gate_layers / dt, 1), "proof_bytes": prover.nbytes}
    if plain_ms:
        out["commitment_ms_over_plain_proof"] = round(dt * 1e3 - plain_ms, 4)
    if profile_steps:
        prof = profile_pass(gkr, prover, d_in, spec.seed, profile_steps)
        vp = {k: v for k, v in prof.items() if k.startswith("vpd_")}
        out["commitment_kernels_ms"] = {k: round(v["ms"], 4) for k, v in sorted(vp.items(), key=lambda kv: -kv[1]["ms"])}
        out["roofline"] = roofline(vp, "vpd_c3", mac_peak_tops, class_kernel=VPD_CLASS_KERNEL,
                                   sources=VPD_KERNEL_SOURCES)
        out["kernels"] = {k: {"ms": round(v["ms"], 4), "launches": v["launches"]} for k, v in
                          sorted(prof.items(), key=lambda kv: -kv[1]["ms"])[:10]}
    proof = prover.proof_bytes()
    outs = np.ascontiguousarray(gkr.host_elements(prover.outputs))
    del prover, d_in
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    out["verified_by_host"] = gkr.verify_committed(c, outs, spec.seed, proof, queries) == 1
    out["host_verify_s"] = round(time.perf_counter() - t0, 3)
    gd = golden_digest("vpd_c2")
    if gd is not None:
        s2 = gs.data_parallel_c2()
        c2 = gkr.Circuit.from_synth(s2, gs.make_wiring(s2))
        p2 = gkr.CommittedProver(c2, queries)
        p2.prove(gkr.device_elements(gs.make_inputs(s2)), s2.seed)
        torch.cuda.synchronize()
        out["c2_vs_oracle_golden"] = hashlib.sha256(p2.proof_bytes()).hexdigest() == gd
    return out


def golden_digest(name):
    p = os.path.join(ROOT, "tests", "golden", "%s_proof.json" % name)
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f).get("proof_sha256")


def slice_bit_exact(gkr, spec, log_copies, golden_name):
    """Prove the same sub-circuit with fewer copies on the GPU and compare the
    proof digest with the oracle's stored one (None if no golden exists)."""
    import torch
    gd = golden_digest(golden_name)
    if gd is None:
        return None
    sl = gs.copy_slice(spec, log_copies)
    c = gkr.Circuit.from_synth(sl, gs.make_wiring(sl))
    pr = gkr.Prover(c)
    pr.prove(gkr.device_elements(gs.make_inputs(sl)), sl.seed)
    torch.cuda.synchronize()
    ok = hashlib.sha256(pr.proof_bytes()).hexdigest() == gd
    del pr, c
    return ok


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS))
    ap.add_argument("--profile-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true")
    ap.add_argument("--no-batched", action="store_true", help="leave out the 64-job batched leg")
    ap.add_argument("--no-serving", action="store_true", help="leave out the serving leg")
    ap.add_argument("--no-general", action="store_true", help="leave out the general-circuit leg")
    ap.add_argument("--no-goldilocks", action="store_true", help="leave out the Goldilocks-field leg")
    ap.add_argument("--no-committed", action="store_true", help="leave out the committed-input leg")
    ap.add_argument("--mode", default="plain", choices=["plain", "batched", "serving", "copy", "ubench", "committed"])
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--jobs", type=int, default=256)
    ap.add_argument("--slots", type=int, default=32)
    ap.add_argument("--budget-gib", type=float, default=96.0)
    ap.add_argument("--batch-steps", type=int, default=3)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the prover proves one worker's share on a single MI355X "
              "and has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2404_10404_amd import gkr

    if args.mode == "copy":
        # a plain device-to-device copy of known size: the reference for scaling
        # the HBM traffic counters of the prover's kernels
        n = args.copy_mib << 20
        x = torch.empty(n, dtype=torch.uint8, device="cuda")
        y = torch.empty_like(x)
        x.fill_(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            y.copy_(x)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"mode": "copy", "bytes_per_copy": n, "copies": args.steps,
                          "GB_per_s": round(2 * n * args.steps / dt / 1e9, 1)}), flush=True)
        return
    if args.mode == "ubench":
        peaks = alu_peaks(gkr)
        out = {"mode": "ubench", "theoretical_full_rate_valu_per_s": VALU_PEAK_TOPS * 1e12}
        out.update({k: round(v, 1) for k, v in peaks.items()})
        out["mad_vs_full_rate"] = round(peaks["mad_u64_u32_per_s"] / (VALU_PEAK_TOPS * 1e12), 4)
        out["field_product_macs_per_s"] = round(peaks["field_products_per_s"] * MACS_PER_MULMOD, 1)
        print(json.dumps(out), flush=True)
        return
    if args.mode == "committed":
        peaks = None if args.no_profile else alu_peaks(gkr)
        res = committed_leg(gkr, args.steps, args.warmup, 0 if args.no_profile else args.profile_steps,
                            peaks["mad_u64_u32_per_s"] / 1e12 if peaks else None)
        line = {"metric": "GKR prover with committed inputs: ms per proof", "value": res["field_gates_per_s"],
                "unit": "field-gates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                "ms_per_step": res["ms_per_proof"], "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "u32 (BN254 Fr, exact modular integer arithmetic)",
                "data": "synthetic", "config": {"workload": res["workload"]}, "committed": res}
        print(json.dumps(line), flush=True)
        return
    if args.mode == "serving":
        res = serving_comparison(gkr, args.jobs, args.slots, args.budget_gib)
        cb = res["continuous_batching"]
        line = {"metric": "GKR serving: jobs/s and p50/p99 latency, continuous batching vs plain loop",
                "value": cb["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "steps": 1, "warmup": 1,
                "ms_per_step": round(cb["makespan_s"] * 1e3, 3), "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "u32 (BN254 Fr, exact modular integer arithmetic)",
                "data": "synthetic", "config": {"workload": res["workload"]}, "serving": res}
        print(json.dumps(line), flush=True)
        return
    if args.mode == "batched":
        res = batched_comparison(gkr, args.steps, args.warmup)
        line = {"metric": "GKR prover field-gates/sec, batched persistent launch vs plain per-job launches",
                "value": res["batched_persistent"]["field_gates_per_s"], "unit": "field-gates/s", "n_gpus": 1,
                "steps": args.steps, "warmup": args.warmup, "ms_per_step": res["batched_persistent"]["ms"],
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                "dtype": "u32 (BN254 Fr, exact modular integer arithmetic)", "data": "synthetic",
                "config": {"workload": res["workload"]}, "batched": res}
        print(json.dumps(line), flush=True)
        return

    peaks = None
    if not args.no_profile:
        log("integer-multiply peaks (gkr_ubench)")
        peaks = alu_peaks(gkr)
    spec = WORKLOADS[args.workload][0]()
    log("%s: wiring and inputs" % args.workload)
    wiring = gs.make_wiring(spec)
    inputs = gs.make_inputs(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    prover = gkr.Prover(c)
    d_in = gkr.device_elements(inputs)
    del inputs
    log("%s: %d warm-up proofs" % (args.workload, args.warmup))
    for _ in range(args.warmup):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    log("%s: %d timed proofs" % (args.workload, args.steps))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        prover.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = c.gate_layers * args.steps / dt
    proof = prover.proof_bytes()
    exact = {}
    gd = golden_digest(args.workload)
    if gd is not None:
        exact["proof_vs_oracle_golden"] = hashlib.sha256(proof).hexdigest() == gd

    line = {
        "metric": "GKR prover field-gates/sec + p99 job latency, batched vs plain, bit-exact",
        "value": round(value, 1),
        "unit": "field-gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 (BN254 Fr, exact modular integer arithmetic)",
        "data": "synthetic (seeded circuits and inputs; the paper's Ethereum circuits are not available)",
        "config": {"workload": WORKLOADS[args.workload][1], "gate_layers_per_proof": c.gate_layers,
                   "proof_bytes": c.proof_bytes, "seed": spec.seed},
    }
    if not args.no_profile:
        log("%s: profile pass (HIP events per launch)" % args.workload)
        prof = profile_pass(gkr, prover, d_in, spec.seed, args.profile_steps)
        line["roofline"] = roofline(prof, args.workload, peaks["mad_u64_u32_per_s"] / 1e12,
                                    stream_gbs=peaks["round_stream_bytes_per_s"] / 1e9)
        line["kernel_classes"] = class_fractions(prof, peaks["mad_u64_u32_per_s"] / 1e12,
                                                 peaks.get("field_products_per_s"))
        line["kernels"] = {k: {"ms": round(v["ms"], 4), "launches": v["launches"]} for k, v in
                           sorted(prof.items(), key=lambda kv: -kv[1]["ms"])}
        line["alu_peaks_measured"] = {k: round(v, 1) for k, v in peaks.items()}
    del prover, d_in
    torch.cuda.empty_cache()
    if args.workload == "c3":
        log("c3: the same sub-circuit with 2^4 copies against the oracle's proof")
        exact["c3_slice_2^4_copies_vs_oracle_golden"] = slice_bit_exact(gkr, spec, 4, "c3slice")
        torch.cuda.empty_cache()
    if not args.no_general:
        log("general-circuit leg")
        line["general"] = general_leg(gkr, 5, 1, 0 if args.no_profile else 1,
                                      peaks["mad_u64_u32_per_s"] / 1e12 if peaks else None)
        exact["general_vs_oracle_golden"] = line["general"].get("bit_exact_vs_oracle_golden")
        torch.cuda.empty_cache()
    if not args.no_goldilocks:
        log("Goldilocks-field leg")
        line["goldilocks"] = goldilocks_leg(gkr, 5, 1, 0 if args.no_profile else 1,
                                            peaks["mad_u64_u32_per_s"] / 1e12 if peaks else None,
                                            line["ms_per_step"] if args.workload == "c3" else None)
        exact["goldilocks_slice_vs_oracle_golden"] = line["goldilocks"].get("slice_2^4_copies_vs_oracle_golden")
        torch.cuda.empty_cache()
    if not args.no_committed:
        log("committed-input leg")
        line["committed"] = committed_leg(gkr, 3, 1, 0 if args.no_profile else 1,
                                          peaks["mad_u64_u32_per_s"] / 1e12 if peaks else None,
                                          line["ms_per_step"] if args.workload == "c3" else None)
        exact["committed_c2_vs_oracle_golden"] = line["committed"].get("c2_vs_oracle_golden")
        exact["committed_c3_verified"] = line["committed"]["verified_by_host"]
        torch.cuda.empty_cache()
    if not args.no_batched:
        log("batched leg: 64 uneven jobs")
        line["batched"] = batched_comparison(gkr, args.batch_steps, 1)
        exact["batched_64_jobs_vs_oracle_golden"] = line["batched"]["bit_exact_vs_oracle_golden"]
        torch.cuda.empty_cache()
    if not args.no_serving:
        log("serving leg: %d jobs" % args.jobs)
        line["serving"] = serving_comparison(gkr, args.jobs, args.slots, args.budget_gib)
        exact["serving_alone_vs_in_mix"] = line["serving"]["proofs_identical_alone_and_in_mix"]
        torch.cuda.empty_cache()
    line["bit_exact"] = exact
    if not args.no_cpu_baseline:
        log("cpu baseline: the oracle on a slice")
        line["cpu_baseline"] = cpu_baseline(spec)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
