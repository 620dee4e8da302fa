"""Write the stored expected proofs under tests/golden/ from the CPU oracle.

Only the oracle and the seeded generator are used. Each file records the
workload, the SHA-256 of the outputs and of the proof, and the proof itself
(hex) for the smaller cases. "c4" proves the 64 jobs of the uneven batch
(one oracle process per CPU) and stores each job's digests.

    python tests/golden/make_golden.py c1 c2 c3slice c4 g1slice g1

"g1" is the general-circuit workload (accumulation gates, right inputs from
up to four layers back, oracle/general.py); "g1slice" the same sub-circuit
with 2^2 copies. "gl_c3slice" and "gl_c2" are the Goldilocks variant
(oracle/goldilocks.py) of the c3 slice and of c2. "vpd_c2" is the
committed-input proof (oracle/vpd.py, 64 queries) of c2.
"""
import hashlib
import json
import multiprocessing
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import dataclasses  # noqa: E402

import gkr_synth as gs  # noqa: E402
from oracle import circuit as oc  # noqa: E402
from oracle import general as og  # noqa: E402
from oracle import goldilocks as ogl  # noqa: E402
from oracle import prover as op  # noqa: E402
from oracle import vpd  # noqa: E402
from oracle.field import encode_all  # noqa: E402

CASES = {
    "c1": (gs.plain_c1, True),
    "c2": (gs.data_parallel_c2, True),
    # the single-worker share's sub-circuit (depth 24, 2^14 gates, 30% MUL) with 2^4 copies
    "c3slice": (lambda: gs.copy_slice(gs.worker_share_c3(), 4), True),
}


GENERAL_CASES = {
    "g1": (gs.general_data_parallel, False),
    "g1slice": (lambda: dataclasses.replace(gs.general_data_parallel(), log_copies=2), True),
}


def make_general(name):
    spec = GENERAL_CASES[name][0]()
    t0 = time.time()
    wiring = gs.make_general_wiring(spec)
    inputs = gs.elements_to_ints(gs.make_general_inputs(spec))
    pt = og.prove(og.GeneralCircuit.from_synth(spec, wiring), inputs, spec.seed)
    proof = pt.proof_bytes()
    rec = {
        "workload": name, "depth": spec.depth, "log_copies": spec.log_copies,
        "log_sub_width": list(spec.log_sub_width), "max_fanin": spec.max_fanin, "reach": spec.reach,
        "cross": list(spec.cross), "mu": list(spec.mu), "seed": spec.seed,
        "outputs_sha256": hashlib.sha256(encode_all(pt.outputs)).hexdigest(),
        "proof_sha256": hashlib.sha256(proof).hexdigest(),
        "proof_len": len(proof),
        "oracle_seconds": round(time.time() - t0, 1),
        "writer": "tests/golden/make_golden.py (CPU oracle)",
    }
    if GENERAL_CASES[name][1]:
        rec["proof_hex"] = proof.hex()
    with open(os.path.join(HERE, "%s_proof.json" % name), "w") as f:
        json.dump(rec, f, indent=1)
    print(name, "done in %.1f s" % (time.time() - t0), flush=True)


# the Goldilocks variant (oracle/goldilocks.py) of the layered workloads
GOLDILOCKS_CASES = {
    "gl_c3slice": lambda: gs.copy_slice(gs.worker_share_c3(), 4),
    "gl_c2": gs.data_parallel_c2,
}


def make_goldilocks(name):
    spec = GOLDILOCKS_CASES[name]()
    t0 = time.time()
    wiring = gs.make_wiring(spec)
    inputs = [int(v) for v in gs.make_goldilocks_inputs(spec)]
    pt = ogl.prove(oc.Circuit.from_synth(spec, wiring), inputs, spec.seed)
    proof = pt.proof_bytes()
    rec = {
        "workload": name, "field": "goldilocks", "depth": spec.depth, "log_copies": spec.log_copies,
        "log_sub_width": list(spec.log_sub_width), "mu": list(spec.mu), "seed": spec.seed,
        "outputs_sha256": hashlib.sha256(ogl.encode_all(pt.outputs)).hexdigest(),
        "proof_sha256": hashlib.sha256(proof).hexdigest(),
        "proof_len": len(proof),
        "oracle_seconds": round(time.time() - t0, 1),
        "writer": "tests/golden/make_golden.py (CPU oracle)",
    }
    with open(os.path.join(HERE, "%s_proof.json" % name), "w") as f:
        json.dump(rec, f, indent=1)
    print(name, "done in %.1f s" % (time.time() - t0), flush=True)


# committed-input proofs (oracle/vpd.py)
COMMITTED_CASES = {
    "vpd_c2": (gs.data_parallel_c2, 64),
}


def make_committed(name):
    spec_fn, queries = COMMITTED_CASES[name]
    spec = spec_fn()
    t0 = time.time()
    wiring = gs.make_wiring(spec)
    inputs = gs.elements_to_ints(gs.make_inputs(spec))
    pf = vpd.prove_committed(oc.Circuit.from_synth(spec, wiring), inputs, spec.seed, queries)
    proof = pf.proof_bytes()
    rec = {
        "workload": name, "depth": spec.depth, "log_copies": spec.log_copies,
        "log_sub_width": list(spec.log_sub_width), "mu": list(spec.mu), "seed": spec.seed, "queries": queries,
        "root_hex": pf.root.hex(),
        "outputs_sha256": hashlib.sha256(encode_all(pf.outputs)).hexdigest(),
        "proof_sha256": hashlib.sha256(proof).hexdigest(),
        "proof_len": len(proof),
        "oracle_seconds": round(time.time() - t0, 1),
        "writer": "tests/golden/make_golden.py (CPU oracle)",
    }
    with open(os.path.join(HERE, "%s_proof.json" % name), "w") as f:
        json.dump(rec, f, indent=1)
    print(name, "done in %.1f s" % (time.time() - t0), flush=True)


def make(name):
    if name in COMMITTED_CASES:
        return make_committed(name)
    if name in GENERAL_CASES:
        return make_general(name)
    if name in GOLDILOCKS_CASES:
        return make_goldilocks(name)
    spec = CASES[name][0]()
    t0 = time.time()
    wiring = gs.make_wiring(spec)
    inputs = gs.elements_to_ints(gs.make_inputs(spec))
    c = oc.Circuit.from_synth(spec, wiring)
    pt = op.prove(c, inputs, spec.seed)
    proof = pt.proof_bytes()
    rec = {
        "workload": name,
        "depth": spec.depth,
        "log_copies": spec.log_copies,
        "log_sub_width": list(spec.log_sub_width),
        "mu": list(spec.mu),
        "seed": spec.seed,
        "outputs_sha256": hashlib.sha256(encode_all(pt.outputs)).hexdigest(),
        "proof_sha256": hashlib.sha256(proof).hexdigest(),
        "proof_len": len(proof),
        "oracle_seconds": round(time.time() - t0, 1),
        "writer": "tests/golden/make_golden.py (CPU oracle)",
    }
    if CASES[name][1]:
        rec["proof_hex"] = proof.hex()
    with open(os.path.join(HERE, "%s_proof.json" % name), "w") as f:
        json.dump(rec, f, indent=1)
    print(name, "done in %.1f s" % (time.time() - t0), flush=True)


def _batch_job(k):
    spec = gs.batch_jobs_c4()[k]
    wiring = gs.make_wiring(spec)
    inputs = gs.elements_to_ints(gs.make_inputs(spec))
    pt = op.prove(oc.Circuit.from_synth(spec, wiring), inputs, spec.seed)
    return {
        "job": k, "seed": spec.seed, "depth": spec.depth, "log_copies": spec.log_copies,
        "log_sub_width": list(spec.log_sub_width),
        "outputs_sha256": hashlib.sha256(encode_all(pt.outputs)).hexdigest(),
        "proof_sha256": hashlib.sha256(pt.proof_bytes()).hexdigest(),
    }


def make_c4():
    t0 = time.time()
    jobs = gs.batch_jobs_c4()
    order = sorted(range(len(jobs)), key=lambda k: -jobs[k].gate_layers)  # longest first
    with multiprocessing.Pool(min(8, os.cpu_count() or 1)) as pool:
        recs = pool.map(_batch_job, order, chunksize=1)
    recs.sort(key=lambda r: r["job"])
    with open(os.path.join(HERE, "c4_batch.json"), "w") as f:
        json.dump({"workload": "c4", "writer": "tests/golden/make_golden.py (CPU oracle)",
                   "oracle_seconds": round(time.time() - t0, 1), "jobs": recs}, f, indent=1)
    print("c4 done in %.1f s" % (time.time() - t0), flush=True)


if __name__ == "__main__":
    for n in sys.argv[1:] or ["c1"]:
        make_c4() if n == "c4" else make(n)
