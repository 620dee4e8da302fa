"""Batched proving on the GPU: every proof of a persistent multi-job launch is
byte-identical to the oracle's proof of the same job, also when the launch is
stopped and resumed (step budget, stop-on-finish), and for the 64 uneven jobs
of the batched workload (tests/golden/c4_batch.json, written by
tests/golden/make_golden.py from the oracle alone).
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import prover as op

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))

MIX = [
    (3, 3, (4, 5, 3, 4), 7, (1, 2)),
    (2, 5, (0, 2, 1), 8, (1, 2)),
    (1, 0, (0, 0), 9, (1, 2)),
    (2, 4, (8, 9, 8), 11, (1, 2)),
    (2, 0, (12, 11, 12), 12, (1, 2)),
    (3, 8, (4, 4, 4, 4), 13, (3, 10)),
    (4, 0, (10,) * 5, 1, (1, 2)),
    (2, 2, (5, 6, 4), 15, (0, 1)),
]


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


class _Job:
    def __init__(self, gkr, spec):
        import torch
        self.spec = spec
        self.wiring = gs.make_wiring(spec)
        self.inputs = gs.make_inputs(spec)
        self.c = gkr.Circuit.from_synth(spec, self.wiring)
        self.d_in = gkr.device_elements(self.inputs)
        self.out = torch.zeros((1 << self.c.s(0), 8), dtype=torch.int32, device="cuda")
        self.proof = gkr.alloc_bytes(self.c.proof_bytes)
        self.ws = gkr.alloc_bytes(self.c.workspace_bytes)
        self.job = gkr.make_job(self.c, self.d_in, spec.seed, self.out, self.proof, self.ws)

    def proof_bytes(self):
        return bytes(self.proof[: self.c.proof_bytes].cpu().numpy().tobytes())

    def oracle_bytes(self):
        ocirc = oc.Circuit.from_synth(self.spec, self.wiring)
        return op.prove(ocirc, gs.elements_to_ints(self.inputs), self.spec.seed).proof_bytes()


@pytest.fixture(scope="module")
def gkr():
    import torch
    assert torch.cuda.is_available()
    from paper_2404_10404_amd import gkr as g
    return g


def _mix(gkr):
    return [_Job(gkr, gs.CircuitSpec(depth=d, log_copies=n, log_sub_width=sig, mu=mu, seed=seed))
            for d, n, sig, seed, mu in MIX]


def test_batch_matches_oracle(gkr):
    import torch
    jobs = _mix(gkr)
    plans = [gkr.Plan(j.job) for j in jobs]
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")
    _log("batch: one persistent launch over %d jobs" % len(jobs))
    gkr.run_batch(plans, ctl)
    torch.cuda.synchronize()
    assert int(ctl[0]) == len(jobs)
    for j, p in zip(jobs, plans):
        done, total = p.progress()
        assert done == total
        assert j.proof_bytes() == j.oracle_bytes(), j.spec
    # run again after a reset: same bytes
    for p in plans:
        p.reset()
    gkr.run_batch(plans, ctl, workgroups=64)
    torch.cuda.synchronize()
    for j in jobs:
        assert j.proof_bytes() == j.oracle_bytes(), j.spec


def test_batch_stop_and_resume(gkr):
    import torch
    jobs = _mix(gkr)
    plans = [gkr.Plan(j.job) for j in jobs]
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")
    total = sum(p.progress()[1] for p in plans)
    _log("batch: resumable launches with a step budget")
    launches = 0
    while launches < 2000:
        gkr.run_batch(plans, ctl, step_budget=25)
        torch.cuda.synchronize()
        launches += 1
        if all(d == t for d, t in (p.progress() for p in plans)):
            break
    assert launches > 3 and all(d == t for d, t in (p.progress() for p in plans))
    for j in jobs:
        assert j.proof_bytes() == j.oracle_bytes(), j.spec
    # stop-on-finish: every launch retires at least one job
    for p in plans:
        p.reset()
    launches = 0
    while launches < 100 and not all(d == t for d, t in (p.progress() for p in plans)):
        gkr.run_batch(plans, ctl, stop_on_finish=True)
        torch.cuda.synchronize()
        launches += 1
        assert int(ctl[0]) >= 1
    assert launches >= 2
    for j in jobs:
        assert j.proof_bytes() == j.oracle_bytes(), j.spec


def test_uneven_batch_of_64_bit_exact(gkr):
    import torch
    with open(os.path.join(HERE, "golden", "c4_batch.json")) as f:
        gold = json.load(f)["jobs"]
    specs = gs.batch_jobs_c4()
    _log("batch: building the 64 uneven jobs")
    jobs = [_Job(gkr, s) for s in specs]
    plans = [gkr.Plan(j.job) for j in jobs]
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")
    _log("batch: one persistent launch over 64 jobs")
    gkr.run_batch(plans, ctl)
    torch.cuda.synchronize()
    assert int(ctl[0]) == 64
    for k, j in enumerate(jobs):
        assert gold[k]["seed"] == j.spec.seed
        outs = np.ascontiguousarray(gkr.host_elements(j.out))
        assert hashlib.sha256(outs.tobytes()).hexdigest() == gold[k]["outputs_sha256"], k
        assert hashlib.sha256(j.proof_bytes()).hexdigest() == gold[k]["proof_sha256"], k


def test_graph_captured_proof_replays_bit_exact(gkr):
    """A whole proof captured in a HIP graph gives the oracle's bytes on every replay,
    with eager proofs of another job (and synchronisations) between the replays."""
    import torch
    jobs = _mix(gkr)
    a, b = jobs[3], jobs[0]
    want_a, want_b = a.oracle_bytes(), b.oracle_bytes()
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        gkr.prove_circuit(a.c, a.d_in, a.spec.seed, a.out, a.proof, a.ws, stream=stream)  # warm-up
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            gkr.prove_circuit(a.c, a.d_in, a.spec.seed, a.out, a.proof, a.ws, stream=stream)
    torch.cuda.synchronize()
    for rep in range(4):
        a.proof.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert a.proof_bytes() == want_a, rep
        gkr.prove_circuit(b.c, b.d_in, b.spec.seed, b.out, b.proof, b.ws)
        torch.cuda.synchronize()
        assert b.proof_bytes() == want_b, rep


def test_large_jobs_in_one_persistent_launch_match_plain_and_verify(gkr):
    """The 16 largest jobs of the serving mix (up to 2^22 gates per layer, 2^5..2^10
    copies) in one persistent launch: each step has hundreds of tiles spread over
    every XCD, and the next step's tiles read the tables they wrote. Every proof
    and output vector equals the plain launch's for the same job, and the host
    verifier accepts it. (A tile that published its writes before all of its
    waves' stores had reached the L2 gave wrong proofs for some of these jobs.)"""
    import torch
    specs = gs.serving_jobs_c5(96)
    big = sorted(range(len(specs)), key=lambda k: (-specs[k].gate_layers, k))[:16]
    _log("batch: building the 16 largest serving jobs %s" % big)
    jobs = [_Job(gkr, specs[k]) for k in big]
    plans = [gkr.Plan(j.job) for j in jobs]
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")
    _log("batch: one persistent launch over %d jobs" % len(jobs))
    gkr.run_batch(plans, ctl)
    torch.cuda.synchronize()
    assert int(ctl[0]) == len(jobs)
    for k, j in zip(big, jobs):
        batched = j.proof_bytes()
        outs = np.ascontiguousarray(gkr.host_elements(j.out)).copy()
        j.out.zero_()
        j.proof.zero_()
        gkr.prove_circuit(j.c, j.d_in, j.spec.seed, j.out, j.proof, j.ws)
        torch.cuda.synchronize()
        assert j.proof_bytes() == batched, (k, j.spec)
        assert np.array_equal(gkr.host_elements(j.out), outs), (k, j.spec)
        assert gkr.verify(j.c, j.inputs, outs, j.spec.seed, batched) == 1, (k, j.spec)
    for p in plans:
        p.close()


@pytest.mark.parametrize("tun", [(1, 4, 1), (2, 1, 1), (16, 64, 2)], ids=["grid-rounds", "one-tile-rounds", "tails"])
def test_batch_schedules_with_stops_match_oracle(gkr, tun):
    """Plans recorded under extreme schedules (nearly every round a grid round,
    each leaving its claim move pending for the next step; or whole phases in
    tails), run in short launches that stop after a few steps: every round's
    pending claim move crosses launch boundaries, and the proofs stay the
    oracle's."""
    import torch
    old = gkr.get_tuning()
    try:
        gkr.set_tuning(*tun)
        jobs = _mix(gkr)
        plans = [gkr.Plan(j.job) for j in jobs]
    finally:
        gkr.set_tuning(*old)
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")
    _log("batch: schedule %s, launches of at most 7 steps" % (tun,))
    launches = 0
    while launches < 5000:
        gkr.run_batch(plans, ctl, step_budget=7)
        torch.cuda.synchronize()
        launches += 1
        if all(d == t for d, t in (p.progress() for p in plans)):
            break
    assert all(d == t for d, t in (p.progress() for p in plans))
    for j in jobs:
        assert j.proof_bytes() == j.oracle_bytes(), j.spec
    for p in plans:
        p.close()
