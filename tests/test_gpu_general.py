"""GPU parity of general circuits (accumulation gates, right inputs from any
later layer): outputs and proof bytes of the HIP path equal the oracle's
(oracle/general.py) on the same seeded circuits; the library's host verifier
accepts them. Shapes cover one copy and many, fan-in 1 (no accumulation) to 4,
right inputs from the next layer only and from up to four layers back, tables
inside the single-workgroup tail and grid-wide rounds in both phases."""
import dataclasses
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import gkr_synth as gs
from oracle import general as og

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gkr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2404_10404_amd import gkr as g
    return g


SHAPES = [
    # depth, n, sigmas, seed, max_fanin, reach, cross
    (2, 0, (2, 3, 2), 101, 3, 3, (1, 2)),
    (3, 2, (3, 4, 2, 3), 102, 4, 4, (1, 2)),
    (1, 0, (0, 0), 103, 1, 1, (0, 1)),              # one gate reading one input
    (3, 1, (1, 0, 2, 1), 104, 2, 3, (1, 1)),        # every right input from beyond the next layer
    (4, 3, (4, 4, 4, 4, 4), 105, 1, 1, (0, 1)),     # fan-in 1, next layer only
    (3, 4, (8, 9, 8, 9), 106, 4, 3, (1, 3)),        # grid-wide rounds in both phases
    (2, 0, (12, 11, 12), 107, 2, 2, (1, 2)),        # one copy, 2^12 gates: grid-wide sub-circuit rounds
    (5, 2, (3, 5, 4, 3, 5, 4), 108, 4, 5, (1, 2)),  # many sources per layer
]


def _prove_both(gkr, spec):
    import torch
    wiring = gs.make_general_wiring(spec)
    inputs = gs.make_general_inputs(spec)
    c = gkr.GeneralCircuit.from_synth(spec, wiring)
    pr = gkr.Prover(c)
    pr.prove(gkr.device_elements(inputs), spec.seed)
    torch.cuda.synchronize()
    proof = pr.proof_bytes()
    outs = np.ascontiguousarray(gkr.host_elements(pr.outputs))
    ref = og.prove(og.GeneralCircuit.from_synth(spec, wiring), gs.elements_to_ints(inputs), spec.seed)
    return c, inputs, outs, proof, ref


@pytest.mark.parametrize("shape", SHAPES)
def test_general_proof_bit_exact(gkr, shape):
    depth, n, sig, seed, fanin, reach, cross = shape
    spec = gs.GeneralSpec(depth=depth, log_copies=n, log_sub_width=sig, max_fanin=fanin, reach=reach, cross=cross,
                          seed=seed)
    _log("general %s" % (shape,))
    c, inputs, outs, proof, ref = _prove_both(gkr, spec)
    assert gs.elements_to_ints(outs) == ref.outputs, "outputs differ from the oracle"
    want = ref.proof_bytes()
    if proof != want:
        first = next(i for i in range(len(want)) if want[i] != proof[i])
        raise AssertionError("proof differs from the oracle's at element %d of %d" % (first // 32, len(want) // 32))
    assert gkr.verify(c, inputs, outs, seed, proof) == 1


def test_general_workload_small_bit_exact(gkr):
    """The small general workload: 2^4 copies x depth 6, 2^8 gates/layer, up to 4 nested gates."""
    spec = gs.general_small()
    _log("general_small")
    c, inputs, outs, proof, ref = _prove_both(gkr, spec)
    assert gs.elements_to_ints(outs) == ref.outputs
    assert proof == ref.proof_bytes()


def test_general_no_alloc_and_repeat(gkr):
    """The no-allocation entry point proves general circuits too (same bytes),
    and a second proof in the same workspace gives the same bytes."""
    import torch
    spec = gs.GeneralSpec(depth=3, log_copies=2, log_sub_width=(4, 5, 4, 5), max_fanin=3, reach=3, cross=(1, 2),
                          seed=110)
    wiring = gs.make_general_wiring(spec)
    inputs = gs.make_general_inputs(spec)
    c = gkr.GeneralCircuit.from_synth(spec, wiring)
    d_in = gkr.device_elements(inputs)
    pr = gkr.Prover(c)
    pr.prove(d_in, spec.seed)
    pr.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    a = pr.proof_bytes()
    out = torch.zeros_like(pr.outputs)
    proof = gkr.alloc_bytes(c.proof_bytes)
    gkr.prove_circuit_noalloc(c, d_in, spec.seed, out, proof)
    torch.cuda.synchronize()
    assert bytes(proof[: c.proof_bytes].cpu().numpy().tobytes()) == a
    ref = og.prove(og.GeneralCircuit.from_synth(spec, wiring), gs.elements_to_ints(inputs), spec.seed)
    assert a == ref.proof_bytes()


HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("name,log_copies", [("g1slice", 2), ("g1", 8)])
def test_general_workload_matches_oracle_golden(gkr, name, log_copies):
    """The general-circuit workload bench.py times (2^8 copies x depth 8, 2^12
    gates/layer, up to 4 nested gates) and its 2^2-copy slice, against the
    oracle's stored digests (tests/golden/make_golden.py); the host verifier
    accepts the full-size proof."""
    import torch
    path = os.path.join(HERE, "golden", "%s_proof.json" % name)
    with open(path) as f:
        gold = json.load(f)
    spec = dataclasses.replace(gs.general_data_parallel(), log_copies=log_copies)
    assert gold["seed"] == spec.seed and gold["log_copies"] == spec.log_copies
    _log("general golden %s: proving" % name)
    wiring = gs.make_general_wiring(spec)
    inputs = gs.make_general_inputs(spec)
    c = gkr.GeneralCircuit.from_synth(spec, wiring)
    pr = gkr.Prover(c)
    pr.prove(gkr.device_elements(inputs), spec.seed)
    torch.cuda.synchronize()
    proof = pr.proof_bytes()
    outs = np.ascontiguousarray(gkr.host_elements(pr.outputs))
    assert hashlib.sha256(outs.tobytes()).hexdigest() == gold["outputs_sha256"]
    if hashlib.sha256(proof).hexdigest() != gold["proof_sha256"]:
        if "proof_hex" in gold:
            ref = bytes.fromhex(gold["proof_hex"])
            first = next(i for i in range(len(ref)) if ref[i] != proof[i])
            raise AssertionError("proof differs from the oracle's at element %d" % (first // 32))
        raise AssertionError("proof digest differs from the oracle's")
    _log("general golden %s: host verifier" % name)
    assert gkr.verify(c, inputs, outs, spec.seed, proof) == 1
