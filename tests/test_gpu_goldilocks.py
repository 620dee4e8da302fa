"""GPU parity of the Goldilocks-field prover (Section 4.1, the field choice):
outputs and proof bytes of gkr_gl_prove_circuit equal the Goldilocks
oracle's (oracle/goldilocks.py) on the same seeded circuits, and the host
verifier accepts them. Shapes cover one copy and many, ragged widths, a
one-gate layer, tables inside the single-workgroup tail and grid-wide rounds,
all-MUL and all-ADD layers; the single-worker share's sub-circuit with 2^4
copies is compared with the oracle's stored proof."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import goldilocks as ogl

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gkr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2404_10404_amd import gkr as g
    return g


def _gpu(gkr, spec, wiring, inputs):
    import torch
    c = gkr.Circuit.from_synth(spec, wiring, field=gkr.FIELD_GOLDILOCKS)
    pr = gkr.GlProver(c)
    pr.prove(gkr.gl_device_elements(inputs), spec.seed)
    torch.cuda.synchronize()
    return c, pr.host_outputs(), pr.proof_bytes()


SHAPES = [
    (4, 0, (10,) * 5, 1, (1, 2)),
    (3, 3, (4, 5, 3, 4), 7, (1, 2)),
    (2, 5, (0, 2, 1), 8, (1, 2)),
    (1, 0, (0, 0), 9, (1, 2)),
    (2, 4, (8, 9, 8), 11, (1, 2)),        # grid-wide rounds
    (2, 0, (12, 11, 12), 12, (1, 2)),     # one copy, 2^12 gates
    (3, 8, (4, 4, 4, 4), 13, (3, 10)),    # many copies
    (2, 1, (11, 3, 12), 14, (1, 1)),      # all MUL
    (2, 2, (5, 6, 4), 15, (0, 1)),        # all ADD
    (2, 11, (3, 2, 3), 16, (1, 2)),       # 2^11 copies: grid-wide copy rounds in phase 2
]


@pytest.mark.parametrize("shape", SHAPES)
def test_goldilocks_proof_bit_exact(gkr, shape):
    depth, n, sig, seed, mu = shape
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=sig, mu=mu, seed=seed)
    _log("goldilocks %s" % (shape,))
    wiring = gs.make_wiring(spec)
    inputs = gs.make_goldilocks_inputs(spec)
    c, outs, proof = _gpu(gkr, spec, wiring, inputs)
    ref = ogl.prove(oc.Circuit.from_synth(spec, wiring), [int(v) for v in inputs], seed)
    assert [int(v) for v in outs] == ref.outputs, "outputs differ from the oracle"
    want = ref.proof_bytes()
    if proof != want:
        first = next(i for i in range(len(want)) if want[i] != proof[i])
        raise AssertionError("proof differs from the oracle's at element %d of %d" % (first // 8, len(want) // 8))
    assert gkr.gl_verify(c, inputs, outs, seed, proof) == 1


GOLDEN = {
    "gl_c3slice": lambda: gs.copy_slice(gs.worker_share_c3(), 4),
    "gl_c2": gs.data_parallel_c2,
}


@pytest.mark.parametrize("name", sorted(GOLDEN))
def test_goldilocks_workloads_match_oracle_golden(gkr, name):
    """Over Goldilocks, against the oracle's stored digests
    (tests/golden/make_golden.py): the single-worker share's sub-circuit (depth
    24, 2^14 gates, 30% MUL) with 2^4 copies, and the data-parallel workload of
    2^8 copies x depth 16, 2^12 gates/layer."""
    with open(os.path.join(HERE, "golden", "%s_proof.json" % name)) as f:
        gold = json.load(f)
    spec = GOLDEN[name]()
    assert gold["seed"] == spec.seed and gold["log_copies"] == spec.log_copies and gold["depth"] == spec.depth
    wiring = gs.make_wiring(spec)
    inputs = gs.make_goldilocks_inputs(spec)
    _log("goldilocks golden %s: proving" % name)
    c, outs, proof = _gpu(gkr, spec, wiring, inputs)
    assert len(proof) == gold["proof_len"]
    assert hashlib.sha256(np.ascontiguousarray(outs).tobytes()).hexdigest() == gold["outputs_sha256"]
    assert hashlib.sha256(proof).hexdigest() == gold["proof_sha256"]
    _log("goldilocks golden %s: host verifier" % name)
    assert gkr.gl_verify(c, inputs, outs, spec.seed, proof) == 1
