"""gkr_prove_circuit_noalloc (workspace in the library's static device array)
against gkr_prove_circuit (caller workspace): the same outputs and proof
bytes, on two calls in a row, the second with a smaller circuit (the static
array keeps the first call's contents), both also equal to the oracle's
proof; a circuit whose workspace exceeds the static array is refused with a
clear error and nothing is written."""
import sys

import numpy as np
import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import prover as op

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


def _both(gkr, spec):
    import torch
    wiring = gs.make_wiring(spec)
    inputs = gs.make_inputs(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    assert c.workspace_bytes <= gkr.NOALLOC_WORKSPACE_BYTES
    d_in = gkr.device_elements(inputs)
    out_a = torch.zeros((1 << c.s(0), 8), dtype=torch.int32, device="cuda")
    out_b = torch.zeros_like(out_a)
    proof_a = gkr.alloc_bytes(c.proof_bytes)
    proof_b = gkr.alloc_bytes(c.proof_bytes)
    ws = gkr.alloc_bytes(c.workspace_bytes)
    _log("no-alloc: %s, workspace %d bytes" % (spec, c.workspace_bytes))
    n_a = gkr.prove_circuit(c, d_in, spec.seed, out_a, proof_a, ws)
    n_b = gkr.prove_circuit_noalloc(c, d_in, spec.seed, out_b, proof_b)
    torch.cuda.synchronize()
    assert n_a == n_b == c.proof_bytes
    pa = bytes(proof_a[:n_a].cpu().numpy().tobytes())
    pb = bytes(proof_b[:n_b].cpu().numpy().tobytes())
    assert torch.equal(out_a, out_b)
    assert pa == pb
    ref = op.prove(oc.Circuit.from_synth(spec, wiring), gs.elements_to_ints(inputs), spec.seed)
    assert pb == ref.proof_bytes()
    return c


def test_noalloc_matches_caller_workspace_on_two_calls(gkr):
    # first a circuit with grid-wide rounds and several tiles, then a smaller one
    big = gs.CircuitSpec(depth=3, log_copies=5, log_sub_width=(8, 9, 8, 9), mu=(1, 2), seed=31)
    small = gs.CircuitSpec(depth=2, log_copies=2, log_sub_width=(3, 5, 4), mu=(3, 10), seed=32)
    _both(gkr, big)
    _both(gkr, small)


def test_noalloc_refuses_a_workspace_above_the_static_size(gkr):
    import torch
    # 2^23 gates per layer, depth 4: a workspace far above 256 MiB
    spec = gs.CircuitSpec(depth=4, log_copies=3, log_sub_width=(20,) * 5, mu=(1, 2), seed=33)
    c = gkr.Circuit.from_synth(spec, gs.make_wiring(spec))
    assert c.workspace_bytes > gkr.NOALLOC_WORKSPACE_BYTES
    d_in = torch.zeros((1 << c.s(spec.depth), 8), dtype=torch.int32, device="cuda")
    out = torch.full((1 << c.s(0), 8), 7, dtype=torch.int32, device="cuda")
    proof = gkr.alloc_bytes(c.proof_bytes)
    proof.fill_(5)
    with pytest.raises(gkr.GkrError) as e:
        gkr.prove_circuit_noalloc(c, d_in, spec.seed, out, proof)
    assert e.value.code == gkr.GKR_EUNSUPPORTED
    assert "static workspace" in str(e.value)
    torch.cuda.synchronize()
    assert bool((out == 7).all()) and bool((proof == 5).all())
