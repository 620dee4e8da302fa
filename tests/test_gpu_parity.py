"""GPU parity: proofs from the HIP path are byte-identical to the oracle's.

Field arithmetic is exact, so the bar is bit-exactness: the whole proof, the
outputs and every intermediate value handed back through the C ABI must equal
the oracle's bytes. Shapes cover several tiles and the single-workgroup tail
(tables above and below 2^10 entries), ragged layer widths, a single copy,
zero-width layers, the multi-workgroup sub-circuit rounds of phase 2 and
the matrix-core copy contraction (2^10 copies, at least 2^8 wires).
"""
import sys

import numpy as np
import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import mle
from oracle import prover as op
from oracle import verifier as ov
from oracle.field import P
from oracle.transcript import Transcript

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


def _oracle_case(spec):
    wiring = gs.make_wiring(spec)
    inputs = gs.make_inputs(spec)
    ocirc = oc.Circuit.from_synth(spec, wiring)
    layers = oc.evaluate(ocirc, gs.elements_to_ints(inputs))
    pt = op.prove_from_layers(ocirc, layers, spec.seed)
    return wiring, inputs, ocirc, layers, pt


SHAPES = [
    # depth, n, sigmas, seed, mu
    (4, 0, (10,) * 5, 1, (1, 2)),            # the plain single-instance circuit
    (3, 3, (4, 5, 3, 4), 7, (1, 2)),          # ragged widths
    (2, 5, (0, 2, 1), 8, (1, 2)),             # a one-gate sub-circuit layer
    (1, 0, (0, 0), 9, (1, 2)),                # one gate, one input
    (3, 2, (2, 0, 3, 1), 10, (3, 10)),
    (2, 4, (8, 9, 8), 11, (1, 2)),            # 2^13 tables: grid-wide rounds
    (2, 0, (12, 11, 12), 12, (1, 2)),         # one copy, 2^12 sub-circuit: grid-wide phase-2 rounds
    (3, 8, (4, 4, 4, 4), 13, (3, 10)),        # many copies: grid-wide copy rounds
    (2, 1, (11, 3, 12), 14, (1, 1)),          # all MUL, mismatched widths
    (2, 2, (5, 6, 4), 15, (0, 1)),            # all ADD
    (2, 10, (8, 8, 8), 16, (1, 2)),           # 2^10 copies: matrix-core copy contraction, one K block per chunk
    (2, 10, (7, 8, 9), 17, (3, 10)),          # ragged widths: one, then two row tiles
]


@pytest.mark.parametrize("shape", SHAPES, ids=[str(s[:4]) for s in SHAPES])
def test_prove_circuit_bit_exact(gkr, shape):
    import torch
    depth, n, sig, seed, mu = shape
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=sig, mu=mu, seed=seed)
    wiring, inputs, ocirc, layers, pt = _oracle_case(spec)
    _log("case %s: proving on the GPU" % (shape,))
    c = gkr.Circuit.from_synth(spec, wiring)
    pr = gkr.Prover(c)
    d_in = gkr.device_elements(inputs)
    plen = pr.prove(d_in, seed)
    torch.cuda.synchronize()
    assert plen == len(pt.proof_bytes())
    outs = gkr.host_elements(pr.outputs)
    assert gs.elements_to_ints(outs) == pt.outputs
    proof = pr.proof_bytes()
    if proof != pt.proof_bytes():
        ob = pt.proof_bytes()
        first = next(i for i in range(len(ob)) if ob[i] != proof[i])
        raise AssertionError("proof differs from the oracle at byte %d (element %d)" % (first, first // 32))
    assert gkr.verify(c, inputs, outs, seed, proof) == 1
    # a second run on the same workspace gives the same bytes
    pr.prove(d_in, seed)
    torch.cuda.synchronize()
    assert pr.proof_bytes() == proof


@pytest.mark.parametrize("shape", [(2, 4, (8, 9, 8), 11, (1, 2)), (2, 0, (12, 11, 12), 12, (1, 2)),
                                   (2, 9, (4, 3, 4), 16, (1, 2))], ids=["grid", "subcircuit", "copies"])
def test_tuning_never_changes_proof_bytes(gkr, shape):
    """Every schedule (tails from 2 to 2^16 entries, one to 4096 round
    workgroups, several pairs per thread) gives the oracle's bytes."""
    import torch
    depth, n, sig, seed, mu = shape
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=sig, mu=mu, seed=seed)
    wiring, inputs, ocirc, layers, pt = _oracle_case(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    pr = gkr.Prover(c)
    d_in = gkr.device_elements(inputs)
    old = gkr.get_tuning()
    try:
        for tun in [(1, 1, 1), (1, 4096, 1), (4, 7, 3), (6, 512, 1), (9, 64, 2), (12, 512, 1), (16, 4096, 5)]:
            _log("tuning %s on %s" % (tun, shape))
            gkr.set_tuning(*tun)
            pr.prove(d_in, seed)
            torch.cuda.synchronize()
            assert pr.proof_bytes() == pt.proof_bytes(), tun
    finally:
        gkr.set_tuning(*old)


def test_matrix_core_contraction_matches_scalar(gkr):
    """The phase-2 copy contraction on the int8 matrix cores gives the same
    proof bytes as the scalar pass where its tiling is the full one: 2^12
    copies x 2^12 wires, so 16 row tiles, 16 K chunks and 32 staged blocks
    per chunk; the library's verifier accepts the proof."""
    import torch
    spec = gs.CircuitSpec(depth=2, log_copies=12, log_sub_width=(12, 12, 12), mu=(1, 2), seed=18)
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    inputs = gs.make_inputs(spec)
    d_in = gkr.device_elements(inputs)
    proofs, outs = [], None
    try:
        for mode in (True, False):
            _log("2^24-gate layers, contraction on the matrix cores: %s" % mode)
            gkr.set_contraction(mode)
            pr = gkr.Prover(c)
            pr.prove(d_in, spec.seed)
            torch.cuda.synchronize()
            proofs.append(pr.proof_bytes())
            outs = np.ascontiguousarray(gkr.host_elements(pr.outputs))
            del pr
            torch.cuda.empty_cache()
    finally:
        gkr.set_contraction(True)
    assert proofs[0] == proofs[1]
    _log("host verifier")
    assert gkr.verify(c, inputs, outs, spec.seed, proofs[0]) == 1


def test_layer_entry_points_compose_and_resume(gkr):
    """transcript_init + output_claim + prove_layer (each layer resumed from the
    oracle's transcript state) give the oracle's bytes layer by layer."""
    import torch
    spec = gs.CircuitSpec(depth=3, log_copies=3, log_sub_width=(6, 7, 5, 6), mu=(1, 2), seed=21)
    wiring, inputs, ocirc, layers, pt = _oracle_case(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    ws = gkr.alloc_bytes(c.workspace_bytes)
    d_in = gkr.device_elements(inputs)
    d_out = gkr.device_elements(gs.ints_to_elements(layers[0]))
    d_state = torch.zeros(32, dtype=torch.uint8, device="cuda")
    _log("layer entry points: transcript_init")
    gkr.transcript_init(c, spec.seed, d_in, d_out, d_state, ws)
    tr = op.bind_statement(ocirc, layers[-1], layers[0], spec.seed)
    torch.cuda.synchronize()
    assert bytes(d_state.cpu().numpy()) == tr.state
    d_g = torch.zeros((max(1, c.s(0)), 8), dtype=torch.int32, device="cuda")
    d_claim = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
    _log("layer entry points: output_claim")
    gkr.output_claim(c, d_out, d_state, d_g, d_claim, ws)
    g = [tr.squeeze() for _ in range(ocirc.s(0))]
    torch.cuda.synchronize()
    assert gs.elements_to_ints(gkr.host_elements(d_g))[: len(g)] == g
    assert gs.elements_to_ints(gkr.host_elements(d_claim)) == [mle.evaluate(layers[0], g)]
    assert bytes(d_state.cpu().numpy()) == tr.state
    u, v, vu, vv = g, g, mle.evaluate(layers[0], g), 0
    for i in range(spec.depth):
        _log("layer entry points: prove_layer %d" % i)
        s1 = ocirc.s(i + 1)
        # resume from a fresh copy of the oracle's state
        d_state = torch.from_numpy(np.frombuffer(tr.state, dtype=np.uint8).copy()).cuda()
        d_next = gkr.device_elements(gs.ints_to_elements(layers[i + 1]))
        d_u = gkr.device_elements(gs.ints_to_elements(u))
        d_v = gkr.device_elements(gs.ints_to_elements(v))
        d_cu = gkr.device_elements(gs.ints_to_elements([vu]))
        d_cv = gkr.device_elements(gs.ints_to_elements([vv]))
        d_rx = torch.zeros((s1, 8), dtype=torch.int32, device="cuda")
        d_ry = torch.zeros((s1, 8), dtype=torch.int32, device="cuda")
        d_vx = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
        d_vy = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
        d_lp = gkr.alloc_bytes(c.layer_proof_bytes(i))
        gkr.prove_layer(c, i, d_next, d_u, d_v, d_cu, d_cv, d_state, d_rx, d_ry, d_vx, d_vy, d_lp, ws)
        if i == 0:
            alpha, beta = 1, 0
        else:
            alpha, beta = tr.squeeze(), tr.squeeze()
        lt = op.prove_layer(ocirc, i, layers[i + 1], u, None if i == 0 else v, alpha, beta,
                            (alpha * vu + beta * vv) % P, tr)
        torch.cuda.synchronize()
        assert bytes(d_lp[: c.layer_proof_bytes(i)].cpu().numpy()) == lt.proof_bytes()
        assert gs.elements_to_ints(gkr.host_elements(d_rx)) == lt.rx
        assert gs.elements_to_ints(gkr.host_elements(d_ry)) == lt.ry
        assert gs.elements_to_ints(gkr.host_elements(d_vx)) == [lt.vx]
        assert gs.elements_to_ints(gkr.host_elements(d_vy)) == [lt.vy]
        assert bytes(d_state.cpu().numpy()) == tr.state
        u, v, vu, vv = lt.rx, lt.ry, lt.vx, lt.vy


def test_error_paths(gkr):
    import torch
    spec = gs.CircuitSpec(depth=1, log_copies=1, log_sub_width=(3, 3), seed=5)
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    d_in = gkr.device_elements(gs.make_inputs(spec))
    outs = torch.zeros((16, 8), dtype=torch.int32, device="cuda")
    small = gkr.alloc_bytes(64)
    ws = gkr.alloc_bytes(c.workspace_bytes)
    with pytest.raises(gkr.GkrError) as e:
        gkr.prove_circuit(c, d_in, 5, outs, small, ws)
    assert e.value.code == gkr.GKR_EBUFSZ
    proof = gkr.alloc_bytes(c.proof_bytes)
    with pytest.raises(gkr.GkrError) as e:
        gkr.prove_circuit(c, d_in, 5, outs, proof, small)
    assert e.value.code == gkr.GKR_EBUFSZ
    # a valid call still works afterwards
    gkr.prove_circuit(c, d_in, 5, outs, proof, ws)
    torch.cuda.synchronize()
