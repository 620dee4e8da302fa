"""GPU parity of the input-layer commitment and the committed-input proof
(Section 2.4) against the oracle (oracle/vpd.py): commitment roots for 2^1 ..
2^13 values (one-pass and multi-pass transforms), committed proofs byte for
byte on shapes from one input bit to 2^11 inputs with 1 .. 256 queries, and the
single-worker share at full size (2^26 inputs) checked through the library's
verifier, an independent replay of its transcript, the input MLE at the last
layer's points and the opened values of f against Horner evaluation."""
import sys

import numpy as np
import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import fast, vpd
from oracle.field import P
from oracle.transcript import TAG_DIGEST, TAG_VALUE, Transcript, circuit_digest, tree_digest

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


@pytest.mark.parametrize("log_n", [1, 2, 3, 9, 10, 11, 12, 13])
def test_commitment_root_matches_oracle(gkr, log_n):
    import torch
    _log("commit 2^%d" % log_n)
    limbs = gs.field_elements(gs.stream_key(900 + log_n, gs.PURPOSE_INPUT, 0), 1 << log_n)
    ws = gkr.alloc_bytes(gkr.vpd_workspace_bytes(log_n))
    root = gkr.alloc_bytes(32)
    gkr.vpd_commit(log_n, gkr.device_elements(limbs), root, ws)
    torch.cuda.synchronize()
    got = bytes(root[:32].cpu().numpy().tobytes())
    assert got == vpd.commit(gs.elements_to_ints(limbs)).root


SHAPES = [
    # depth, n, sigmas, seed, queries
    (1, 0, (2, 1), 201, 8),          # one input bit: the smallest commitment
    (1, 0, (2, 3), 202, 8),
    (3, 2, (3, 4, 3, 4), 203, 64),
    (2, 3, (2, 1, 3), 204, 1),       # a single query
    (2, 2, (4, 5, 9), 205, 8),       # 2^11 inputs: multi-pass transforms of 2^12 and 2^13
    (2, 1, (3, 3, 2), 206, 256),     # the most queries
]


def _prove_both(gkr, spec, queries):
    import torch
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    inputs = gs.make_inputs(spec)
    pr = gkr.CommittedProver(c, queries)
    pr.prove(gkr.device_elements(inputs), spec.seed)
    torch.cuda.synchronize()
    proof = pr.proof_bytes()
    outs = np.ascontiguousarray(gkr.host_elements(pr.outputs))
    ref = vpd.prove_committed(oc.Circuit.from_synth(spec, wiring), gs.elements_to_ints(inputs), spec.seed, queries)
    return c, outs, proof, ref


@pytest.mark.parametrize("shape", SHAPES)
def test_committed_proof_bit_exact(gkr, shape):
    depth, n, sig, seed, queries = shape
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=sig, mu=(1, 2), seed=seed)
    _log("committed %s" % (shape,))
    c, outs, proof, ref = _prove_both(gkr, spec, queries)
    assert gs.elements_to_ints(outs) == ref.outputs, "outputs differ from the oracle"
    want = ref.proof_bytes()
    assert len(proof) == len(want)
    if proof != want:
        first = next(i for i in range(len(want)) if want[i] != proof[i]) // 32
        gkr_units = sum(6 * c.s(i + 1) + 2 for i in range(depth))
        part = "root" if first == 0 else ("layers" if first <= gkr_units else "opening")
        raise AssertionError("proof differs from the oracle's at 32-byte unit %d of %d (%s)"
                             % (first, len(want) // 32, part))
    assert gkr.verify_committed(c, outs, seed, proof, queries) == 1
    bad = bytearray(proof)
    bad[-1] ^= 1
    assert gkr.verify_committed(c, outs, seed, bytes(bad), queries) == 0


def test_committed_proof_repeats_in_the_same_workspace(gkr):
    """Two proofs in a row with one prover (the workspace keeps the previous
    proof's tables) give the same bytes as a fresh prover."""
    import torch
    spec = gs.CircuitSpec(depth=2, log_copies=2, log_sub_width=(3, 4, 5), mu=(1, 2), seed=207)
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    d_in = gkr.device_elements(gs.make_inputs(spec))
    pr = gkr.CommittedProver(c, 16)
    other = gs.make_inputs(gs.CircuitSpec(depth=2, log_copies=2, log_sub_width=(3, 4, 5), mu=(1, 2), seed=208))
    pr.prove(gkr.device_elements(other), 208)
    pr.prove(d_in, spec.seed)
    torch.cuda.synchronize()
    a = pr.proof_bytes()
    ref = vpd.prove_committed(oc.Circuit.from_synth(spec, wiring), gs.elements_to_ints(gs.make_inputs(spec)),
                              spec.seed, 16)
    assert a == ref.proof_bytes()


def _replay(circuit, root, out_limbs, seed, proof, queries):
    """The committed proof's transcript replayed from its bytes (challenges
    only, no checks): the last layer's points and values and the query leaves."""
    tr = Transcript(seed)
    tr.absorb(TAG_DIGEST, circuit_digest(circuit.depth, circuit.n, circuit.sigma, circuit.wiring))
    tr.absorb(TAG_DIGEST, root)
    tr.absorb(TAG_DIGEST, tree_digest(np.ascontiguousarray(out_limbs).tobytes()))
    pos = 32

    def elem():
        nonlocal pos
        v = int.from_bytes(proof[pos:pos + 32], "little")
        pos += 32
        return v

    for _ in range(circuit.s(0)):
        tr.squeeze()
    rx = ry = None
    vx = vy = None
    for i in range(circuit.depth):
        if i:
            tr.squeeze()
            tr.squeeze()
        pts = []
        vals = []
        for _ph in range(2):
            r = []
            for _ in range(circuit.s(i + 1)):
                e0, _e1, e2 = elem(), elem(), elem()
                r.append(tr.round_challenge(e0, e2))
            v = elem()
            tr.absorb_elements(TAG_VALUE, [v])
            pts.append(r)
            vals.append(v)
        rx, ry = pts
        vx, vy = vals
    s = circuit.s(circuit.depth)
    m = 1 << (s + vpd.LOG_BLOWUP)
    tr.squeeze()                                  # lam
    tr.absorb(vpd.TAG_COMMIT, proof[pos:pos + 32])
    pos += 32
    for _ in range(4):
        tr.squeeze()
    for i in range(s):
        tr.squeeze()
        if i + 1 < s:
            tr.absorb(vpd.TAG_COMMIT, proof[pos:pos + 32])
            pos += 32
    final = proof[pos:pos + 32]
    pos += 32
    tr.absorb(TAG_VALUE, final)
    idx = [tr.squeeze() % (m // 2) for _ in range(queries)]
    return rx, ry, vx, vy, idx, pos


def test_committed_worker_share_full_size(gkr):
    """The single-worker share (2^12 copies x depth 24 x 2^14 gates/layer, 2^26
    inputs, M = 2^28) with 64 queries: the library's verifier accepts; an
    independent replay of the transcript finds the last layer's claims equal to
    the input MLE (C oracle helper) and the opened f values equal to f(x), f(-x)
    by Horner evaluation at four queried leaves."""
    import torch
    spec = gs.worker_share_c3()
    queries = gkr.DEFAULT_QUERIES
    _log("committed c3: wiring and inputs")
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    inputs = gs.make_inputs(spec)
    _log("committed c3: proving")
    pr = gkr.CommittedProver(c, queries)
    pr.prove(gkr.device_elements(inputs), spec.seed)
    torch.cuda.synchronize()
    proof = pr.proof_bytes()
    outs = np.ascontiguousarray(gkr.host_elements(pr.outputs))
    del pr
    torch.cuda.empty_cache()
    _log("committed c3: host verifier")
    assert gkr.verify_committed(c, outs, spec.seed, proof, queries) == 1
    _log("committed c3: replay")
    ocirc = oc.Circuit.from_synth(spec, wiring)
    rx, ry, vx, vy, idx, pos = _replay(ocirc, proof[:32], outs, spec.seed, proof, queries)
    assert fast.mle_limbs(inputs, rx) == vx and fast.mle_limbs(inputs, ry) == vy
    s = c.s(spec.depth)
    m = 1 << (s + vpd.LOG_BLOWUP)
    d0 = s + vpd.LOG_BLOWUP - 1
    per_query = (2 + d0) + (4 + d0) + sum(2 + d0 - i for i in range(1, s))
    for j in (0, 1, queries // 2, queries - 1):
        _log("committed c3: query %d (leaf %d)" % (j, idx[j]))
        base = pos + 32 * per_query * j
        f0 = int.from_bytes(proof[base:base + 32], "little")
        f1 = int.from_bytes(proof[base + 32:base + 64], "little")
        x = vpd.point_of_position(2 * idx[j], m, vpd.SHIFT)
        assert f0 == fast.poly_eval_limbs(inputs, x)
        assert f1 == fast.poly_eval_limbs(inputs, (P - x) % P)


def test_committed_data_parallel_matches_oracle_golden(gkr):
    """The committed-input proof of the data-parallel circuit (2^8 copies x
    depth 16, 2^12 gates/layer: 2^20 inputs, a coset of 2^22, transforms of
    three passes) with 64 queries, against the oracle's stored root and digests
    (tests/golden/make_golden.py)."""
    import hashlib
    import json
    import os
    import torch
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "vpd_c2_proof.json")) as f:
        gold = json.load(f)
    spec = gs.data_parallel_c2()
    assert gold["seed"] == spec.seed and gold["log_copies"] == spec.log_copies and gold["depth"] == spec.depth
    wiring = gs.make_wiring(spec)
    c = gkr.Circuit.from_synth(spec, wiring)
    pr = gkr.CommittedProver(c, gold["queries"])
    _log("committed c2 golden: proving")
    pr.prove(gkr.device_elements(gs.make_inputs(spec)), spec.seed)
    torch.cuda.synchronize()
    proof = pr.proof_bytes()
    outs = np.ascontiguousarray(gkr.host_elements(pr.outputs))
    assert len(proof) == gold["proof_len"]
    assert proof[:32].hex() == gold["root_hex"]
    assert hashlib.sha256(outs.tobytes()).hexdigest() == gold["outputs_sha256"]
    assert hashlib.sha256(proof).hexdigest() == gold["proof_sha256"]
    _log("committed c2 golden: host verifier")
    assert gkr.verify_committed(c, outs, spec.seed, proof, gold["queries"]) == 1
