"""Pins of the Goldilocks oracle (oracle/goldilocks.py) against the field's
structure, hashlib, brute-force hypercube sums and the protocol invariants.

The brute-force checks recompute every round polynomial from the layer
relation with multilinear predicates (no bookkeeping tables), mod the
Goldilocks prime, as tests/test_oracle_gkr.py does for BN254."""
import hashlib
import itertools
import random
import struct

import numpy as np
import pytest

import gkr_synth as gs
from oracle import goldilocks as gl
from oracle.circuit import MUL, Circuit
from oracle.mle import bits_msb_first

P = gl.P


def _miller_rabin(n, bases=(2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)):
    d, r = n - 1, 0
    while d % 2 == 0:
        d //= 2
        r += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_goldilocks_prime_structure():
    assert P == 0xFFFFFFFF00000001
    assert _miller_rabin(P)  # deterministic for n < 3.3e24 with these bases
    assert pow(2, 64, P) == (1 << 32) - 1
    assert pow(2, 96, P) == P - 1
    assert (P - 1) % (1 << 32) == 0 and ((P - 1) >> 32) % 2 == 1  # 2-adicity 32
    rng = random.Random(1)
    for _ in range(50):
        a, b, c = (rng.randrange(P) for _ in range(3))
        assert (a * (b + c) - (a * b + a * c)) % P == 0
        if a:
            assert a * pow(a, P - 2, P) % P == 1
    assert gl.HALF * 2 % P == 1


def test_element_encoding_and_generator():
    assert gl.to_bytes(P - 1) == struct.pack("<Q", P - 1)
    with pytest.raises(ValueError):
        gl.to_bytes(P)
    with pytest.raises(ValueError):
        gl.from_bytes(struct.pack("<Q", P))
    spec = gs.CircuitSpec(depth=1, log_copies=2, log_sub_width=(3, 3), seed=4)
    x = gs.make_goldilocks_inputs(spec)
    assert x.dtype == np.uint64 and len(x) == 32 and (x < np.uint64(P)).all()
    assert (gs.make_goldilocks_inputs(spec, 5, 3) == x[5:8]).all()  # any slice alone


def test_transcript_steps():
    tr = gl.Transcript(7)
    assert tr.state == hashlib.sha256(b"SISU-GKR-GL-v1" + struct.pack("<Q", 7)).digest()
    tr.absorb(b"GKRD", b"\x01" * 32)
    want = hashlib.sha256(hashlib.sha256(b"SISU-GKR-GL-v1" + struct.pack("<Q", 7)).digest()
                          + b"GKRD" + b"\x01" * 32).digest()
    assert tr.state == want
    st = tr.state
    r = tr.squeeze()
    assert r == int.from_bytes(hashlib.sha256(st + b"GKRC").digest()[:8], "little") and r < P
    # rejection: a state whose first eight bytes encode a value >= p is rehashed
    tr.state = b"\xff" * 8 + tr.state[8:]
    st = tr.state
    r = tr.accept()
    assert r == int.from_bytes(hashlib.sha256(st + b"GKRC").digest()[:8], "little")
    # a round is one compression of LE64(e0) || LE64(e2) || 47 zero bytes || 0x01
    tr2 = gl.Transcript(9)
    st = tr2.state
    r = tr2.round_challenge(5, P - 2)
    blk = struct.pack("<QQ", 5, P - 2) + bytes(47) + b"\x01"
    from oracle.transcript import compress
    assert tr2.state == compress(st, blk) and r == int.from_bytes(tr2.state[:8], "little")


def test_eq_and_mle_identities():
    rng = random.Random(3)
    r = [rng.randrange(P) for _ in range(4)]
    assert sum(gl.eq_table(r)) % P == 1
    table = [rng.randrange(P) for _ in range(16)]
    assert gl.mle(table, r) == gl.mle_by_eq(table, r)
    for b in range(16):
        assert gl.mle(table, bits_msb_first(b, 4)) == table[b]


def _small(depth, n, sig, seed, mu=(1, 2)):
    spec = gs.CircuitSpec(depth=depth, log_copies=n, log_sub_width=tuple(sig), mu=mu, seed=seed)
    c = Circuit.from_synth(spec, gs.make_wiring(spec))
    inputs = [int(v) for v in gs.make_goldilocks_inputs(spec)]
    return c, inputs


def _cube(k):
    return [list(b) for b in itertools.product([0, 1], repeat=k)]


def _f(c, i, T, W, x, y):
    s1 = c.s(i + 1)
    wx, wy = gl.mle(W, x), gl.mle(W, y)
    acc = 0
    for z, (gx, gy, t) in enumerate(c.flat_gates(i)):
        w = T[z] * gl.mle_by_eq([1 if k == gx else 0 for k in range(1 << s1)], x) % P \
            * gl.mle_by_eq([1 if k == gy else 0 for k in range(1 << s1)], y) % P
        acc += w * (wx * wy if t == MUL else wx + wy)
    return acc % P


@pytest.mark.parametrize("shape", [(2, 0, (2, 2, 2), 1), (2, 1, (1, 2, 1), 2), (1, 0, (0, 3), 4), (2, 2, (0, 1, 0), 5)])
def test_round_polynomials_by_brute_force(shape):
    depth, n, sig, seed = shape
    c, inputs = _small(depth, n, sig, seed)
    layers = gl.evaluate(c, inputs)
    pt = gl.prove(c, inputs, seed)
    u, v = pt.g, None
    for i, lt in enumerate(pt.layers):
        s1 = c.s(i + 1)
        W = layers[i + 1]
        T = gl.combined_eq(u, v, lt.alpha, lt.beta)
        direct = (lt.alpha * gl.mle(layers[i], u) + (lt.beta * gl.mle(layers[i], v) if v else 0)) % P
        assert lt.claim == direct
        for j, e in enumerate(lt.messages1):
            for t in (0, 1, 2, 3):
                brute = sum(_f(c, i, T, W, lt.rx[:j] + [t] + rest, y) for rest in _cube(s1 - j - 1)
                            for y in _cube(s1)) % P
                assert (e[t] if t < 3 else gl.interpolate(e, 3)) == brute
        for j, e in enumerate(lt.messages2):
            for t in (0, 1, 2, 3):
                brute = sum(_f(c, i, T, W, lt.rx, lt.ry[:j] + [t] + rest) for rest in _cube(s1 - j - 1)) % P
                assert (e[t] if t < 3 else gl.interpolate(e, 3)) == brute
        assert lt.vx == gl.mle(W, lt.rx) and lt.vy == gl.mle(W, lt.ry)
        u, v = lt.rx, lt.ry


def test_forward_by_hand_and_wraparound():
    c = Circuit(1, 0, [1, 1], [([0, 1], [1, 1], [MUL, 0])])
    assert gl.evaluate(c, [P - 1, 5])[0] == [(P - 1) * 5 % P, 10]
    assert gl.evaluate(c, [3, P - 1])[0] == [3 * (P - 1) % P, (2 * (P - 1)) % P]


@pytest.mark.parametrize("shape", [(3, 2, (3, 4, 2, 3), 11), (4, 0, (5, 5, 5, 5, 5), 12), (1, 0, (0, 0), 13)])
def test_verifier_accepts_honest_and_rejects_tampered(shape):
    depth, n, sig, seed = shape
    c, inputs = _small(depth, n, sig, seed)
    pt = gl.prove(c, inputs, seed)
    proof = pt.proof_bytes()
    assert len(proof) == gl.proof_length(c)
    assert gl.verify(c, inputs, pt.outputs, seed, proof)
    for k in range(len(proof) // 8):
        bad = bytearray(proof)
        bad[8 * k] ^= 1
        try:
            ok = gl.verify(c, inputs, pt.outputs, seed, bytes(bad))
        except gl.MalformedProof:
            ok = False
        assert not ok, k
    outs = list(pt.outputs)
    outs[0] = (outs[0] + 1) % P
    assert not gl.verify(c, inputs, outs, seed, proof)
