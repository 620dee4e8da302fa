"""Pins of the oracle's C helper against the Python oracle (field ops and MLE)."""
import random

import gkr_synth as gs
from oracle import fast, mle
from oracle.field import P

R = random.Random(77)
EDGE = [0, 1, 2, P - 1, P - 2, (1 << 64) % P, (1 << 128) % P, (1 << 192) % P, (1 << 253) % P, (P + 1) // 2]


def test_mulmod_addsub_match_python_ints():
    xs = EDGE + [R.randrange(P) for _ in range(3000)]
    ys = [R.choice(xs) for _ in xs]
    assert fast.mulmod_many(xs, ys) == [x * y % P for x, y in zip(xs, ys)]
    s, d = fast.addsub_many(xs, ys)
    assert s == [(x + y) % P for x, y in zip(xs, ys)]
    assert d == [(x - y) % P for x, y in zip(xs, ys)]
    # all-max operands exercise every carry of the reduction
    big = [P - 1] * 8
    assert fast.mulmod_many(big, big) == [1] * 8


def test_mle_matches_python_oracle():
    for k in (0, 1, 2, 5, 9):
        limbs = gs.field_elements(gs.stream_key(5, gs.PURPOSE_INPUT, k), 1 << k)
        vals = gs.elements_to_ints(limbs)
        r = [R.randrange(P) for _ in range(k)]
        assert fast.mle_limbs(limbs, r) == mle.evaluate(vals, r)
        # Boolean points give table entries
        if k:
            b = R.randrange(1 << k)
            assert fast.mle_limbs(limbs, mle.bits_msb_first(b, k)) == vals[b]


def test_limb_verifier_matches_int_verifier():
    from oracle import circuit as oc
    from oracle import prover as op
    from oracle import verifier as ov
    spec = gs.CircuitSpec(depth=3, log_copies=3, log_sub_width=(5, 6, 4, 5), mu=(1, 2), seed=17)
    wiring = gs.make_wiring(spec)
    limbs = gs.make_inputs(spec)
    c = oc.Circuit.from_synth(spec, wiring)
    pt = op.prove(c, gs.elements_to_ints(limbs), spec.seed)
    outs = gs.ints_to_elements(pt.outputs)
    proof = pt.proof_bytes()
    assert ov.verify_limbs(c, limbs, outs, spec.seed, proof)
    bad = bytearray(proof)
    bad[40] ^= 1
    assert not ov.verify_limbs(c, limbs, outs, spec.seed, bytes(bad))
    outs[3, 0] ^= 1
    assert not ov.verify_limbs(c, limbs, outs, spec.seed, proof)


def test_poly_eval_matches_horner_in_python():
    """The blocked C Horner evaluation against plain Python Horner, across block
    boundaries (2^16 coefficients per block) and at x = 0, 1, -1."""
    from oracle import vpd
    for count in (1, 3, 1 << 16, (1 << 16) + 5):
        limbs = gs.field_elements(gs.stream_key(6, gs.PURPOSE_INPUT, count % 97), count)
        vals = gs.elements_to_ints(limbs)
        for x in (0, 1, P - 1, R.randrange(P)):
            assert fast.poly_eval_limbs(limbs, x) == vpd.poly_eval(vals, x)
