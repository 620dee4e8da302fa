"""Pins of eq / multilinear extensions (identity polynomial of Section 3.2.2)."""
import itertools
import random

from oracle import mle
from oracle.field import P

R = random.Random(7)


def rnd(k):
    return [R.randrange(P) for _ in range(k)]


def test_eq_sums_to_one_and_is_an_indicator_on_booleans():
    for k in range(0, 6):
        r = rnd(k)
        assert sum(mle.eq_table(r)) % P == 1
        for a in itertools.product([0, 1], repeat=k):
            for b in itertools.product([0, 1], repeat=k):
                assert mle.eq(list(a), list(b)) == (1 if a == b else 0)


def test_eq_table_matches_definition_msb_first():
    r = rnd(4)
    tab = mle.eq_table(r)
    for b in range(16):
        assert tab[b] == mle.eq(r, mle.bits_msb_first(b, 4))
    # variable 1 is the most significant bit
    assert mle.bits_msb_first(0b1000, 4) == [1, 0, 0, 0]


def test_mle_agrees_on_boolean_points_and_two_evaluators_agree():
    for k in range(0, 7):
        v = rnd(1 << k)
        for b in range(1 << k):
            assert mle.evaluate_by_folding(v, mle.bits_msb_first(b, k)) == v[b]
        r = rnd(k)
        assert mle.evaluate_by_folding(v, r) == mle.evaluate_by_eq(v, r)


def test_mle_is_multilinear():
    # V~ restricted to a line in one variable is affine: f(2) = 2 f(1) - f(0)
    v = rnd(32)
    base = rnd(5)
    for j in range(5):
        pts = []
        for t in (0, 1, 2, 3):
            q = list(base)
            q[j] = t
            pts.append(mle.evaluate(v, q))
        assert (pts[2] - 2 * pts[1] + pts[0]) % P == 0
        assert (pts[3] - 3 * pts[1] + 2 * pts[0]) % P == 0


def test_worker_split_identity():
    """f(r) = sum_i beta~(r_worker, i) f^{(i)}(r_local) (distributed PC identity, Section 3.2.2).

    With index g = z * 2^n + c the copy (worker) bits are the last n variables.
    """
    sigma, n = 3, 2
    v = rnd(1 << (sigma + n))
    r = rnd(sigma + n)
    rl, rc = r[:sigma], r[sigma:]
    total = 0
    for c in range(1 << n):
        part = [v[(z << n) | c] for z in range(1 << sigma)]
        total += mle.eq(rc, mle.bits_msb_first(c, n)) * mle.evaluate(part, rl)
    assert total % P == mle.evaluate(v, r)


def test_fold_is_binding_the_msb():
    v = rnd(8)
    r = R.randrange(P)
    f = mle.fold(v, r)
    for b in range(4):
        assert f[b] == (v[b] * (1 - r) + v[b + 4] * r) % P
