"""Pins of the oracle's field arithmetic against number theory (BN254 scalar field)."""
import random

import pytest

from oracle import field as F

R = random.Random(12345)


def _miller_rabin(n: int, bases) -> bool:
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in bases:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def test_modulus_is_the_bn254_scalar_prime():
    assert F.P == 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
    assert F.P.bit_length() == 254
    assert _miller_rabin(F.P, [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53])
    # 2-adicity 28: P - 1 = 2^28 * odd
    assert (F.P - 1) % (1 << 28) == 0 and ((F.P - 1) >> 28) % 2 == 1
    # the Miller-Rabin helper rejects composites (so the check above means something)
    assert not _miller_rabin(F.P * 3, [2, 3, 5])
    assert not _miller_rabin(561, [2, 3, 5])  # Carmichael number


EDGE = [0, 1, 2, F.P - 1, F.P - 2, (1 << 128) % F.P, (1 << 253) % F.P, (1 << 256) % F.P, F.HALF]


def _samples(k=60):
    return EDGE + [R.randrange(F.P) for _ in range(k)]


def test_field_laws():
    xs = _samples()
    for _ in range(300):
        a, b, c = R.choice(xs), R.choice(xs), R.choice(xs)
        assert F.add(a, b) == F.add(b, a)
        assert F.mul(a, b) == F.mul(b, a)
        assert F.add(F.add(a, b), c) == F.add(a, F.add(b, c))
        assert F.mul(F.mul(a, b), c) == F.mul(a, F.mul(b, c))
        assert F.mul(a, F.add(b, c)) == F.add(F.mul(a, b), F.mul(a, c))
        assert F.add(a, 0) == a and F.mul(a, 1) == a
        assert F.add(a, F.neg(a)) == 0
        assert F.sub(a, b) == F.add(a, F.neg(b))
        assert 0 <= F.mul(a, b) < F.P


def test_inverse():
    for a in _samples():
        if a == 0:
            with pytest.raises(ZeroDivisionError):
                F.inv(a)
            continue
        assert F.mul(a, F.inv(a)) == 1
    assert F.mul(2, F.HALF) == 1


def test_encoding_roundtrip_and_rejection():
    for a in _samples():
        b = F.to_bytes(a)
        assert len(b) == 32 and F.from_bytes(b) == a
    assert F.to_bytes(1) == b"\x01" + b"\x00" * 31
    with pytest.raises(ValueError):
        F.from_bytes(F.P.to_bytes(32, "little"))
    with pytest.raises(ValueError):
        F.to_bytes(F.P)
    with pytest.raises(ValueError):
        F.from_bytes(b"\x00" * 31)


def test_montgomery_constant_relations():
    """Relations any Montgomery implementation with R = 2^256 must satisfy."""
    Rm = (1 << 256) % F.P
    R2 = Rm * Rm % F.P
    assert Rm * pow(1 << 256, -1, F.P) % F.P == 1
    assert R2 == pow(2, 512, F.P)
    # -P^{-1} mod 2^32, the per-limb Montgomery factor
    n0 = (-pow(F.P, -1, 1 << 32)) % (1 << 32)
    assert (F.P * n0 + 1) % (1 << 32) == 0
