"""Lazy (unreduced) products of the prover's field code, checked on the host
against Python integers: sums of up to 16 Montgomery products with a single
reduction (through the carried 512-bit accumulator and through the column
accumulator), including the all-(p-1) worst case that bounds both."""
import os
import random
import subprocess

import pytest

P = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
R = 1 << 256
RINV = pow(R, -1, P)
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("lazy") / "fr_lazy_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", exe, os.path.join(HERE, "native", "fr_lazy_check.cpp")],
                   check=True)
    return exe


def _hex(v):
    return "%064x" % v


def test_sums_of_products_single_reduction(checker):
    rng = random.Random(7)
    cases = []
    for k in range(1, 17):
        cases.append([(P - 1, P - 1)] * k)                      # accumulator bound
        cases.append([(rng.randrange(P), rng.randrange(P)) for _ in range(k)])
        cases.append([(0, rng.randrange(P))] * k)
    cases.append([(1, 1)])
    lines = ["%d %s" % (len(c), " ".join("%s %s" % (_hex(a), _hex(b)) for a, b in c)) for c in cases]
    out = subprocess.run([checker], input="\n".join(lines) + "\n", capture_output=True, text=True,
                         check=True).stdout.split()
    pos = 0
    for c in cases:
        want = sum(a * b for a, b in c) * RINV % P
        assert int(out[pos], 16) == want, (len(c), c[:1])
        assert int(out[pos + 1], 16) == want, ("columns", len(c), c[:1])
        pos += 2
        if len(c) == 2:
            assert int(out[pos], 16) == want
            pos += 1
        if len(c) == 1:
            assert int(out[pos], 16) == c[0][1] * pow(2, -1, P) % P  # halving
            pos += 1
    assert pos == len(out)
