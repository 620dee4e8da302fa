"""Device parity of the prover's field code on edge operands.

The kernels run the device branch of paper_2404_10404_amd/csrc/fr.hpp (inline
v_mad_u64_u32 / v_addc multiply-accumulates, the product-scanning Montgomery
product, lazy 512-bit and column accumulators). tests/native/libfrcheck.so
(built by build() from tests/native/fr_device_check.hip) runs each routine
on the GPU, one case per thread; every result is compared with Python
integers: 0, 1, 2, p-1, p-2, (p-1)/2, (p+1)/2, 2^k mod p, R mod p and
random values, all pairs, and sums of up to 16 products of p-1 (the bound
of both lazy accumulators).
"""
import ctypes
import os
import random
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
R = 1 << 256
RINV = pow(R, -1, P)
HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "native", "libfrcheck.so")

EDGE = sorted({0, 1, 2, 3, P - 1, P - 2, (P - 1) // 2, (P + 1) // 2, R % P, (R * R) % P,
               (1 << 32) % P, (1 << 64) % P, (1 << 128) % P, (1 << 253) % P, (1 << 254) % P,
               (1 << 255) % P, 0xFFFFFFFF, P - (1 << 32), 0x0E0A77C19A07DF2F666EA36F7879462E36FC76959F60CD29AC96341C4FFFFFFB})


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _limbs(vals):
    a = np.zeros((len(vals), 8), dtype=np.uint32)
    for i, v in enumerate(vals):
        for k in range(8):
            a[i, k] = (v >> (32 * k)) & 0xFFFFFFFF
    return a


def _ints(arr):
    return [sum(int(arr[i, k]) << (32 * k) for k in range(8)) for i in range(arr.shape[0])]


@pytest.fixture(scope="module")
def run():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    if not os.path.exists(LIB):
        raise ImportError("tests/native/libfrcheck.so is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB)
    L.frcheck_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                              ctypes.c_uint32]
    L.frcheck_run.restype = ctypes.c_int

    def go(op, terms, a_vals, b_vals):
        n = len(a_vals) // terms
        da = torch.from_numpy(_limbs(a_vals).view(np.int32)).cuda()
        db = torch.from_numpy(_limbs(b_vals).view(np.int32)).cuda()
        out = torch.zeros((max(1, n), 8), dtype=torch.int32, device="cuda")
        _log("frcheck op %d terms %d cases %d" % (op, terms, n))
        rc = L.frcheck_run(op, terms, da.data_ptr(), db.data_ptr(), out.data_ptr(), n)
        assert rc == 0, rc
        return _ints(out.cpu().numpy().view(np.uint32)[:n])
    return go


def _pairs():
    rng = random.Random(2024)
    vals = EDGE + [rng.randrange(P) for _ in range(12)]
    a = [x for x in vals for _ in vals]
    b = [y for _ in vals for y in vals]
    return a, b


def test_product_and_add_sub_on_edge_pairs(run):
    a, b = _pairs()
    assert run(0, 1, a, b) == [x * y * RINV % P for x, y in zip(a, b)]
    assert run(4, 1, a, b) == [(x - y) % P for x, y in zip(a, b)]
    assert run(5, 1, a, b) == [(x + y) % P for x, y in zip(a, b)]


def test_unary_ops(run):
    rng = random.Random(5)
    vals = EDGE + [rng.randrange(P) for _ in range(64)]
    assert run(6, 1, vals, vals) == [x * pow(2, -1, P) % P for x in vals]
    assert run(7, 1, vals, vals) == [2 * x % P for x in vals]
    assert run(8, 1, vals, vals) == [x * R % P for x in vals]
    assert run(9, 1, vals, vals) == [x * RINV % P for x in vals]


def test_mul_add2(run):
    rng = random.Random(11)
    cases = [(P - 1, P - 1, P - 1, P - 1), (0, 0, 0, 0), (1, 1, P - 1, P - 1), (P - 1, 1, 1, P - 1)]
    cases += [(rng.choice(EDGE), rng.choice(EDGE), rng.choice(EDGE), rng.choice(EDGE)) for _ in range(200)]
    cases += [tuple(rng.randrange(P) for _ in range(4)) for _ in range(200)]
    a = [v for c in cases for v in (c[0], c[2])]
    b = [v for c in cases for v in (c[1], c[3])]
    assert run(1, 2, a, b) == [(c[0] * c[1] + c[2] * c[3]) * RINV % P for c in cases]


@pytest.mark.parametrize("op", [2, 3])
def test_lazy_sums_up_to_the_accumulator_bound(run, op):
    rng = random.Random(100 + op)
    for terms in range(1, 17):
        cases = [[(P - 1, P - 1)] * terms, [(P - 1, P - 2)] * terms, [(0, P - 1)] * terms]
        cases += [[(rng.choice(EDGE), rng.choice(EDGE)) for _ in range(terms)] for _ in range(40)]
        cases += [[(rng.randrange(P), rng.randrange(P)) for _ in range(terms)] for _ in range(40)]
        a = [x for c in cases for x, _ in c]
        b = [y for c in cases for _, y in c]
        want = [sum(x * y for x, y in c) * RINV % P for c in cases]
        assert run(op, terms, a, b) == want, (op, terms)
