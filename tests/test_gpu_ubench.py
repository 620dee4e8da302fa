"""The measured ceilings the bench line reads its roofline fractions against
(gkr_ubench): every rate is positive and below what the chip can physically
do, so a wrong operation or byte count in a microbenchmark shows up here.
Kinds 0-3 count 32-bit VALU operations (at most 32 lanes x 4 SIMDs x 256 CUs
per cycle at 2.4 GHz, the fp32 vector rate counted as single operations), kind 4 Montgomery products (each at least 64
multiply-adds), kind 5 bytes of the folding-round access pattern (at most the
8 TB/s HBM peak, and far more than a slow path would reach)."""
import sys

import pytest

pytestmark = pytest.mark.gpu

VALU_ISSUE = 256 * 4 * 32 * 2.4e9


@pytest.fixture(scope="module")
def gkr():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2404_10404_amd import gkr as g
    return g


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_valu_rates_below_issue_rate(gkr, kind):
    rate, ms = gkr.ubench(kind, 256)
    print("kind %d: %.3g op/s in %.3f ms" % (kind, rate, ms), flush=True)
    assert 0.05 * VALU_ISSUE < rate <= VALU_ISSUE * 1.001 and ms > 0


def test_field_product_rate_below_multiply_add_rate(gkr):
    mad, _ = gkr.ubench(0, 256)
    prod, ms = gkr.ubench(4, 16)
    print("field products: %.3g /s in %.3f ms" % (prod, ms), flush=True)
    assert 0 < prod * 64 < mad


def test_round_stream_rate_below_hbm_peak(gkr):
    rate, ms = gkr.ubench(5, 4)
    print("round stream: %.1f GB/s in %.3f ms" % (rate / 1e9, ms), flush=True)
    sys.stdout.flush()
    assert 1.0e12 < rate < 8.0e12
