"""The seeded generator: splitmix64 reference values, canonical uniform elements, shapes."""
import dataclasses

import numpy as np

import gkr_synth as gs


def test_splitmix64_reference_outputs():
    # splitmix64 with state 0: published first outputs of the reference generator
    assert [int(v) for v in gs.stream(0, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert gs.stream_at(0, 2) == 0x06C45D188009454F
    assert [int(v) for v in gs.stream(12345, 4, start=2)] == [int(v) for v in gs.stream(12345, 6)[2:]]


def test_elements_are_canonical_and_slices_agree():
    key = gs.stream_key(9, gs.PURPOSE_INPUT)
    full = gs.field_elements(key, 3000)
    vals = gs.elements_to_ints(full)
    assert all(0 <= v < gs.MODULUS for v in vals)
    assert len(set(vals)) == len(vals)
    part = gs.field_elements(key, 100, start=1234)
    assert np.array_equal(part, full[1234:1334])
    assert gs.elements_to_ints(gs.ints_to_elements(vals[:50])) == vals[:50]
    # roughly uniform: the top limb spreads over [0, top limb of the modulus]
    top = full[:, 7].astype(np.float64) / (gs.MODULUS >> 224)
    assert 0.45 < top.mean() < 0.55


def test_wiring_ranges_and_mul_fraction():
    spec = gs.CircuitSpec(depth=3, log_copies=2, log_sub_width=(12, 5, 12, 3), mu=(3, 10), seed=4)
    w = gs.make_wiring(spec)
    for i, layer in enumerate(w):
        assert layer.x.shape == (1 << spec.log_sub_width[i],)
        assert layer.x.max() < 1 << spec.log_sub_width[i + 1]
        assert layer.y.max() < 1 << spec.log_sub_width[i + 1]
        assert set(np.unique(layer.kind)) <= {gs.GATE_ADD, gs.GATE_MUL}
    assert abs(w[0].kind.mean() - 0.3) < 0.03
    assert abs(w[2].kind.mean() - 0.3) < 0.03
    # deterministic
    w2 = gs.make_wiring(spec)
    assert all(np.array_equal(a.x, b.x) and np.array_equal(a.kind, b.kind) for a, b in zip(w, w2))


def test_workload_shapes():
    c1, c2, c3 = gs.plain_c1(), gs.data_parallel_c2(), gs.worker_share_c3()
    assert c1.log_width(0) == 10 and c1.depth == 4 and c1.log_copies == 0
    assert c2.log_width(0) == 20 and c2.log_copies == 8 and c2.depth == 16
    assert c3.log_width(0) == 26 and c3.log_copies == 12 and c3.depth == 24 and c3.mu == (3, 10)
    jobs = gs.batch_jobs_c4()
    assert len(jobs) == 64
    for j in jobs:
        s = j.log_width(0)
        assert 10 <= s <= 18 and 8 <= j.depth <= 32 and 4 <= j.log_copies <= min(10, s - 4)
    srv = gs.serving_jobs_c5()
    assert len(srv) == 256
    for j in srv:
        assert 12 <= j.log_width(0) <= 22 and 8 <= j.depth <= 24
    gaps = gs.poisson_gaps(10000, rate=4.0)
    assert abs(gaps.mean() - 0.25) < 0.02 and gaps.min() >= 0


def test_threaded_generation_matches_blocks():
    key = gs.stream_key(21, gs.PURPOSE_INPUT)
    n = (1 << 21) + 777
    full = gs.field_elements(key, n)  # threaded path
    for off in (0, (1 << 20) - 5, (1 << 21) + 100):
        cnt = min(4096, n - off)
        assert np.array_equal(full[off:off + cnt], gs._field_elements_block(key, cnt, off))


def test_general_wiring_is_seeded_and_in_range():
    spec = gs.GeneralSpec(depth=5, log_copies=2, log_sub_width=(3, 4, 2, 5, 3, 4), max_fanin=3, reach=3,
                          cross=(1, 2), seed=9)
    a, b = gs.make_general_wiring(spec), gs.make_general_wiring(spec)
    for i, (w, v) in enumerate(zip(a, b)):
        for f in ("z", "x", "src", "y", "kind"):
            assert (getattr(w, f) == getattr(v, f)).all()
        assert (w.z[1:] >= w.z[:-1]).all()  # grouped by output gate
        counts = np.bincount(w.z, minlength=1 << spec.log_sub_width[i])
        assert counts.min() >= 1 and counts.max() <= spec.max_fanin
        assert (w.x < 1 << spec.log_sub_width[i + 1]).all()
        assert ((w.src > i) & (w.src <= min(spec.depth, i + spec.reach))).all()
        for j in np.unique(w.src):
            assert (w.y[w.src == j] < 1 << spec.log_sub_width[j]).all()
    other = gs.make_general_wiring(dataclasses.replace(spec, seed=10))
    assert any((w.x != v.x).any() for w, v in zip(a, other) if len(w.x) == len(v.x)) or \
        [len(w.x) for w in a] != [len(w.x) for w in other]
