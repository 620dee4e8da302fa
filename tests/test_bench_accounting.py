"""The bench line's accounting (bench.py), on hand-made inputs: which class the
roofline takes, its bound and fractions, the traffic records read from
profiles/ (and voided when a kernel source changes), and the per-class
fractions. Every expected value below is worked out by hand from the
definitions, not by calling the function under test."""
import json
import os

import pytest

import bench


def _prof():
    # round: 10 launches, 10 ms, 40 GB moved, 1e8 products; forward: shorter
    return {
        "round": {"launches": 10, "ms": 10.0, "bytes": 40e9, "mulmods": 1e8},
        "forward": {"launches": 2, "ms": 4.0, "bytes": 24e9, "mulmods": 0.0},
    }


def test_constants():
    # 8 x 8 limb products for the product, 8 x 8 + 8 for the reduction
    assert bench.MACS_PER_MULMOD == 136
    # 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz, in T operations per second
    assert bench.VALU_PEAK_TOPS == pytest.approx(78.6432)
    assert bench.HBM_PEAK_GBS == 8000.0


def test_roofline_takes_the_longest_class_and_its_hbm_bound():
    r = bench.roofline(_prof(), mac_peak_tops=27.0, stream_gbs=5000.0)
    assert r["kernel"] == "round"
    # 40e9 bytes in 10 ms: 4000 GB/s, half the 8 TB/s peak
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0) and r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(0.5) and r["hbm_frac"] == pytest.approx(0.5)
    assert r["hbm_frac_of_stream"] == pytest.approx(0.8)
    # 1e8 products x 136 multiply-adds in 10 ms: 1.36 T/s of a 27 T/s peak
    assert r["alu_tops"] == pytest.approx(1.36) and r["alu_frac"] == pytest.approx(1.36 / 27.0, abs=1e-4)
    assert r["launches_per_step"] == 10 and r["avg_launch_us"] == pytest.approx(1000.0)
    assert r["algorithmic_bytes_per_launch"] == 4_000_000_000
    assert r["traffic"] is None  # no workload named: no record looked up


def test_roofline_alu_bound_when_products_dominate():
    prof = {"p1": {"launches": 1, "ms": 2.0, "bytes": 1e9, "mulmods": 4e8}}
    r = bench.roofline(prof, mac_peak_tops=27.2)
    # t_hbm = 1e9 / 8e12 = 0.125 ms < t_alu = 4e8 x 136 / 27.2e12 = 2 ms
    assert r["bound"] == "alu"
    assert r["achieved"] == pytest.approx(27.2) and r["frac"] == pytest.approx(1.0)
    assert "hbm_frac_of_stream" not in r
    # without a measured peak the theoretical issue rate is the roof
    r2 = bench.roofline(prof)
    assert r2["peak"] == pytest.approx(78.643, abs=1e-3) and r2["peak_source"] == "theoretical full-rate VALU"


def test_class_fractions():
    out = bench.class_fractions(_prof(), mac_peak_tops=27.0, product_rate=1e11, top=1)
    assert list(out) == ["round"]  # only the longest class with top=1
    d = out["round"]
    assert d["hbm_frac"] == pytest.approx(0.5)
    assert d["alu_frac"] == pytest.approx(1.36 / 27.0, abs=1e-4)
    # 1e8 products in 10 ms = 1e10 per second, a tenth of 1e11
    assert d["product_frac"] == pytest.approx(0.1)
    both = bench.class_fractions(_prof(), mac_peak_tops=27.0)
    assert set(both) == {"round", "forward"} and "alu_frac" not in both["forward"]
    assert both["forward"]["hbm_frac"] == pytest.approx(0.75)  # 24e9 B in 4 ms = 6000 GB/s


def test_traffic_record_is_voided_by_a_source_change(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2404_10404_amd" / "csrc"
    csrc.mkdir(parents=True)
    for name in bench.KERNEL_SOURCES:
        (csrc / name).write_text("// %s\n" % name)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    digest = bench.kernel_sources_digest()
    prof_dir = tmp_path / "profiles"
    prof_dir.mkdir()
    rec = {"kernel": "k_round_a", "workload": "c3", "sources_sha256": digest,
           "read_bytes_per_launch": 700, "write_bytes_per_launch": 300}
    (prof_dir / "k_round_a_x.md").write_text("# summary\n\ntraffic-record: " + json.dumps(rec) + "\n")
    assert bench.traffic_record("k_round_a", "c3") == 1000
    assert bench.traffic_record("k_round_a", "c2") is None  # no record for that workload
    assert bench.traffic_record("k_forward", "c3") is None
    r = bench.roofline(_prof(), workload="c3")
    assert r["traffic"] == 1000
    # any change to a kernel source voids the record
    (csrc / "gkr_bodies.hpp").write_text("// changed\n")
    assert bench.traffic_record("k_round_a", "c3") is None


def test_committed_records_name_their_sources():
    """Every record under profiles/ carries the digest it was taken against,
    the scale factors of the counter calibration and a positive byte count."""
    d = os.path.join(bench.ROOT, "profiles")
    seen = 0
    for name in sorted(os.listdir(d)):
        with open(os.path.join(d, name)) as f:
            for line in f:
                if line.startswith("traffic-record:"):
                    rec = json.loads(line[len("traffic-record:"):])
                    assert len(rec["sources_sha256"]) == 64
                    assert rec["fetch_factor"] == 2.0 and rec["write_factor"] == 1.0
                    assert rec["read_bytes_per_launch"] > 0 and rec["write_bytes_per_launch"] > 0
                    seen += 1
    assert seen >= 4
