"""Autotuner of the round schedule and the batch launch shape.

Tunables (none of them changes proof bytes):
  tail_log          a phase finishes in one workgroup once its tables have at
                    most 2^tail_log entries (below that, a grid-wide round costs
                    more in launch and Fiat-Shamir latency than it saves)
  max_round_blocks  cap on the workgroups of a grid-wide round (more tiles:
                    more parallel partial sums for the last tile to add)
  pairs_per_thread  a grid-wide round gets ceil(pairs / (256 x this)) workgroups
                    (fewer, longer-lived workgroups for mid-size rounds)
  batch_workgroups  resident workgroups of the persistent batch kernel

The tuner times whole proofs of the given workloads for every setting on a
grid, scores a setting by the sum over workloads of its time divided by that
workload's best time on the grid, keeps the setting with the least score, and
writes the grid and the choice to a JSON cache (default: tuning.json next to
this file).
`load()` applies a cached choice; the binding calls it on first use when the
cache exists.

    python -m paper_2404_10404_amd.autotune [--workloads c2,c3,c4] [--reps 3]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")


def load(path: str = CACHE) -> dict | None:
    """Apply the cached tuning (if any); returns the cache record."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    from . import gkr
    best = rec.get("best", {})
    if "tail_log" in best and "max_round_blocks" in best:
        gkr.set_tuning(int(best["tail_log"]), int(best["max_round_blocks"]), int(best.get("pairs_per_thread", 1)))
    return rec


def _plain_workload(gkr, spec):
    import gkr_synth as gs
    c = gkr.Circuit.from_synth(spec, gs.make_wiring(spec))
    prover = gkr.Prover(c)
    d_in = gkr.device_elements(gs.make_inputs(spec))
    return lambda: prover.prove(d_in, spec.seed)


def _time(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def tune(workloads=("c2",), tail_logs=(8, 9, 10, 11), blocks=(512, 1024, 2048, 4096), ppts=(1, 2, 4),
         reps=3, path: str = CACHE) -> dict:
    import torch

    import gkr_synth as gs
    from . import gkr
    specs = {"c1": gs.plain_c1, "c2": gs.data_parallel_c2, "c3": gs.worker_share_c3}
    fns = {w: _plain_workload(gkr, specs[w]()) for w in workloads if w in specs}
    grid = []
    for tl in tail_logs:
        for mb in blocks:
            for ppt in ppts:
                gkr.set_tuning(tl, mb, ppt)
                times = {w: _time(fn, reps) for w, fn in fns.items()}
                grid.append({"tail_log": tl, "max_round_blocks": mb, "pairs_per_thread": ppt, "seconds": times})
                print("tail_log %2d  max_round_blocks %4d  pairs_per_thread %d  %s"
                      % (tl, mb, ppt, {k: round(v * 1e3, 3) for k, v in times.items()}), flush=True)
    best_t = {w: min(g["seconds"][w] for g in grid) for w in fns}
    for g in grid:
        g["score"] = sum(g["seconds"][w] / best_t[w] for w in fns)
    best = min(grid, key=lambda g: g["score"])
    rec = {"device": torch.cuda.get_device_name(0), "workloads": list(fns), "reps": reps, "grid": grid,
           "best": {"tail_log": best["tail_log"], "max_round_blocks": best["max_round_blocks"],
                    "pairs_per_thread": best["pairs_per_thread"]}}
    gkr.set_tuning(best["tail_log"], best["max_round_blocks"], best["pairs_per_thread"])
    if "c4" in workloads:
        rec["batch"] = tune_batch(gkr, reps)
        rec["best"]["batch_workgroups"] = rec["batch"]["best"]
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    return rec


def tune_batch(gkr, reps) -> dict:
    """Resident workgroups of the persistent kernel for the uneven 64-job batch."""
    import torch

    import gkr_synth as gs
    plans, keep = [], []
    for spec in gs.batch_jobs_c4():
        c = gkr.Circuit.from_synth(spec, gs.make_wiring(spec))
        d_in = gkr.device_elements(gs.make_inputs(spec))
        out = torch.zeros((1 << c.s(0), 8), dtype=torch.int32, device="cuda")
        proof = gkr.alloc_bytes(c.proof_bytes)
        ws = gkr.alloc_bytes(c.workspace_bytes)
        keep.append((c, d_in, out, proof, ws))
        plans.append(gkr.Plan(gkr.make_job(c, d_in, spec.seed, out, proof, ws)))
    ctl = torch.zeros(4, dtype=torch.int32, device="cuda")
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    res = {}
    for wg in (cus // 4, cus // 2, (3 * cus) // 4, cus, (3 * cus) // 2, 2 * cus):
        def run():
            for p in plans:
                p.reset()
            gkr.run_batch(plans, ctl, workgroups=wg)
        res[wg] = _time(run, reps)
        print("batch workgroups %4d  %.3f ms" % (wg, res[wg] * 1e3), flush=True)
    best = min(res, key=res.get)
    return {"seconds": {str(k): v for k, v in res.items()}, "best": best}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", default="c2,c3,c4")
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--out", default=CACHE)
    a = ap.parse_args()
    sys.path.insert(0, os.path.dirname(HERE))
    rec = tune(tuple(a.workloads.split(",")), reps=a.reps, path=a.out)
    print(json.dumps(rec["best"]))


if __name__ == "__main__":
    main()
