"""Serving on the GPU: requests that arrive while others are being proved join
the running set, and every proof is byte-identical to the same job proved
alone (and, for these sizes, to the oracle's proof)."""
import sys

import pytest

import gkr_synth as gs
from oracle import circuit as oc
from oracle import prover as op

pytestmark = pytest.mark.gpu


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("executor", ["streams", "persistent"])
def test_results_identical_alone_and_in_the_mix(executor):
    import torch

    from paper_2404_10404_amd import gkr, serve
    shapes = [
        (6, 4, 8, 101), (3, 5, 9, 102), (8, 4, 10, 103), (2, 6, 7, 104),
        (5, 4, 12, 105), (4, 7, 6, 106), (7, 4, 9, 107), (3, 4, 11, 108),
    ]
    reqs, refs = [], {}
    for k, (d, n, sig, seed) in enumerate(shapes):
        spec = gs.CircuitSpec(depth=d, log_copies=n, log_sub_width=(sig,) * (d + 1), mu=(1, 2), seed=seed)
        wiring = gs.make_wiring(spec)
        inputs = gs.make_inputs(spec)
        c = gkr.Circuit.from_synth(spec, wiring)
        # arrivals 2 ms apart: later jobs arrive while earlier ones are on the GPU
        reqs.append(serve.Request(rid=k, circuit=c, inputs=inputs, seed=seed, arrival=0.002 * k,
                                  gate_layers=spec.gate_layers))
        refs[k] = op.prove(oc.Circuit.from_synth(spec, wiring), gs.elements_to_ints(inputs), seed).proof_bytes()
    _log("serving: continuous batching (%s) over %d requests" % (executor, len(reqs)))
    ex = serve.StreamExecutor() if executor == "streams" else serve.GpuExecutor()
    mixed = serve.serve(reqs, ex, max_slots=4, budget_bytes=1 << 34)
    _log("serving: the plain loop")
    alone = serve.serve_plain(reqs)
    for k in range(len(reqs)):
        assert mixed[k].error is None
        assert mixed[k].proof == alone[k].proof == refs[k], k
        assert mixed[k].outputs == alone[k].outputs
    # some request was admitted while another was still running
    overlap = any(mixed[j].admitted < mixed[i].done and mixed[j].admitted > mixed[i].admitted
                  for i in mixed for j in mixed if i != j)
    assert overlap
    s = serve.summary(mixed, reqs)
    assert s["jobs"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"]
    torch.cuda.synchronize()


@pytest.mark.parametrize("executor", ["streams", "persistent"])
def test_serving_mix_of_96_matches_plain(executor):
    """The 96-job serving mix (2^12..2^22 gates per layer, depth 8..24), all queued at
    once: up to 32 jobs run together, and the persistent executor's launches end
    whenever a job finishes, so a job's steps are split over many launches while
    other jobs join. Every proof and output vector equals the plain loop's."""
    import torch

    from paper_2404_10404_amd import gkr, serve
    specs = gs.serving_jobs_c5(96)
    reqs = []
    for k, spec in enumerate(specs):
        c = gkr.Circuit.from_synth(spec, gs.make_wiring(spec))
        reqs.append(serve.Request(rid=k, circuit=c, inputs=gs.make_inputs(spec), seed=spec.seed, arrival=0.0,
                                  gate_layers=spec.gate_layers))
    _log("serving mix: the plain loop over %d jobs" % len(reqs))
    alone = serve.serve_plain(reqs)
    _log("serving mix: continuous batching (%s)" % executor)
    ex = serve.StreamExecutor() if executor == "streams" else serve.GpuExecutor()
    mixed = serve.serve(reqs, ex, max_slots=32, budget_bytes=96 << 30)
    torch.cuda.synchronize()
    wrong = [k for k in range(len(reqs)) if mixed[k].proof != alone[k].proof or mixed[k].outputs != alone[k].outputs]
    assert not wrong, wrong
