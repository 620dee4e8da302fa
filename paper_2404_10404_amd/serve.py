"""Continuous-batching proof server (the serving form of the prover).

Requests (a circuit, its inputs, a seed, an arrival time) enter a FIFO queue.
The server admits the head of the queue when a slot is free and the job's
device footprint (workspace + proof + inputs + outputs) fits the HBM budget,
uploads its inputs and hands it to an executor; running jobs stay resident
on the device until they finish, then their memory is returned and the next
requests are admitted. Requests that arrive while others are on the GPU join
the running set as slots and memory free up, and their work overlaps on the
device. Two executors:

  StreamExecutor  each admitted proof is enqueued whole (its step launches)
                  on one of a few HIP streams; jobs on different streams run
                  concurrently on the hardware queues, so one job's
                  latency-bound rounds overlap another's bandwidth-bound
                  sweeps. Completion is seen by polling an event per job.
  GpuExecutor     the running set is proved by epochs of the persistent
                  batch kernel; an epoch ends when any job finishes or, when
                  a queued request could be admitted at its arrival, after a
                  step budget sized to end near that arrival (steps are timed
                  as they run); finished jobs retire, new ones are admitted,
                  and the next epoch continues every unfinished job where it
                  stopped.

The plain one-job-at-a-time loop over the same trace is `serve_plain`.
Latency = completion - arrival; p50/p99 use the nearest-rank definition.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Callable, Dict, List, Optional, Sequence


@dataclasses.dataclass
class Request:
    rid: int
    circuit: object          # gkr.Circuit (or anything the executor understands)
    inputs: object           # host canonical limbs, shape (2^{s_d}, 8) uint32
    seed: int
    arrival: float           # seconds after the start of the trace
    footprint: int = 0       # device bytes while admitted (filled by the executor)
    gate_layers: int = 0


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    proof: Optional[bytes] = None
    outputs: Optional[bytes] = None
    error: Optional[str] = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def nearest_rank(values: Sequence[float], q: float) -> float:
    """Nearest-rank percentile (q in (0, 100])."""
    if not values:
        return math.nan
    v = sorted(values)
    k = max(1, math.ceil(q / 100.0 * len(v)))
    return v[k - 1]


class Admission:
    """FIFO admission by free slots and device-memory footprint.

    The head of the queue is admitted when it has arrived, a slot is free and
    its footprint fits what is left of the budget; a later request never
    overtakes the head. A request larger than the whole budget is rejected.
    """

    def __init__(self, max_slots: int, budget_bytes: int):
        if max_slots < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot and a positive budget")
        self.max_slots = max_slots
        self.budget = budget_bytes
        self.used = 0

    def take(self, queue: "collections.deque[Request]", now: float, running: int):
        """Yields ('admit' | 'reject', request) for the requests to act on now."""
        while queue and queue[0].arrival <= now:
            r = queue[0]
            if r.footprint > self.budget:
                queue.popleft()
                yield "reject", r
                continue
            if running >= self.max_slots or self.used + r.footprint > self.budget:
                return
            queue.popleft()
            self.used += r.footprint
            running += 1
            yield "admit", r

    def release(self, r: Request):
        self.used -= r.footprint
        assert self.used >= 0


class Executor:
    """What the server needs from the device (see GpuExecutor)."""

    def footprint(self, r: Request) -> int:
        raise NotImplementedError

    def admit(self, r: Request) -> object:
        raise NotImplementedError

    def epoch(self, running: List[object], timeout: Optional[float] = None) -> None:
        """Advance the running jobs; return once some job has finished or, when
        `timeout` is given, after about that many seconds (the next arrival)."""
        raise NotImplementedError

    def finished(self, slot: object) -> bool:
        raise NotImplementedError

    def retire(self, slot: object, result: Result) -> None:
        raise NotImplementedError


def serve(requests: Sequence[Request], executor: Executor, max_slots: int, budget_bytes: int,
          clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep
          ) -> Dict[int, Result]:
    """Continuous batching over the trace; returns the result of every request."""
    for r in requests:
        r.footprint = executor.footprint(r)
    queue = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
    adm = Admission(max_slots, budget_bytes)
    results = {r.rid: Result(r.rid, r.arrival) for r in requests}
    running = []  # (request, slot)
    t0 = clock()
    while queue or running:
        now = clock() - t0
        for what, r in adm.take(queue, now, len(running)):
            if what == "reject":
                results[r.rid].error = "footprint %d exceeds the budget %d" % (r.footprint, budget_bytes)
                continue
            slot = executor.admit(r)
            results[r.rid].admitted = clock() - t0
            running.append((r, slot))
        if not running:
            if queue:
                sleep(max(0.0, min(0.05, queue[0].arrival - (clock() - t0))))
            continue
        # wake up for the next arrival if it could be admitted now
        timeout = None
        if queue and len(running) < max_slots and adm.used + queue[0].footprint <= budget_bytes:
            timeout = max(0.0, queue[0].arrival - (clock() - t0))
        executor.epoch([s for _, s in running], timeout)
        keep = []
        for r, slot in running:
            if executor.finished(slot):
                res = results[r.rid]
                res.done = clock() - t0
                executor.retire(slot, res)
                adm.release(r)
            else:
                keep.append((r, slot))
        running = keep
    return results


class GpuExecutor(Executor):
    """Runs admitted requests as plans of the persistent batch kernel.

    epoch_step_budget caps every epoch (0: no cap). When the server passes a
    timeout (the next arrival could be admitted then), the epoch's step
    budget is timeout / (seconds per step), the rate measured over earlier
    epochs (min_steps before the first measurement, and never below it), so
    the epoch ends near the arrival instead of at the next completion.
    """

    def __init__(self, epoch_step_budget: int = 0, keep_proofs: bool = True, workgroups: int = -1,
                 min_steps: int = 64, gkr_module=None, torch_module=None,
                 clock: Callable[[], float] = time.perf_counter):
        if torch_module is None:
            import torch as torch_module
        if gkr_module is None:
            from . import gkr as gkr_module
        self.gkr = gkr_module
        self.torch = torch_module
        self.budget = epoch_step_budget
        self.keep = keep_proofs
        self.workgroups = workgroups
        self.min_steps = max(1, int(min_steps))
        self.clock = clock
        self.sec_per_step = None  # measured: epoch wall time / steps completed
        self.ctl = self.torch.zeros(4, dtype=self.torch.int32, device="cuda")

    def epoch_budget(self, timeout: Optional[float]) -> int:
        """Step budget of the next epoch (0 = run until some job finishes)."""
        if timeout is None:
            return self.budget
        if self.sec_per_step is None:
            b = self.min_steps
        else:
            b = max(self.min_steps, int(timeout / self.sec_per_step))
        return min(b, self.budget) if self.budget else b

    def footprint(self, r: Request) -> int:
        c = r.circuit
        return (c.workspace_bytes + c.proof_bytes + 32 * ((1 << c.s(c.depth)) + (1 << c.s(0)))
                + 64 * 1024)

    def admit(self, r: Request):
        torch, gkr = self.torch, self.gkr
        c = r.circuit
        d_in = gkr.device_elements(r.inputs)
        out = torch.empty((1 << c.s(0), 8), dtype=torch.int32, device="cuda")
        proof = gkr.alloc_bytes(c.proof_bytes)
        ws = gkr.alloc_bytes(c.workspace_bytes)
        plan = gkr.Plan(gkr.make_job(c, d_in, r.seed, out, proof, ws))
        return {"r": r, "plan": plan, "bufs": (d_in, out, proof, ws), "done": False}

    def epoch(self, running, timeout=None):
        live = [s for s in running if not s["done"]]
        budget = self.epoch_budget(timeout)
        t0 = self.clock()
        steps = finished = 0
        for k in range(0, len(live), 64):
            self.gkr.run_batch([s["plan"] for s in live[k:k + 64]], self.ctl, workgroups=self.workgroups,
                               step_budget=budget, stop_on_finish=True)
            self.torch.cuda.synchronize()
            ctl = self.ctl.tolist() if hasattr(self.ctl, "tolist") else list(self.ctl)  # one read
            finished += int(ctl[0])
            steps += int(ctl[2])
        dt = self.clock() - t0
        if steps > 0:
            rate = dt / steps
            self.sec_per_step = rate if self.sec_per_step is None else 0.5 * (self.sec_per_step + rate)
        if finished:  # ctl[0] counts the plans that finished in the launch
            for s in live:
                d, t = s["plan"].progress()
                s["done"] = d == t

    def finished(self, slot) -> bool:
        return slot["done"]

    def retire(self, slot, result: Result):
        d_in, out, proof, ws = slot["bufs"]
        c = slot["r"].circuit
        if self.keep:
            result.proof = bytes(proof[: c.proof_bytes].cpu().numpy().tobytes())
            result.outputs = bytes(out.cpu().numpy().tobytes())
        slot["plan"].close()
        slot["bufs"] = None


class StreamExecutor(Executor):
    """Runs each admitted proof whole on one of `streams` HIP streams."""

    def __init__(self, streams: int = 4, keep_proofs: bool = True, poll_s: float = 1e-4):
        import torch

        from . import gkr
        self.gkr = gkr
        self.torch = torch
        self.keep = keep_proofs
        self.poll = poll_s
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        self.load = [0] * len(self.streams)

    def footprint(self, r: Request) -> int:
        c = r.circuit
        return (c.workspace_bytes + c.proof_bytes + 32 * ((1 << c.s(c.depth)) + (1 << c.s(0)))
                + 64 * 1024)

    def admit(self, r: Request):
        torch, gkr = self.torch, self.gkr
        k = min(range(len(self.streams)), key=lambda i: self.load[i])
        s = self.streams[k]
        c = r.circuit
        with torch.cuda.stream(s):
            d_in = gkr.device_elements(r.inputs)
            out = torch.empty((1 << c.s(0), 8), dtype=torch.int32, device="cuda")
            proof = gkr.alloc_bytes(c.proof_bytes)
            ws = gkr.alloc_bytes(c.workspace_bytes)
            gkr.prove_circuit(c, d_in, r.seed, out, proof, ws, stream=s)
            ev = torch.cuda.Event()
            ev.record(s)
        self.load[k] += 1
        return {"r": r, "k": k, "ev": ev, "bufs": (d_in, out, proof, ws), "done": False}

    def epoch(self, running, timeout=None):
        t0 = time.perf_counter()
        while True:
            for s in running:
                if not s["done"] and s["ev"].query():
                    s["done"] = True
            if any(s["done"] for s in running):
                return
            if timeout is not None and time.perf_counter() - t0 >= timeout:
                return
            time.sleep(self.poll)

    def finished(self, slot) -> bool:
        return slot["done"]

    def retire(self, slot, result: Result):
        d_in, out, proof, ws = slot["bufs"]
        c = slot["r"].circuit
        if self.keep:
            result.proof = bytes(proof[: c.proof_bytes].cpu().numpy().tobytes())
            result.outputs = bytes(out.cpu().numpy().tobytes())
        self.load[slot["k"]] -= 1
        slot["bufs"] = None


def serve_plain(requests: Sequence[Request], keep_proofs: bool = True,
                clock: Callable[[], float] = time.perf_counter, sleep: Callable[[float], None] = time.sleep
                ) -> Dict[int, Result]:
    """The plain loop: one proof at a time, in arrival order, with gkr_prove_circuit."""
    import torch

    from . import gkr
    results = {r.rid: Result(r.rid, r.arrival) for r in requests}
    t0 = clock()
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        wait = r.arrival - (clock() - t0)
        if wait > 0:
            sleep(wait)
        res = results[r.rid]
        res.admitted = clock() - t0
        c = r.circuit
        d_in = gkr.device_elements(r.inputs)
        out = torch.empty((1 << c.s(0), 8), dtype=torch.int32, device="cuda")
        proof = gkr.alloc_bytes(c.proof_bytes)
        ws = gkr.alloc_bytes(c.workspace_bytes)
        gkr.prove_circuit(c, d_in, r.seed, out, proof, ws)
        torch.cuda.synchronize()
        res.done = clock() - t0
        if keep_proofs:
            res.proof = bytes(proof[: c.proof_bytes].cpu().numpy().tobytes())
            res.outputs = bytes(out.cpu().numpy().tobytes())
        del d_in, out, proof, ws
    return results


def summary(results: Dict[int, Result], requests: Sequence[Request]) -> dict:
    ok = [r for r in results.values() if r.error is None]
    lat = [r.latency for r in ok]
    span = max(r.done for r in ok) - min(r.arrival for r in ok) if ok else math.nan
    gates = sum(q.gate_layers for q in requests if results[q.rid].error is None)
    return {"jobs": len(ok), "rejected": len(results) - len(ok), "makespan_s": round(span, 4),
            "jobs_per_s": round(len(ok) / span, 3) if ok else None,
            "field_gates_per_s": round(gates / span, 1) if ok else None,
            "p50_latency_s": round(nearest_rank(lat, 50), 5), "p99_latency_s": round(nearest_rank(lat, 99), 5),
            "mean_latency_s": round(sum(lat) / len(lat), 5) if lat else None}
