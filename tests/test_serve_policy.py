"""Host-only tests of the serving loop: admission by footprint and slots, FIFO
order, rejection of oversized jobs, continuous batching (late arrivals join
running work), latency bookkeeping. The device is replaced by a fake executor
and the clock by a fake clock."""
import pytest

from paper_2404_10404_amd import serve


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor(serve.Executor):
    """Each request needs `need[rid]` epochs; an epoch costs `dt` seconds."""

    def __init__(self, clock, need, size, dt=1.0):
        self.clock, self.need, self.size, self.dt = clock, need, size, dt
        self.max_used = 0
        self.max_running = 0
        self.admit_order = []
        self.epochs = 0

    def footprint(self, r):
        return self.size[r.rid]

    def admit(self, r):
        self.admit_order.append(r.rid)
        return {"r": r, "left": self.need[r.rid]}

    def epoch(self, running, timeout=None):
        self.epochs += 1
        self.max_running = max(self.max_running, len(running))
        self.max_used = max(self.max_used, sum(self.size[s["r"].rid] for s in running))
        self.clock.t += self.dt
        for s in running:
            s["left"] -= 1

    def finished(self, slot):
        return slot["left"] <= 0

    def retire(self, slot, result):
        result.proof = b"proof-%d" % slot["r"].rid


def _reqs(arrivals):
    return [serve.Request(rid=i, circuit=None, inputs=None, seed=i, arrival=a) for i, a in enumerate(arrivals)]


def test_budget_slots_and_fifo_hold():
    clock = FakeClock()
    arrivals = [0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 5.0, 5.5]
    size = {0: 40, 1: 30, 2: 50, 3: 10, 4: 10, 5: 60, 6: 20, 7: 20}
    need = {i: 1 + (i * 7) % 4 for i in range(8)}
    ex = FakeExecutor(clock, need, size)
    res = serve.serve(_reqs(arrivals), ex, max_slots=3, budget_bytes=100, clock=clock.now, sleep=clock.sleep)
    assert ex.max_used <= 100 and ex.max_running <= 3
    assert ex.admit_order == sorted(ex.admit_order)  # FIFO: nobody overtakes the head
    assert all(r.error is None and r.proof == b"proof-%d" % r.rid for r in res.values())
    for r in res.values():
        assert r.arrival <= r.admitted <= r.done


def test_oversized_request_is_rejected_and_others_proceed():
    clock = FakeClock()
    ex = FakeExecutor(clock, {0: 1, 1: 1, 2: 1}, {0: 10, 1: 500, 2: 10})
    res = serve.serve(_reqs([0.0, 0.0, 0.0]), ex, max_slots=4, budget_bytes=100, clock=clock.now, sleep=clock.sleep)
    assert res[1].error and res[0].error is None and res[2].error is None
    assert ex.admit_order == [0, 2]


def test_late_arrivals_join_running_work():
    """Continuous batching: a short job arriving while a long one runs finishes first."""
    clock = FakeClock()
    ex = FakeExecutor(clock, {0: 10, 1: 1}, {0: 10, 1: 10})
    res = serve.serve(_reqs([0.0, 1.5]), ex, max_slots=4, budget_bytes=100, clock=clock.now, sleep=clock.sleep)
    assert res[1].done < res[0].done
    assert res[1].admitted < res[0].done  # admitted while job 0 was still on the device
    assert res[1].latency < 2.0


def test_queue_waits_for_memory_not_for_arrivals():
    clock = FakeClock()
    # job 1 does not fit next to job 0; it is admitted once job 0 retires
    ex = FakeExecutor(clock, {0: 3, 1: 1}, {0: 80, 1: 50})
    res = serve.serve(_reqs([0.0, 0.0]), ex, max_slots=4, budget_bytes=100, clock=clock.now, sleep=clock.sleep)
    assert res[1].admitted >= res[0].done


def test_nearest_rank():
    v = [5, 1, 4, 2, 3]
    assert serve.nearest_rank(v, 50) == 3
    assert serve.nearest_rank(v, 99) == 5
    assert serve.nearest_rank(v, 20) == 1
    assert serve.nearest_rank(list(range(1, 101)), 99) == 99


def test_admission_rejects_bad_config():
    with pytest.raises(ValueError):
        serve.Admission(0, 10)


class _FakePlan:
    def __init__(self, total):
        self.total, self.done = total, 0

    def progress(self):
        return self.done, self.total

    def close(self):
        pass


class _FakeDevice:
    """Stand-in for the binding and torch under GpuExecutor: run_batch advances
    the plans round-robin one step at a time (each step costs `dt` on the fake
    clock) until the step budget is spent or, with stop_on_finish, a plan
    finishes, and reports the steps it ran in ctl[2], as the persistent kernel
    does."""

    int32 = "int32"

    class cuda:
        @staticmethod
        def synchronize():
            pass

    def __init__(self, clock, steps, dt):
        self.clock, self.steps, self.dt = clock, steps, dt
        self.budgets = []

    # torch-like
    def zeros(self, n, dtype=None, device=None):
        return [0] * n

    def empty(self, shape, dtype=None, device=None):
        return None

    # binding-like
    def device_elements(self, arr):
        return arr

    def alloc_bytes(self, n):
        return None

    def make_job(self, c, d_in, seed, out, proof, ws):
        return seed

    def Plan(self, job):
        return _FakePlan(self.steps[job])

    def run_batch(self, plans, ctl, workgroups=-1, step_budget=0, stop_on_finish=False):
        self.budgets.append(step_budget)
        n = fin = 0
        stop = False
        while not stop and any(p.done < p.total for p in plans):
            for p in plans:
                if p.done >= p.total:
                    continue
                p.done += 1
                n += 1
                fin += p.done == p.total
                self.clock.t += self.dt
                if (stop_on_finish and p.done == p.total) or (step_budget and n >= step_budget):
                    stop = True
                    break
        ctl[0], ctl[2] = fin, n


class _FakeCircuit:
    depth = 1
    workspace_bytes = 1000
    proof_bytes = 100

    def s(self, i):
        return 4


def test_persistent_executor_admits_an_arrival_before_running_jobs_finish():
    """A request that arrives while a slot is free is admitted near its
    arrival, not when the long job already on the device finishes: the epoch
    is cut by a step budget sized from the measured step time."""
    clock = FakeClock()
    dev = _FakeDevice(clock, steps={0: 2000, 1: 20}, dt=0.001)
    ex = serve.GpuExecutor(keep_proofs=False, min_steps=16, gkr_module=dev, torch_module=dev, clock=clock.now)
    reqs = [serve.Request(rid=i, circuit=_FakeCircuit(), inputs=None, seed=i, arrival=a)
            for i, a in enumerate([0.0, 0.5])]
    res = serve.serve(reqs, ex, max_slots=4, budget_bytes=10 ** 9, clock=clock.now, sleep=clock.sleep)
    assert res[1].admitted < res[0].done, "the arrival waited for the running job to finish"
    assert res[1].admitted - reqs[1].arrival < 0.05
    assert res[1].done < res[0].done
    assert ex.sec_per_step == pytest.approx(0.001)
    assert all(b > 0 for b in dev.budgets[:2])  # epochs before the arrival had a budget


def test_persistent_executor_budget_rule():
    clock = FakeClock()
    dev = _FakeDevice(clock, steps={}, dt=0.001)
    ex = serve.GpuExecutor(epoch_step_budget=0, gkr_module=dev, torch_module=dev, clock=clock.now, min_steps=8)
    assert ex.epoch_budget(None) == 0          # no arrival pending: run until a job finishes
    assert ex.epoch_budget(1.0) == 8           # no measurement yet
    ex.sec_per_step = 0.002
    assert ex.epoch_budget(1.0) == 500
    assert ex.epoch_budget(0.0) == 8           # never below min_steps
    capped = serve.GpuExecutor(epoch_step_budget=100, gkr_module=dev, torch_module=dev, clock=clock.now)
    capped.sec_per_step = 0.002
    assert capped.epoch_budget(1.0) == 100 and capped.epoch_budget(None) == 100
