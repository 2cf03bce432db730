"""The serving scheduler on the CPU, against a simulated executor whose jobs
take a modelled number of iterations of modelled duration (no GPU)."""
import pytest

from paper_2208_11422_amd.serve import (ERR_NOMEM, ERR_NUMERIC, Executor, ExecutorError,
                                        Request, Scheduler, latency_stats)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor(Executor):
    """Job state = remaining iterations; one step costs step_s of clock time
    plus per_job_s per job in the batch."""

    def __init__(self, clock, iters_of, step_s=1e-3, per_job_s=2e-4, nomem_once=(),
                 copy_s=0.0):
        self.clock = clock
        self.copy_s = copy_s
        self.iters_of = iters_of
        self.step_s = step_s
        self.per_job_s = per_job_s
        self.nomem_once = set(nomem_once)
        self.live = {}
        self.created = []
        self.max_live_bytes = 0
        self.live_bytes = 0

    def footprint(self, req):
        return req.h * req.w

    def create(self, req):
        if req.image == "nan":
            raise ExecutorError(ERR_NUMERIC, "image has non-finite values")
        if req.rid in self.nomem_once:
            self.nomem_once.discard(req.rid)
            raise ExecutorError(ERR_NOMEM, "out of memory")
        h = object()
        self.live[h] = [self.iters_of(req), req]
        self.created.append(req.rid)
        self.live_bytes += self.footprint(req)
        self.max_live_bytes = max(self.max_live_bytes, self.live_bytes)
        return h

    def step(self, handles):
        self.clock.t += self.step_s + self.per_job_s * len(handles)
        out = []
        for h in handles:
            self.live[h][0] -= 1
            out.append(self.live[h][0] <= 0)
        return out

    def result_begin(self, handle, req):
        req.iters = self.iters_of(req)
        req.best_iter = max(1, req.iters - 1)
        return ("volume", req.rid, self.clock.t + self.copy_s)

    def result_ready(self, token):
        return self.clock.t >= token[2]

    def result_finish(self, token, req):
        req.result = token[:2]

    def destroy(self, handle):
        self.live_bytes -= self.footprint(self.live[handle][1])
        del self.live[handle]


def make(n, arrival_gap=0.0, size=10, image="ok"):
    return [Request(rid=i, plan=i % 2, h=size, w=size, image=image, arrival=i * arrival_gap)
            for i in range(n)]


def test_all_complete_within_budget_in_arrival_order():
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 3 + r.rid % 4)
    reqs = make(20, arrival_gap=0.0005)
    sched = Scheduler(ex, budget_bytes=5 * 100, clock=clk, sleep=clk.sleep)
    sched.run(reqs)
    assert all(r.status == "done" for r in reqs)
    assert ex.created == sorted(ex.created)          # FIFO admission
    assert sched.peak_bytes <= 500 and ex.max_live_bytes <= 500
    assert sched.peak_active == 5                     # the budget, not the count, limits
    assert all(r.iters == 3 + r.rid % 4 for r in reqs)
    assert all(r.finished >= r.admitted >= r.arrival for r in reqs)


def test_continuous_batching_admits_while_others_run():
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 50 if r.rid == 0 else 2)
    reqs = make(4, arrival_gap=0.01)
    sched = Scheduler(ex, budget_bytes=10_000, clock=clk, sleep=clk.sleep)
    sched.run(reqs)
    long = reqs[0]
    for r in reqs[1:]:
        assert r.admitted < long.finished             # joined the running batch
        assert r.finished < long.finished
    assert max(sched.batch_sizes) >= 2


def test_numeric_failure_is_isolated():
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 3)
    reqs = make(6)
    reqs[2].image = "nan"
    Scheduler(ex, budget_bytes=10_000, clock=clk, sleep=clk.sleep).run(reqs)
    assert reqs[2].status == "failed" and "non-finite" in reqs[2].error
    assert all(r.status == "done" for i, r in enumerate(reqs) if i != 2)


def test_allocation_failure_requeues():
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 4, nomem_once={3})
    reqs = make(6)
    sched = Scheduler(ex, budget_bytes=10_000, clock=clk, sleep=clk.sleep)
    sched.run(reqs)
    assert all(r.status == "done" for r in reqs)
    assert ex.created.index(3) > ex.created.index(2)  # retried, order kept
    assert reqs[3].admitted >= min(r.finished for r in reqs[:3])


def test_oversized_request_rejected():
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 2)
    reqs = make(3)
    reqs[1].h = reqs[1].w = 1000
    Scheduler(ex, budget_bytes=5000, clock=clk, sleep=clk.sleep).run(reqs)
    assert reqs[1].status == "rejected"
    assert reqs[0].status == reqs[2].status == "done"
    st = latency_stats(reqs)
    assert st["completed"] == 2 and st["rejected"] == 1


def test_open_loop_waits_for_arrivals():
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 1, step_s=1e-4, per_job_s=0.0)
    reqs = make(5, arrival_gap=0.5)
    Scheduler(ex, budget_bytes=10_000, clock=clk, sleep=clk.sleep).run(reqs)
    for r in reqs:
        assert r.admitted >= r.arrival
        assert r.latency == pytest.approx(1e-4, abs=2e-3)


def test_results_in_flight_to_the_host():
    """A request finishes when its volume reaches the host; its job's memory
    is released when the copy starts, so admission does not wait for it."""
    clk = FakeClock()
    ex = FakeExecutor(clk, iters_of=lambda r: 2, copy_s=0.01)
    reqs = make(4)
    sched = Scheduler(ex, budget_bytes=200, clock=clk, sleep=clk.sleep)
    sched.run(reqs)
    assert all(r.status == "done" and r.result == ("volume", r.rid) for r in reqs)
    for r in reqs:
        assert r.finished - r.admitted >= 0.01
    # two at a time fit the budget; the second pair is admitted before the first
    # pair's volumes have landed
    assert reqs[2].admitted < reqs[0].finished


def test_latency_percentiles():
    reqs = []
    for i in range(100):
        r = Request(rid=i, plan=0, h=1, w=1, image=None, arrival=0.0)
        r.finished = (i + 1) * 1e-3
        r.status = "done"
        reqs.append(r)
    st = latency_stats(reqs, span=1.0)
    assert st["p50_ms"] == pytest.approx(50.0)
    assert st["p99_ms"] == pytest.approx(99.0)
    assert st["frames_per_s"] == pytest.approx(100.0)
