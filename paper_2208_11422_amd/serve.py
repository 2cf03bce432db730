"""Serving loop for light-field deconvolution requests.

Requests arrive over time, each an image for one of several resident PSF sets
(plans).  The loop admits them in arrival order while their device state fits
in a memory budget (the per-job figure of ``lfrl_job_footprint``, in the
spirit of the paper's memory estimate made before anything is placed on the
card, Fig. 1), steps every admitted job one Richardson-Lucy iteration per
round through ``lfrl_job_step`` (jobs of one PSF set share each projection
launch), lets new requests join at every round (continuous batching), and
hands each result volume back to the host as soon as its stop rule fires (the
paper returns only the final result to the CPU, sec. 2.1).

The scheduler is independent of the device: it drives an executor with five
operations (footprint, create, step, result, destroy).  ``JobExecutor`` is
the one backed by the HIP library; tests drive the same scheduler with a
simulated executor.

Failure handling per request: an image the library refuses as numerically
invalid fails that request only; a job whose memory cannot be allocated is put
back at the head of the queue until a running job finishes; a request larger
than the whole budget is rejected at once.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, List, Optional, Sequence

ERR_NOMEM = -2
ERR_NUMERIC = -5


@dataclasses.dataclass
class Request:
    rid: int
    plan: int              # index of the PSF set
    h: int
    w: int
    image: Any             # host image [h][w] (executor-specific type)
    arrival: float = 0.0   # seconds after the start of the run
    # filled in by the loop
    admitted: Optional[float] = None
    finished: Optional[float] = None
    status: str = "pending"   # pending | done | failed | rejected
    error: str = ""
    iters: int = 0
    best_iter: int = 0
    result: Any = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.finished is None else self.finished - self.arrival


class ExecutorError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(msg)
        self.code = code


class Executor:
    """What the scheduler needs from the device side."""

    def footprint(self, req: Request) -> int:
        raise NotImplementedError

    def create(self, req: Request) -> Any:
        """Start a job for req; raise ExecutorError(code) on failure."""
        raise NotImplementedError

    def step(self, handles: Sequence[Any]) -> List[bool]:
        """One iteration for every handle; returns the done flag of each."""
        raise NotImplementedError

    def result_begin(self, handle: Any, req: Request) -> Any:
        """Start handing the job's result to the host (fills req.iters and
        req.best_iter); returns a token.  The job may be destroyed as soon as
        this returns."""
        raise NotImplementedError

    def result_ready(self, token: Any) -> bool:
        """Whether the result volume behind `token` has reached the host."""
        raise NotImplementedError

    def result_finish(self, token: Any, req: Request) -> None:
        """Complete a ready result (req.result for kept requests)."""
        raise NotImplementedError

    def destroy(self, handle: Any) -> None:
        raise NotImplementedError


class Scheduler:
    """FIFO admission under a memory budget with continuous batching."""

    def __init__(self, executor: Executor, budget_bytes: int, max_active: int = 64,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = max_active
        self.clock = clock
        self.sleep = sleep
        self.peak_bytes = 0
        self.peak_active = 0
        self.rounds = 0
        self.batch_sizes: List[int] = []
        self.op_seconds = {"create": 0.0, "step": 0.0, "result": 0.0, "destroy": 0.0,
                           "drain": 0.0}

    def _timed(self, op: str, fn, *a):
        t = self.clock()
        try:
            return fn(*a)
        finally:
            self.op_seconds[op] += self.clock() - t

    def run(self, requests: Sequence[Request]) -> List[Request]:
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: collections.deque = collections.deque()
        active: list = []    # [req, handle, bytes]
        draining: list = []  # [req, token]: result on its way to the host
        used = 0
        nomem_wait = False  # an allocation failed: admit nothing until a job finishes
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731

        def drain():
            still = []
            for req, tok in draining:
                if self.ex.result_ready(tok):
                    self.ex.result_finish(tok, req)
                    req.finished = now()
                    req.status = "done"
                else:
                    still.append([req, tok])
            draining[:] = still

        while pending or queue or active or draining:
            t = now()
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
            if draining:
                self._timed("drain", drain)
            # admission, in arrival order (no overtaking: a large request at
            # the head waits for memory rather than starving)
            while queue and not nomem_wait and len(active) < self.max_active:
                req = queue[0]
                fp = self.ex.footprint(req)
                if fp > self.budget:
                    queue.popleft()
                    req.status, req.error = "rejected", f"needs {fp} bytes, budget {self.budget}"
                    req.finished = now()
                    continue
                if used + fp > self.budget:
                    break
                try:
                    handle = self._timed("create", self.ex.create, req)
                except ExecutorError as e:
                    if e.code == ERR_NOMEM and active:
                        nomem_wait = True     # retry once a running job has finished
                        break
                    queue.popleft()
                    req.status, req.error = "failed", str(e)
                    req.finished = now()
                    continue
                queue.popleft()
                req.admitted = now()
                used += fp
                active.append([req, handle, fp])
            self.peak_bytes = max(self.peak_bytes, used)
            self.peak_active = max(self.peak_active, len(active))
            if not active:
                if queue and not nomem_wait:
                    continue       # head was rejected or failed: look at the next
                if draining or pending:
                    wait = pending[0].arrival - now() if pending else 0.0
                    self.sleep(min(max(wait, 0.0), 0.001) if pending else 0.0001)
                continue
            done = self._timed("step", self.ex.step, [a[1] for a in active])
            self.rounds += 1
            self.batch_sizes.append(len(active))
            still = []
            for (req, handle, fp), d in zip(active, done):
                if not d:
                    still.append([req, handle, fp])
                    continue
                tok = self._timed("result", self.ex.result_begin, handle, req)
                self._timed("destroy", self.ex.destroy, handle)
                used -= fp
                nomem_wait = False
                draining.append([req, tok])
            active = still
        return list(requests)


def latency_stats(reqs: Sequence[Request], span: Optional[float] = None) -> dict:
    """p50 / p99 latency (ms) and frames per second over the completed requests."""
    lat = sorted(r.latency for r in reqs if r.status == "done")
    if not lat:
        return {"completed": 0}

    def pct(p):
        # nearest-rank percentile
        k = max(0, min(len(lat) - 1, int(-(-p * len(lat) // 100)) - 1))
        return lat[k]

    if span is None:
        span = max(r.finished for r in reqs if r.finished is not None) - min(
            r.arrival for r in reqs)
    return {"completed": len(lat), "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99),
            "mean_ms": 1e3 * sum(lat) / len(lat), "frames_per_s": len(lat) / span,
            "failed": sum(r.status == "failed" for r in reqs),
            "rejected": sum(r.status == "rejected" for r in reqs)}


class JobExecutor(Executor):
    """Executor backed by the HIP library's job API.

    ``plans`` are ``paper_2208_11422_amd.Plan`` objects; request images are
    host float32 tensors (pinned for an asynchronous copy).  Each result volume
    is copied to a device buffer, then to a pooled pinned host buffer on a copy
    stream; the results of requests listed in ``keep`` are kept (as host
    tensors) in ``req.result``."""

    def __init__(self, plans, opts_for: Callable[[Request], dict], stream=None, keep=()):
        import torch
        import paper_2208_11422_amd as lf
        self.lf = lf
        self.torch = torch
        self.plans = plans
        self.opts_for = opts_for
        self.stream = stream
        self.device = plans[0].device
        self.keep = set(keep)
        self.pinned = {}                            # numel -> free pinned buffers
        self.copy_stream = torch.cuda.Stream()      # device-to-host result copies

    def footprint(self, req: Request) -> int:
        return self.lf.lfrl_job_footprint(self.plans[req.plan].handle, req.h, req.w)

    def create(self, req: Request):
        img = req.image.to(self.device, non_blocking=True)
        try:
            return self.lf.Job(self.plans[req.plan], img, stream=self.stream,
                               **self.opts_for(req))
        except self.lf.LfrlError as e:
            raise ExecutorError(e.code, str(e))

    def step(self, handles):
        self.lf.Job.step(handles, self.stream)
        return [h.poll()[0] for h in handles]

    def result_begin(self, handle, req: Request):
        vol, rep = handle.result(stream=self.stream)   # device copy; synchronises
        req.iters = rep["iters_run"]
        req.best_iter = rep["best_iter"]
        n = vol.numel()
        free = self.pinned.setdefault(n, [])
        host = free.pop() if free else self.torch.empty(n, dtype=self.torch.float32,
                                                          pin_memory=True)
        with self.torch.cuda.stream(self.copy_stream):
            host.copy_(vol.view(-1), non_blocking=True)
            ev = self.torch.cuda.Event()
            ev.record(self.copy_stream)
        return (vol, host, ev)

    def result_ready(self, token) -> bool:
        return token[2].query()

    def result_finish(self, token, req: Request) -> None:
        vol, host, ev = token
        if req.rid in self.keep:
            req.result = host.view(vol.shape).clone()
        self.pinned.setdefault(host.numel(), []).append(host)

    def destroy(self, handle) -> None:
        handle.close()
