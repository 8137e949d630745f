"""Continuous-batching server for time-stepping FDE solves on one GPU.

Requests are whole implicit time-stepping jobs (a ``fde_inputs.Problem``:
coefficients, initial state, number of steps).  The server keeps a fixed
number of slots; each slot owns a HIP stream and a host worker thread that
drives the C ABI (ctypes releases the GIL during each call, so the workers
enqueue concurrently).  A request is admitted as soon as a slot is free and
its HBM footprint (``fde_plan_bytes`` plus its state vectors) fits the
budget; requests that arrive while others are on the GPU therefore start
while those are still running, and their kernels overlap on the device.
Per-request state stays on the device for the whole job: the plan (symbol
samples, circulant eigenvalues, twiddles, coefficients, Krylov workspace)
and the current and previous time levels.

Results do not depend on the mix: every reduction in the library sums in a
fixed order within one solve, so a request's iterates are the same alone and
in any mix.

A request can be cancelled by name: a pending one is dropped at once, a
running one stops before its next time step (the step in flight finishes),
and either comes back as a result with status CANCELLED and the steps it
completed.
"""
from __future__ import annotations

import threading
import time
from dataclasses import dataclass, field
from typing import List, Optional

from . import fde


@dataclass
class Result:
    name: str
    arrival: float          # seconds since the stream started
    start: float            # admission time
    finish: float           # completion time
    steps: int
    iters: List[int] = field(default_factory=list)
    inner_iters: List[int] = field(default_factory=list)
    relres: List[float] = field(default_factory=list)
    u: Optional[object] = None   # final state (device tensor) when keep_state
    states: Optional[list] = None  # every step's state (host arrays) when keep_state == "all"
    status: int = 0              # fde status of the failed call (0: every step solved)
    error: str = ""              # its message

    @property
    def ok(self) -> bool:
        return self.status == 0

    @property
    def cancelled(self) -> bool:
        return self.status == CANCELLED

    @property
    def latency(self) -> float:
        return self.finish - self.arrival


AUTO = "auto"
CANCELLED = -100   # Result.status of a cancelled request (a server status, not a library one)
INNER_2D = 16   # float32 inner GMRES steps of a 2D mixed request
MIXED_2D_MIN_N = 511   # smallest 2D grid side served in the mixed form under precision="auto"


def request_kw(problem, solve_kw: dict) -> dict:
    """Solver options of one request, with the per-class choices measured on
    the benchmark's workloads:
      precision="auto": the mixed form for 2D requests from MIXED_2D_MIN_N
        up, where its float32 inner steps move half the bytes (at 511^2 and
        1023^2 about 10 % and 30 % faster than float64), and float64 for
        smaller 2D grids (at 127^2 and 255^2 float64 is 10 % faster: their
        launches, not their bytes, set the pace) and for 1D requests, whose
        long-line iterations are launch-bound too and need fewer iterations
        in float64;
      inner_steps="auto" (mixed requests): GMRES(INNER_2D) in float32 for 2D,
        and no inner steps (the float32 preconditioner alone inside the
        float64 FGMRES) for 1D, where the float32 inner iterations do not pay
        for themselves."""
    kw = dict(solve_kw)
    if kw.get("precision") == AUTO:
        kw["precision"] = fde.MIXED if problem.dim == 2 and min(problem.n) >= MIXED_2D_MIN_N else fde.FP64
    if kw.get("precision") != fde.MIXED:
        kw.pop("inner_steps", None)
    elif kw.get("inner_steps") == AUTO:
        kw["inner_steps"] = INNER_2D if problem.dim == 2 else 0
    return kw


def footprint(problem, **kw) -> int:
    """HBM bytes a request holds while it runs: the plan plus three state vectors."""
    p = fde.params_for(problem, **request_kw(problem, kw))
    return fde.fde_plan_bytes(p) + 3 * problem.N * 8


def run_job(problem, stream=None, keep_state=False, stop=None, **kw):
    """One time-stepping job on the current device: assemble, then for every
    step b = rhs(u), solve M u_new = b from u_new = u.  Returns (infos, u);
    keep_state="all" returns (infos, u, host copies of the state after every
    step) instead (checking only: a host copy per step).  `stop`, if given, is
    called before each step; when it returns true the job ends there (infos
    then covers the steps done)."""
    import torch
    dev = torch.device("cuda", torch.cuda.current_device())
    T = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64, device=dev).reshape(-1).contiguous()
    coef = [T(problem.dplus), T(problem.dminus), T(problem.eplus), T(problem.eminus)]
    u = T(problem.u0)
    x = torch.empty_like(u)
    b = torch.empty_like(u)
    params = fde.params_for(problem, **kw)
    handle = fde.fde_assemble(params, *coef, stream=stream)
    infos, states = [], []
    try:
        for _ in range(problem.steps):
            if stop is not None and stop():
                break
            fde.fde_rhs(handle, u, None, b, stream=stream)
            x.copy_(u)
            infos.append(fde.fde_solve(handle, b, x, stream=stream))
            u, x = x, u
            if keep_state == "all":
                states.append(u.detach().cpu().numpy())
    finally:
        fde.fde_destroy(handle)
    if keep_state == "all":
        return infos, u, states
    return infos, (u if keep_state else None)


class Server:
    """Slots x (stream, worker thread); admission by HBM footprint."""

    def __init__(self, slots: int = 4, hbm_budget: float = 64e9, keep_state: bool = False, **solve_kw):
        import torch
        self.slots = slots
        self.budget = hbm_budget
        self.keep_state = keep_state
        self.solve_kw = solve_kw
        self.streams = [torch.cuda.Stream() for _ in range(slots)]
        self.cv = threading.Condition()
        self.pending: list = []       # (arrival time, request) in arrival order
        self.in_use = 0.0
        self.closed = False
        self.results: List[Result] = []
        self.running: set = set()      # names of the requests in service
        self.cancel_flags: set = set()  # running requests asked to stop
        self.t0 = None
        self.threads = [threading.Thread(target=self._worker, args=(i,), daemon=True) for i in range(slots)]

    def start(self):
        self.t0 = time.perf_counter()
        for t in self.threads:
            t.start()

    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, problem, arrival: Optional[float] = None):
        with self.cv:
            self.pending.append((self.now() if arrival is None else arrival, problem))
            self.cv.notify_all()

    def cancel(self, name: str) -> bool:
        """Cancels the request `name` (the first pending one of that name, else
        a running one).  Returns False when no such request is pending or
        running (it finished already, or never came)."""
        with self.cv:
            for i, (arr, prob) in enumerate(self.pending):
                if prob.name == name:
                    self.pending.pop(i)
                    t = self.now()
                    self.results.append(Result(name, arr, t, t, prob.steps, status=CANCELLED,
                                               error="cancelled before admission"))
                    self.cv.notify_all()
                    return True
            if name in self.running:
                self.cancel_flags.add(name)
                return True
            return False

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()

    def _take(self):
        """Oldest pending request whose footprint fits the free budget."""
        with self.cv:
            while True:
                for i, (arr, prob) in enumerate(self.pending):
                    need = footprint(prob, **self.solve_kw)
                    if self.in_use + need <= self.budget or self.in_use == 0.0:
                        self.pending.pop(i)
                        self.in_use += need
                        return arr, prob, need
                    break   # first come, first served: do not overtake a blocked request
                if self.closed and not self.pending:
                    return None
                self.cv.wait()

    def _release(self, need):
        with self.cv:
            self.in_use -= need
            self.cv.notify_all()

    def _worker(self, slot: int):
        import torch
        stream = self.streams[slot]
        while True:
            item = self._take()
            if item is None:
                return
            arr, prob, need = item
            start = self.now()
            with self.cv:
                self.running.add(prob.name)
            stop = lambda: prob.name in self.cancel_flags
            try:
                states = None
                with torch.cuda.stream(stream):
                    out = run_job(prob, stream=stream.cuda_stream, keep_state=self.keep_state, stop=stop,
                                  **request_kw(prob, self.solve_kw))
                    stream.synchronize()
                infos, u = out[0], out[1]
                if self.keep_state == "all":
                    states = out[2]
                res = Result(prob.name, arr, start, self.now(), prob.steps,
                             [i.iters for i in infos], [i.inner_iters for i in infos],
                             [i.relres_true for i in infos], u, states)
                if len(infos) < prob.steps:
                    res.status = CANCELLED
                    res.error = "cancelled after %d of %d steps" % (len(infos), prob.steps)
            except Exception as e:   # a failed request is reported; the slot keeps serving
                stream.synchronize()
                status = e.status if isinstance(e, fde.FdeError) else fde.FDE_EINVAL
                res = Result(prob.name, arr, start, self.now(), prob.steps, status=status, error=str(e))
            finally:
                self._release(need)
            with self.cv:
                self.running.discard(prob.name)
                self.cancel_flags.discard(prob.name)
                self.results.append(res)


def serve_stream(arrivals, slots: int = 4, hbm_budget: float = 64e9, keep_state: bool = False,
                 time_scale: float = 1.0, **solve_kw):
    """Replays a list of fde_inputs.Arrival (Poisson times) against a Server.
    Returns (results, wall seconds)."""
    srv = Server(slots=slots, hbm_budget=hbm_budget, keep_state=keep_state, **solve_kw)
    srv.start()
    for a in arrivals:
        delay = a.t * time_scale - srv.now()
        if delay > 0:
            time.sleep(delay)
        srv.submit(a.problem, arrival=a.t * time_scale)
    srv.close()
    return srv.results, srv.now()


def latency_stats(results, slots: Optional[int] = None) -> dict:
    """Latency percentiles and throughput over the completed requests; failed
    and cancelled requests are counted separately and contribute no solves.  With `slots`,
    also the utilisation: the fraction of the span during which at least one
    request was in service, the mean number in service, and the mean wait
    between arrival and admission."""
    import numpy as np
    done = [r for r in results if r.ok]
    lat = np.array([r.latency for r in done]) if done else np.zeros(1)
    solves = sum(r.steps for r in done)
    t0 = min(r.arrival for r in results) if results else 0.0
    span = (max(r.finish for r in results) - t0) if results else 0.0
    cancelled = sum(1 for r in results if r.cancelled)
    out = {"requests": len(results), "failed": len(results) - len(done) - cancelled, "cancelled": cancelled,
           "solves": solves,
           "p50_ms": float(1e3 * np.percentile(lat, 50)), "p99_ms": float(1e3 * np.percentile(lat, 99)),
           "mean_ms": float(1e3 * lat.mean()), "solves_per_s": solves / span if span > 0 else 0.0,
           "span_s": span}
    if slots and results and span > 0:
        # busy time: the union of the service intervals
        iv = sorted((r.start, r.finish) for r in results)
        busy, cs, ce = 0.0, iv[0][0], iv[0][1]
        for a, b in iv[1:]:
            if a > ce:
                busy += ce - cs
                cs, ce = a, b
            else:
                ce = max(ce, b)
        busy += ce - cs
        service = sum(r.finish - r.start for r in results)
        out.update(busy_fraction=busy / span, mean_in_service=service / span,
                   slot_utilisation=service / (slots * span),
                   mean_wait_ms=float(1e3 * np.mean([r.start - r.arrival for r in results])))
    return out
