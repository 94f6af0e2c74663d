"""Continuous-batching server for steady 1D solves (Algorithm 1 per request).

Requests arrive over time; a request is admitted as soon as the device memory it needs fits in
the HBM budget, and from then on its Newton iteration runs inside the same batched launches as
every other admitted request (one plan over all of them, ``nmg_plan_*``).  The server works in
ticks: each tick runs a few Newton steps on the current batch, reads the per-request convergence
state, retires finished requests and admits waiting ones.  When the batch changes, a new plan is
made over the new set and every continuing request resumes from its state on the device with its
step count carried over (``nmg_plan_resume``): no request's arithmetic depends on its
neighbours, so each result is bit for bit the result of solving it alone.

The Newton and multigrid state of every request stays in device memory from admission to
retirement; the host only sees the per-request convergence flags.  The engine (device side) is
pluggable so that the scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Dict, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    prob: Any                 # a swe_workloads.Problem1D
    arrival: float            # seconds from the start of the stream


@dataclasses.dataclass
class Result:
    rid: int
    n: int                    # cells
    iters: int
    status: int
    res: float
    arrival: float
    admitted: float
    finished: float
    footprint: int            # device bytes reserved for the request
    state: Any = None         # the final state (device tensor) when kept

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


@dataclasses.dataclass
class ServeReport:
    results: List[Result]
    ticks: int
    plans: int
    max_batch: int
    mean_batch: float
    peak_bytes: int
    span: float               # first arrival to last completion, seconds
    rejected: List[int]

    @property
    def solves_per_s(self) -> float:
        return len(self.results) / self.span if self.span > 0 else float("nan")

    def latency_ms(self, q: float) -> float:
        lat = np.array([r.latency for r in self.results]) * 1e3
        return float(np.percentile(lat, q)) if len(lat) else float("nan")

    def summary(self) -> Dict[str, Any]:
        return dict(completed=len(self.results), rejected=len(self.rejected),
                    solves_per_s=self.solves_per_s, p50_ms=self.latency_ms(50),
                    p99_ms=self.latency_ms(99), ticks=self.ticks, plans=self.plans,
                    max_batch=self.max_batch, mean_batch=self.mean_batch,
                    peak_bytes=self.peak_bytes, span_s=self.span,
                    converged=all(r.status == 0 for r in self.results))


class GpuEngine:
    """Device side of the server: libnmg's batched plan over the admitted requests."""

    def __init__(self, device="cuda:0", precision: Optional[int] = None, use_graph: bool = True):
        from . import _abi as A
        self.A = A
        self.L = A.load()
        self.device = device
        self.precision = A.NMG_FP32_MG if precision is None else precision
        self.use_graph = use_graph

    def footprint(self, prob) -> int:
        """Workspace of the request alone plus its state and geometry arrays (bytes)."""
        import ctypes as C
        from .solver import params_struct
        A = self.A
        d = A.nmg_desc()
        d.dim, d.nx, d.ny, d.levels, d.jac = 1, prob.n, 1, prob.levels, 3
        d.x0, d.x1, d.y0, d.y1, d.g = prob.x0, prob.x1, 0.0, 1.0, prob.g
        p = params_struct(prob.params, self.precision)
        ws = self.L.nmg_workspace_bytes(C.byref(d), C.byref(p))
        if ws == 0:
            raise A.NmgError(A.NMG_EINVAL, self.L.nmg_last_error().decode())
        n = prob.n
        return int(ws) + 8 * (2 * n) + 8 * ((n + 1) + 3 * (2 * n))

    def prepare(self, prob):
        import torch
        from .solver import Problem1DDevice
        dev = Problem1DDevice(prob, self.device, 3)
        U = torch.tensor(np.ascontiguousarray(prob.initial_guess()), dtype=torch.float64,
                         device=self.device)
        return dict(prob=prob, dev=dev, U=U)

    def batch(self, prepared: Sequence[dict]):
        from .solver import BatchSolver1D
        return _GpuBatch(BatchSolver1D([p["prob"] for p in prepared], device=self.device,
                                       precision=self.precision,
                                       devs=[p["dev"] for p in prepared]),
                         [p["U"] for p in prepared], self.use_graph)

    def state(self, prepared):
        return prepared["U"]


class _GpuBatch:
    def __init__(self, bs, Us, use_graph):
        self.bs = bs
        self.Us = Us
        self.use_graph = use_graph
        self.workspace_bytes = bs.ws_bytes

    def resume(self, n_done: Sequence[int]):
        self.bs.resume(self.Us, n_done)

    def steps(self, k: int):
        return self.bs.steps(k, use_graph=self.use_graph)


class Server:
    """Request loop: admit by HBM footprint, batch every admitted request into each launch,
    retire at convergence (or failure), report latency percentiles and throughput."""

    def __init__(self, engine, hbm_budget: int, steps_per_tick: int = 2,
                 keep_states: bool = False):
        if steps_per_tick < 1:
            raise ValueError("steps_per_tick must be >= 1")
        self.engine = engine
        self.budget = int(hbm_budget)
        self.steps_per_tick = steps_per_tick
        self.keep_states = keep_states

    def run(self, requests: Sequence[Request], clock: Optional[Callable[[], float]] = None,
            sleep: Optional[Callable[[float], None]] = None) -> ServeReport:
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        if clock is None:
            t0 = time.perf_counter()
            clock = lambda: time.perf_counter() - t0          # noqa: E731
        if sleep is None:
            sleep = time.sleep
        waiting: collections.deque = collections.deque()
        active: List[dict] = []          # admitted, still iterating
        results: List[Result] = []
        rejected: List[int] = []
        used = 0
        peak = 0
        nxt = 0
        batch = None
        dirty = True
        ticks = plans = max_batch = 0
        batch_sum = 0
        while nxt < len(reqs) or waiting or active:
            now = clock()
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                nxt += 1
                fp = self.engine.footprint(r.prob)
                if fp > self.budget:
                    rejected.append(r.rid)       # can never fit
                    continue
                waiting.append((r, fp))
            # admission in arrival order, while the budget allows
            while waiting and used + waiting[0][1] <= self.budget:
                r, fp = waiting.popleft()
                active.append(dict(req=r, fp=fp, n_done=0, admitted=now,
                                   prep=self.engine.prepare(r.prob)))
                used += fp
                dirty = True
            peak = max(peak, used)
            if not active:
                if nxt < len(reqs):
                    sleep(max(0.0, reqs[nxt].arrival - clock()))
                continue
            if dirty:
                batch = None                     # release the old plan before making a new one
                batch = self.engine.batch([a["prep"] for a in active])
                batch.resume([a["n_done"] for a in active])
                plans += 1
                dirty = False
            flags, stats = batch.steps(self.steps_per_tick)
            ticks += 1
            batch_sum += len(active)
            max_batch = max(max_batch, len(active))
            done_at = clock()
            keep = []
            for a, f, (iters, status, res) in zip(active, flags, stats):
                a["n_done"] = iters
                if f:
                    keep.append(a)
                    continue
                r = a["req"]
                results.append(Result(r.rid, r.prob.n, iters, status, res, r.arrival, a["admitted"],
                                      done_at, a["fp"],
                                      self.engine.state(a["prep"]) if self.keep_states else None))
                used -= a["fp"]
                dirty = True
            active = keep
        arrivals = [r.arrival for r in reqs]
        span = (max(r.finished for r in results) - min(arrivals)) if results else 0.0
        results.sort(key=lambda r: r.rid)
        return ServeReport(results, ticks, plans, max_batch,
                           batch_sum / ticks if ticks else 0.0, peak, span, rejected)


def stream(count: int, rate: float = 200.0, seed: int = 0, n_min: int = 512,
           n_max: int = 32768) -> List[Request]:
    """A seeded Poisson stream of 1D requests (sizes log-uniform in [n_min, n_max])."""
    from swe_workloads import served_arrivals, served_request
    t = served_arrivals(count, rate, seed)
    return [Request(i, served_request(i, seed, n_min, n_max), float(t[i])) for i in range(count)]
