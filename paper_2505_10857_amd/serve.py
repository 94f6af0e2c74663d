"""Continuous-batching server for steady 1D and 2D solves (Algorithm 1 per request).

Requests arrive over time and wait in one queue per lane (1D, 2D); a request is admitted, in
arrival order within its lane, as soon as the device memory it needs fits in the HBM budget (a
2D request also needs a free 2D worker), so a large 2D request that must wait never holds up the
1D requests behind it.  1D requests then run inside the same batched launches as every
other admitted 1D request (one plan over all of them, ``nmg_plan_*``).  The server works in
ticks: each tick runs a few Newton steps on the 1D batch and reads the per-request convergence
state.  A request that converges is retired at once (its result recorded); its slot stays in the
plan, skipped by every launch, until the plan is rebuilt, which happens when new requests join,
when more than half of the slots are retired, or when the memory they hold is needed to admit the
next request.  A rebuilt plan resumes every continuing request from its state on the device with
its step count carried over (``nmg_plan_resume``): no request's arithmetic depends on its
neighbours, so each result is bit for bit the result of solving it alone.

2D requests are solved in admission order by worker threads, each on a stream of its own
(``nmg_newton_solve``; the library call releases the interpreter lock): a 2D Newton step is
hundreds of launches, whose enqueueing can wait for queue space on the device, so it must not
hold up the loop, which only polls for finished 2D requests.  A small 2D grid keeps only a few
compute units busy (its passes are short chains of dependent launches), so several 2D requests
in flight at once, and the 1D lane beside them, share the device.  Every lane's stream sits on a
hardware queue of its own, so that no 1D launch waits behind a 2D solve.

A request whose iteration breaks down is retried once with a smaller SOR weight; a run can be
stopped at a given time, the requests then unfinished being counted.

The Newton and multigrid state of every request stays in device memory from admission to
retirement; the host only sees the convergence flags.  The engine (device side) is pluggable so
that the scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import dataclasses
import queue
import threading
import time
from typing import Any, Callable, Dict, List, Optional, Sequence

import numpy as np

from ._abi import NMG_ENONFINITE


@dataclasses.dataclass
class Request:
    rid: int
    prob: Any                 # a swe_workloads.Problem1D
    arrival: float            # seconds from the start of the stream


@dataclasses.dataclass
class Result:
    rid: int
    n: int                    # cells (nx * ny in 2D)
    iters: int
    status: int
    res: float
    arrival: float
    admitted: float
    finished: float
    footprint: int            # device bytes reserved for the request
    state: Any = None         # the final state (device tensor) when kept
    dim: int = 1
    retries: int = 0          # 1 when the result is the retry's (smaller SOR weight)

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
    unfinished: int = 0       # requests still waiting or iterating when the run was stopped

    @property
    def solves_per_s(self) -> float:
        return len(self.results) / self.span if self.span > 0 else float("nan")

    def latency_ms(self, q: float, dim: Optional[int] = None) -> float:
        lat = np.array([r.latency for r in self.results if dim is None or r.dim == dim]) * 1e3
        return float(np.percentile(lat, q)) if len(lat) else float("nan")

    def summary(self) -> Dict[str, Any]:
        out = dict(completed=len(self.results), rejected=len(self.rejected), unfinished=self.unfinished,
                   solves_per_s=self.solves_per_s, p50_ms=self.latency_ms(50),
                   p99_ms=self.latency_ms(99), ticks=self.ticks, plans=self.plans,
                   max_batch=self.max_batch, mean_batch=self.mean_batch,
                   peak_bytes=self.peak_bytes, span_s=self.span,
                   converged=all(r.status == 0 for r in self.results),
                   retried=sum(r.retries for r in self.results))
        bad = [r for r in self.results if r.status != 0]
        if bad:
            out["not_converged"] = [dict(rid=r.rid, dim=r.dim, n=r.n, status=r.status, iters=r.iters,
                                         res=r.res) for r in bad[:8]]
        n2 = sum(1 for r in self.results if r.dim == 2)
        if n2:
            out.update(completed_1d=len(self.results) - n2, completed_2d=n2,
                       p50_ms_1d=self.latency_ms(50, 1), p99_ms_1d=self.latency_ms(99, 1),
                       p50_ms_2d=self.latency_ms(50, 2), p99_ms_2d=self.latency_ms(99, 2))
        return out


class GpuEngine:
    """Device side of the server: libnmg's batched plan over the admitted requests.

    Each lane (the 1D batch, every 2D worker) works on a stream of its own, by default one on a
    hardware queue of its own (nmg_lane_stream_create): on ordinary streams, which the runtime
    spreads over four hardware queues, a 2D worker could share the 1D lane's queue (or the null
    stream's) and every 1D launch would then wait behind its solve.  The engine's device work
    (geometry and state uploads included) stays on the lanes, none on the null stream."""

    def __init__(self, device="cuda:0", precision: Optional[int] = None, use_graph: bool = True,
                 workers_2d: int = 3, dedicated_queues: bool = True):
        from . import _abi as A
        self.A = A
        self.L = A.load()
        self.device = device
        self.precision = A.NMG_FP32_MG if precision is None else precision
        self.use_graph = use_graph
        self.dedicated_queues = dedicated_queues
        self._jobs2d: Optional[queue.Queue] = None
        self._workers: List[threading.Thread] = []
        self.workers_2d = max(1, workers_2d)
        self._stream1d = None
        self._handle1d = None

    def _new_lane(self):
        """(torch stream, handle to destroy or None) for one lane, on the engine's device."""
        import ctypes as C
        import torch
        if not self.dedicated_queues:
            return torch.cuda.Stream(self.device), None
        with torch.cuda.device(self.device):
            h = C.c_void_p()
            self.A.check(self.L.nmg_lane_stream_create(C.byref(h)))
        return torch.cuda.ExternalStream(h.value, device=self.device), h.value

    def _lane1d(self):
        if self._stream1d is None:
            self._stream1d, self._handle1d = self._new_lane()
        return self._stream1d

    @staticmethod
    def is2d(prob) -> bool:
        return hasattr(prob, "ny")

    def footprint(self, prob) -> int:
        """Workspace of the request alone plus its state and geometry arrays (bytes)."""
        import ctypes as C
        from .solver import params_struct
        A = self.A
        if self.is2d(prob):
            d = A.nmg_desc()
            d.dim, d.nx, d.ny, d.levels, d.jac, d.recon = 2, prob.nx, prob.ny, prob.levels, 9, getattr(prob, "recon", 0)
            d.x0, d.x1, d.y0, d.y1, d.g = prob.x0, prob.x1, prob.y0, prob.y1, prob.g
            for k, bc in enumerate(prob.bc):
                d.bc[k].kind = bc.kind
            p = params_struct(prob.params, self.precision)
            ws = self.L.nmg_workspace_bytes(C.byref(d), C.byref(p))
            if ws == 0:
                raise A.NmgError(A.NMG_EINVAL, self.L.nmg_last_error().decode())
            n = prob.nx * prob.ny
            return int(ws) + 8 * 3 * n + 8 * 8 * n
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
        with torch.cuda.stream(self._lane1d()):
            dev = Problem1DDevice(prob, self.device, 3)
            U = torch.tensor(np.ascontiguousarray(prob.initial_guess()), dtype=torch.float64,
                             device=self.device)
        return dict(prob=prob, dev=dev, U=U)

    # ---- 2D lane: a worker thread solves the admitted 2D requests in order on its own stream

    def _work2d(self):
        import torch
        from .solver import Solver2D
        torch.cuda.set_device(self.device)
        side, handle = self._new_lane()
        while True:
            job = self._jobs2d.get()
            if job is None:
                if handle is not None:
                    self.A.check(self.L.nmg_lane_stream_destroy(handle))
                return
            try:
                with torch.cuda.stream(side):
                    s = Solver2D(job["prob"], device=self.device, precision=self.precision, check_every=4)
                    U = s.state()
                    st, _ = s.newton_solve(U)
                side.synchronize()
                job["U"] = U
                job["out"] = (0, st.iters, st.status, st.res)
            except Exception as e:         # reported by poll2d in the loop's thread
                job["error"] = e
            job["done"].set()

    def prepare2d(self, prob):
        return dict(prob=prob, done=threading.Event(), out=None, U=None)

    def start2d(self, job):
        if not self._workers:
            self._jobs2d = queue.Queue()
            for _ in range(self.workers_2d):
                t = threading.Thread(target=self._work2d, daemon=True)
                t.start()
                self._workers.append(t)
        self._jobs2d.put(job)

    def poll2d(self, job):
        """None while the request is queued or iterating; then (0, iters, status, res)."""
        if not job["done"].is_set():
            return None
        if "error" in job:
            raise job["error"]
        return job["out"]

    def state2d(self, job):
        return job["U"]

    def close(self):
        """Stop the 2D workers: jobs still queued are dropped, running solves are waited for."""
        if self._jobs2d is not None:
            while True:
                try:
                    self._jobs2d.get_nowait()
                except queue.Empty:
                    break
        for _ in self._workers:
            self._jobs2d.put(None)
        for t in self._workers:
            t.join()
        self._workers = []
        if self._handle1d is not None:
            self.A.check(self.L.nmg_lane_stream_destroy(self._handle1d))
        self._stream1d = self._handle1d = None

    def batch(self, prepared: Sequence[dict]):
        import torch
        from .solver import BatchSolver1D
        # the 1D lane's stream (its plans capture and replay their graphs on it, with no stream
        # of their own to create) already holds the uploads of prepare(), in order
        with torch.cuda.stream(self._lane1d()):
            bs = BatchSolver1D([p["prob"] for p in prepared], device=self.device, precision=self.precision,
                               devs=[p["dev"] for p in prepared])
        return _GpuBatch(bs, [p["U"] for p in prepared], self.use_graph, self._stream1d)

    def state(self, prepared):
        return prepared["U"]


class _GpuBatch:
    def __init__(self, bs, Us, use_graph, stream):
        self.bs = bs
        self.Us = Us
        self.use_graph = use_graph
        self.stream = stream
        self.workspace_bytes = bs.ws_bytes

    def resume(self, n_done: Sequence[int]):
        import torch
        with torch.cuda.stream(self.stream):
            self.bs.resume(self.Us, n_done)

    def steps(self, k: int):
        import torch
        with torch.cuda.stream(self.stream):
            return self.bs.steps(k, use_graph=self.use_graph)


class Server:
    """Request loop: admit by HBM footprint, batch every admitted request into each launch,
    retire at convergence (or failure), report latency percentiles and throughput.

    lanes_2d_busy, when set, caps the 2D solves running while 1D requests are waiting or iterating
    (the engine's worker count applies otherwise): a policy for engines whose 2D solves slow the
    1D batch down (their lanes sharing its hardware queue, or the device full).

    retry_omega: a request whose iteration breaks down (a non-finite residual or a non-positive
    depth) is queued once more, at its arrival, with this SOR weight when its own is larger (a
    V-cycle that diverges at the larger weight on a strongly varying channel converges at the
    smaller one); None turns retries off."""

    def __init__(self, engine, hbm_budget: int, steps_per_tick: int = 2,
                 keep_states: bool = False, trace: bool = False, lanes_2d_busy: Optional[int] = None,
                 retry_omega: Optional[float] = 0.6):
        if steps_per_tick < 1:
            raise ValueError("steps_per_tick must be >= 1")
        if lanes_2d_busy is not None and lanes_2d_busy < 1:
            raise ValueError("lanes_2d_busy must be >= 1")
        self.engine = engine
        self.budget = int(hbm_budget)
        self.steps_per_tick = steps_per_tick
        self.keep_states = keep_states
        self.trace = [] if trace else None      # (start, seconds, what) of the loop's phases
        self.lanes_2d_busy = lanes_2d_busy
        self.retry_omega = retry_omega

    def _retried(self, prob):
        """The request's problem with the retry's SOR weight, or None when there is no retry."""
        par = getattr(prob, "params", None)
        if self.retry_omega is None or par is None or not dataclasses.is_dataclass(prob) \
                or par.omega <= self.retry_omega:
            return None
        return dataclasses.replace(prob, params=dataclasses.replace(par, omega=self.retry_omega))

    def run(self, requests: Sequence[Request], clock: Optional[Callable[[], float]] = None,
            sleep: Optional[Callable[[float], None]] = None, poll: float = 2e-4,
            stop_after: Optional[float] = None) -> ServeReport:
        """Serve the stream; stop_after (seconds from the start) ends the run early, counting the
        requests not completed by then as unfinished."""
        reqs = sorted(requests, key=lambda r: (r.arrival, r.rid))
        if clock is None:
            t0 = time.perf_counter()
            clock = lambda: time.perf_counter() - t0          # noqa: E731
        if sleep is None:
            sleep = time.sleep
        eng = self.engine
        is2d = getattr(eng, "is2d", lambda prob: False)
        lanes_2d = getattr(eng, "workers_2d", 1 << 30)
        waiting: collections.deque = collections.deque()      # 1D
        waiting2: collections.deque = collections.deque()     # 2D
        plan_items: List[dict] = []      # the 1D plan's requests in plan order (retired ones kept
        pending: List[dict] = []         # until it is rebuilt); admitted 1D requests not yet in it
        active2d: List[dict] = []
        results: List[Result] = []
        rejected: List[int] = []
        retried: set = set()
        used = held = 0                  # held: bytes of retired 1D requests still in the plan
        peak = 0
        nxt = 0
        batch = None
        ticks = plans = max_batch = 0
        batch_sum = 0

        def phase(what, t0):
            if self.trace is not None:
                self.trace.append((t0, clock() - t0, what))

        def record(a, iters, status, res, t, state, dim, cells):
            r = a["req"]
            if status == NMG_ENONFINITE and not a.get("retry"):
                prob = self._retried(r.prob)
                if prob is not None:
                    # admitted before every request still waiting in its lane: first in line
                    (waiting2 if dim == 2 else waiting).appendleft((Request(r.rid, prob, r.arrival), a["fp"]))
                    retried.add(r.rid)
                    return
            results.append(Result(r.rid, cells, iters, status, res, r.arrival, a["admitted"], t, a["fp"],
                                  state if self.keep_states else None, dim, int(r.rid in retried)))

        stopped = False
        while nxt < len(reqs) or waiting or waiting2 or pending or active2d or \
                any(not a["retired"] for a in plan_items):
            now = clock()
            if stop_after is not None and now >= stop_after:
                stopped = True
                break
            while nxt < len(reqs) and reqs[nxt].arrival <= now:
                r = reqs[nxt]
                nxt += 1
                fp = eng.footprint(r.prob)
                if fp > self.budget:
                    rejected.append(r.rid)       # can never fit
                    continue
                (waiting2 if is2d(r.prob) else waiting).append((r, fp))
            # admission in arrival order within each lane, while the budget allows; the memory of
            # retired 1D slots is reclaimed (the plan rebuilt without them) when a request needs it
            while True:
                heads = []
                if waiting:
                    heads.append(waiting)
                busy1d = waiting or pending or any(not a["retired"] for a in plan_items)
                cap2 = min(lanes_2d, self.lanes_2d_busy) if busy1d and self.lanes_2d_busy else lanes_2d
                if waiting2 and len(active2d) < cap2:
                    heads.append(waiting2)
                if not heads:
                    break
                q = min(heads, key=lambda d: d[0][0].arrival)
                r, fp = q[0]
                if used + fp > self.budget:
                    if held and used - held + fp <= self.budget:
                        plan_items = [a for a in plan_items if not a["retired"]]
                        used -= held
                        held = 0
                        batch = None
                        pending = plan_items + pending
                        plan_items = []
                        continue
                    # this lane's head waits; the other lane may still admit
                    others = [d for d in heads if d is not q]
                    if others and used + others[0][0][1] <= self.budget:
                        q = others[0]
                        r, fp = q[0]
                    else:
                        break
                q.popleft()
                a = dict(req=r, fp=fp, n_done=0, admitted=now, retired=False, retry=r.rid in retried)
                t_a = clock()
                if is2d(r.prob):
                    a["prep"] = eng.prepare2d(r.prob)
                    eng.start2d(a["prep"])
                    active2d.append(a)
                    phase("admit2d", t_a)
                else:
                    a["prep"] = eng.prepare(r.prob)
                    pending.append(a)
                    phase("admit1d", t_a)
                used += fp
            peak = max(peak, used)
            # 2D lane: retire finished requests, keep the others' chunks going (never waits)
            t_p = clock()
            for a in list(active2d):
                out = eng.poll2d(a["prep"])
                if out is None:
                    continue
                act, iters, status, res = out
                a["n_done"] = iters
                if not act:
                    p2 = a["req"].prob
                    record(a, iters, status, res, clock(), eng.state2d(a["prep"]), 2, p2.nx * p2.ny)
                    used -= a["fp"]
                    active2d.remove(a)
            if active2d:
                phase("poll2d", t_p)
            # 1D lane: rebuild the plan when requests join or most of its slots are retired
            live = [a for a in plan_items if not a["retired"]]
            if pending or (plan_items and 2 * len(live) < len(plan_items)):
                plan_items = live + pending
                pending = []
                used -= held
                held = 0
                t_b = clock()
                batch = None                     # release the old plan before making a new one
                if plan_items:
                    batch = eng.batch([a["prep"] for a in plan_items])
                    batch.resume([a["n_done"] for a in plan_items])
                    plans += 1
                phase("plan", t_b)
                live = plan_items
            elif plan_items and not live:
                plan_items = []                  # every slot retired: release the plan
                used -= held
                held = 0
                batch = None
            if live:
                t_s = clock()
                flags, stats = batch.steps(self.steps_per_tick)
                phase("steps", t_s)
                ticks += 1
                batch_sum += len(live)
                max_batch = max(max_batch, len(live))
                done_at = clock()
                for a, f, (iters, status, res) in zip(plan_items, flags, stats):
                    if a["retired"]:
                        continue
                    a["n_done"] = iters
                    if f:
                        continue
                    a["retired"] = True
                    held += a["fp"]
                    record(a, iters, status, res, done_at, eng.state(a["prep"]), 1, a["req"].prob.n)
            elif active2d:
                # only 2D chunks in flight: poll them, but wake for the next arrival
                due = reqs[nxt].arrival - clock() if nxt < len(reqs) else poll
                sleep(max(0.0, min(poll, due)))
            elif nxt < len(reqs) and not waiting:
                due = reqs[nxt].arrival - clock()
                sleep(max(0.0, due if not waiting2 else min(poll, due)))
            elif waiting2:
                sleep(poll)                      # 2D requests wait for memory or a worker
        arrivals = [r.arrival for r in reqs]
        span = (max(r.finished for r in results) - min(arrivals)) if results else 0.0
        results.sort(key=lambda r: r.rid)
        unfinished = len(reqs) - len(results) - len(rejected) if stopped else 0
        return ServeReport(results, ticks, plans, max_batch,
                           batch_sum / ticks if ticks else 0.0, peak, span, rejected, unfinished)


def stream(count: int, rate: float = 200.0, seed: int = 0, n_min: int = 512,
           n_max: int = 32768) -> List[Request]:
    """A seeded Poisson stream of 1D requests (sizes log-uniform in [n_min, n_max])."""
    from swe_workloads import served_arrivals, served_request
    t = served_arrivals(count, rate, seed)
    return [Request(i, served_request(i, seed, n_min, n_max), float(t[i])) for i in range(count)]


def stream_mixed(count: int, rate: float = 200.0, frac_2d: float = 0.3, seed: int = 0, n_min: int = 512,
                 n_max: int = 32768) -> List[Request]:
    """A seeded Poisson stream of 1D and 2D requests: request i is 2D with probability frac_2d
    (drawn from default_rng([8, seed])), a 2D request the jump over a wedge on a grid from 64 x 32
    to 512 x 256 (swe_workloads.served_request_2d), a 1D one as in ``stream``."""
    from swe_workloads import served_arrivals, served_request, served_request_2d
    t = served_arrivals(count, rate, seed)
    is2d = np.random.default_rng([8, seed]).random(count) < frac_2d
    return [Request(i, served_request_2d(i, seed) if is2d[i] else served_request(i, seed, n_min, n_max),
                    float(t[i])) for i in range(count)]
