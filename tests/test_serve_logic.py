"""Scheduling logic of the continuous-batching server, on the CPU with a stand-in engine.

The stand-in engine converges request r after a known number of Newton steps and records what
the server asks of it, so the tests check admission by footprint, arrival order, re-planning
with carried step counts, retirement and the latency statistics without a GPU.
"""
import dataclasses

import numpy as np
import pytest

from paper_2505_10857_amd.serve import Request, Server


class FakeTime:
    def __init__(self):
        self.t = 0.0

    def clock(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 0.0)


class FakeProb:
    def __init__(self, n, need):
        self.n = n
        self.need = need


class FakeBatch:
    def __init__(self, eng, items):
        self.eng = eng
        self.items = items
        self.done = None

    def resume(self, n_done):
        self.eng.resumes.append([(it["rid"], d) for it, d in zip(self.items, n_done)])
        for it, d in zip(self.items, n_done):
            assert it["steps"] == d, "a resumed request must carry its own step count"
        self.done = list(n_done)

    def steps(self, k):
        self.eng.time.t += self.eng.tick
        flags, stats = [], []
        for i, it in enumerate(self.items):
            take = min(k, it["need"] - it["steps"])
            it["steps"] += take
            flags.append(1 if it["steps"] < it["need"] else 0)
            stats.append((it["steps"], 0, 1e-11))
        self.eng.batches.append(len(self.items))
        return flags, stats


class FakeEngine:
    def __init__(self, time, tick=1e-3):
        self.time = time
        self.tick = tick
        self.resumes = []
        self.batches = []
        self.in_use = 0
        self.max_in_use = 0

    def footprint(self, prob):
        return prob.n * 10

    def prepare(self, prob):
        return dict(rid=prob.rid, need=prob.need, steps=0)

    def batch(self, prepared):
        return FakeBatch(self, list(prepared))

    def state(self, prep):
        return prep["steps"]


def _requests(spec):
    out = []
    for rid, (t, n, need) in enumerate(spec):
        p = FakeProb(n, need)
        p.rid = rid
        out.append(Request(rid, p, t))
    return out


def test_every_request_completes_with_its_own_step_count():
    ft = FakeTime()
    eng = FakeEngine(ft)
    reqs = _requests([(0.0, 100, 5), (0.0005, 200, 9), (0.0021, 50, 3), (0.02, 80, 4)])
    rep = Server(eng, hbm_budget=10**9, steps_per_tick=2, keep_states=True).run(
        reqs, clock=ft.clock, sleep=ft.sleep)
    assert [r.rid for r in rep.results] == [0, 1, 2, 3]
    assert [r.iters for r in rep.results] == [5, 9, 3, 4]
    assert [r.state for r in rep.results] == [5, 9, 3, 4]
    assert all(r.finished >= r.admitted >= r.arrival for r in rep.results)
    assert rep.rejected == []


def test_admission_respects_the_budget_and_arrival_order():
    ft = FakeTime()
    eng = FakeEngine(ft)
    # footprints 1000 each, budget 2500: at most two at a time
    reqs = _requests([(0.0, 100, 6)] * 6)
    rep = Server(eng, hbm_budget=2500, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    assert rep.max_batch == 2 and max(eng.batches) == 2
    assert rep.peak_bytes <= 2500
    adm = [r.admitted for r in rep.results]
    assert adm == sorted(adm)                  # FIFO admission
    assert len(rep.results) == 6


def test_oversized_request_is_rejected_not_blocking():
    ft = FakeTime()
    eng = FakeEngine(ft)
    reqs = _requests([(0.0, 10**6, 3), (0.0, 10, 3)])
    rep = Server(eng, hbm_budget=10**5).run(reqs, clock=ft.clock, sleep=ft.sleep)
    assert rep.rejected == [0]
    assert [r.rid for r in rep.results] == [1]


def test_replanning_carries_step_counts_and_happens_when_requests_join():
    ft = FakeTime()
    eng = FakeEngine(ft, tick=1e-3)
    # request 1 arrives while request 0 is mid-solve
    reqs = _requests([(0.0, 100, 8), (0.0025, 100, 4)])
    rep = Server(eng, hbm_budget=10**9, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    # plans: {0}, {0,1} after the arrival; request 1 retires inside that plan (its slot skipped,
    # half the slots still live), and the plan is released once 0 retires too
    assert rep.plans == 2
    assert eng.resumes[0] == [(0, 0)]
    r0_steps_at_join = dict(eng.resumes[1])[0]
    assert r0_steps_at_join > 0 and dict(eng.resumes[1])[1] == 0
    assert [r.iters for r in rep.results] == [8, 4]


def test_idle_server_waits_for_the_next_arrival():
    ft = FakeTime()
    eng = FakeEngine(ft)
    reqs = _requests([(5.0, 100, 2)])
    rep = Server(eng, hbm_budget=10**9).run(reqs, clock=ft.clock, sleep=ft.sleep)
    assert rep.results[0].admitted >= 5.0
    assert rep.results[0].latency == pytest.approx(eng.tick)


def test_latency_percentiles():
    ft = FakeTime()
    eng = FakeEngine(ft, tick=1e-3)
    reqs = _requests([(0.0, 10, k) for k in range(1, 11)])
    rep = Server(eng, hbm_budget=10**9, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    lat = np.array([r.latency for r in rep.results]) * 1e3
    assert np.allclose(sorted(lat), np.arange(1, 11))
    assert rep.latency_ms(50) == pytest.approx(np.percentile(lat, 50))
    assert rep.latency_ms(99) == pytest.approx(np.percentile(lat, 99))
    s = rep.summary()
    assert s["completed"] == 10 and s["converged"]


def test_retired_slots_are_reclaimed_when_the_next_request_needs_their_memory():
    """Budget for two requests: the third waits; when the first retires, its slot's memory is
    held by the plan until the third needs it, then the plan is rebuilt without it."""
    ft = FakeTime()
    eng = FakeEngine(ft)
    reqs = _requests([(0.0, 100, 2), (0.0, 100, 9), (0.0, 100, 3)])
    rep = Server(eng, hbm_budget=2000, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    assert [r.iters for r in rep.results] == [2, 9, 3]
    assert rep.peak_bytes <= 2000 and rep.max_batch == 2
    assert rep.plans == 2                      # {0, 1}, then {1, 2} after the reclaim
    assert eng.resumes[1] == [(1, 2), (2, 0)]  # request 1 carries its two steps
    assert rep.results[2].admitted >= rep.results[0].finished


def test_most_slots_retired_triggers_a_rebuild():
    ft = FakeTime()
    eng = FakeEngine(ft)
    reqs = _requests([(0.0, 10, 1), (0.0, 10, 1), (0.0, 10, 1), (0.0, 10, 8)])
    rep = Server(eng, hbm_budget=10**9, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    # three of four retire after one step: the plan is rebuilt over the survivor
    assert rep.plans == 2 and eng.batches[-1] == 1
    assert [r.iters for r in rep.results] == [1, 1, 1, 8]


class FakeProb2D:
    def __init__(self, nx, ny, need):
        self.nx, self.ny, self.need = nx, ny, need


class FakeStepper:
    def __init__(self, eng, prob):
        self.eng, self.need, self.steps, self.ready_at, self.chunks = eng, prob.need, 0, None, 0


class FakeEngine2D(FakeEngine):
    """1D as FakeEngine; a 2D request needs `need` Newton steps, taken `k` per chunk, each chunk
    ready `chunk_time` seconds after it is enqueued."""

    def __init__(self, time, tick=1e-3, k=4, chunk_time=5e-3):
        super().__init__(time, tick)
        self.k, self.chunk_time = k, chunk_time
        self.started = []

    def is2d(self, prob):
        return hasattr(prob, "ny")

    def footprint(self, prob):
        return prob.nx * prob.ny * 10 if self.is2d(prob) else prob.n * 10

    def prepare2d(self, prob):
        return FakeStepper(self, prob)

    def _launch(self, st):
        st.ready_at = self.time.t + self.chunk_time
        st.chunks += 1

    def start2d(self, st):
        self.started.append(self.time.t)
        self._launch(st)

    def poll2d(self, st):
        if self.time.t < st.ready_at:
            return None
        st.steps = min(st.need, st.chunks * self.k)
        act = st.steps < st.need
        if act:
            self._launch(st)
        return (1 if act else 0), st.steps, 0, 1e-11

    def state2d(self, st):
        return ("2d", st.steps)


def test_2d_requests_run_beside_the_1d_batch():
    """A stream of 1D and 2D requests: every request completes with its own step count; a 2D
    request's chunks are polled while 1D ticks go on, and only-2D periods do not spin forever."""
    ft = FakeTime()
    eng = FakeEngine2D(ft, tick=1e-3, k=4, chunk_time=5e-3)
    reqs = []
    for rid, (t, kind, size, need) in enumerate([(0.0, 1, 100, 6), (0.0, 2, (8, 4), 10),
                                                  (0.002, 1, 50, 3), (0.004, 2, (16, 8), 5),
                                                  (0.05, 2, (8, 4), 3)]):
        p = FakeProb(size, need) if kind == 1 else FakeProb2D(size[0], size[1], need)
        p.rid = rid
        reqs.append(Request(rid, p, t))
    rep = Server(eng, hbm_budget=10**9, steps_per_tick=1, keep_states=True).run(
        reqs, clock=ft.clock, sleep=ft.sleep)
    assert [r.iters for r in rep.results] == [6, 10, 3, 5, 3]
    assert [r.dim for r in rep.results] == [1, 2, 1, 2, 1 + 1]
    assert rep.results[1].state == ("2d", 10) and rep.results[1].n == 32
    # the 10-step 2D request needs three chunks of four: done no earlier than 3 chunk times
    assert rep.results[1].finished >= 3 * 5e-3 - 1e-12
    s = rep.summary()
    assert s["completed_2d"] == 3 and s["completed_1d"] == 2 and s["converged"]


def _req(rid, p, t):
    p.rid = rid
    return Request(rid, p, t)


def test_a_waiting_2d_request_does_not_hold_up_1d_requests():
    """Budget 500: a 1D request (footprint 300) is running when a 2D request (footprint 320) and
    then a small 1D request (footprint 100) arrive.  The 2D request waits for memory; the 1D
    request behind it is admitted at once, and the 2D request once the first 1D request ends."""
    ft = FakeTime()
    eng = FakeEngine2D(ft, tick=1e-3, k=4, chunk_time=5e-3)
    reqs = [_req(0, FakeProb(30, 20), 0.0), _req(1, FakeProb2D(8, 4, 4), 0.001), _req(2, FakeProb(10, 2), 0.002)]
    rep = Server(eng, hbm_budget=500, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    r0, r1, r2 = rep.results
    assert r2.admitted < r0.finished                 # the small 1D request did not wait
    assert r1.admitted >= r0.finished - 1e-12        # the 2D request waited for memory
    assert rep.peak_bytes <= 500 and rep.summary()["converged"]


def test_2d_requests_beyond_the_workers_wait_without_memory():
    """With two 2D workers, a third 2D request is admitted (its memory reserved) only when one
    of the first two is done."""
    ft = FakeTime()
    eng = FakeEngine2D(ft, tick=1e-3, k=4, chunk_time=5e-3)
    eng.workers_2d = 2
    reqs = [_req(i, FakeProb2D(8, 4, 8), 0.0) for i in range(3)]
    rep = Server(eng, hbm_budget=10**6, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    r = rep.results
    assert r[2].admitted >= min(r[0].finished, r[1].finished) - 1e-12
    assert rep.peak_bytes == 2 * 8 * 4 * 10


def test_stop_after_counts_unfinished_requests():
    """A stream longer than the run: requests not completed when it is stopped are reported as
    unfinished, not dropped silently."""
    ft = FakeTime()
    eng = FakeEngine2D(ft, tick=1e-3, k=4, chunk_time=5e-3)
    reqs = [_req(i, FakeProb(10, 5), 0.01 * i) for i in range(20)]
    rep = Server(eng, hbm_budget=10**6, steps_per_tick=1).run(
        reqs, clock=ft.clock, sleep=ft.sleep, stop_after=0.1)
    s = rep.summary()
    assert s["unfinished"] == 20 - s["completed"] > 0
    assert all(r.finished <= 0.1 + 1e-2 for r in rep.results)


@dataclasses.dataclass
class _W:
    omega: float


@dataclasses.dataclass
class BreakingProb:
    """A 1D stand-in whose iteration breaks down at an SOR weight above 0.7 after `fail_at` steps
    and converges after `need` steps otherwise."""
    n: int
    need: int
    fail_at: int
    params: _W
    rid: int = 0


class FakeEngineBreak(FakeEngine2D):
    def prepare(self, prob):
        d = dict(rid=prob.rid, need=prob.need, steps=0)
        if getattr(prob, "params", None) is not None and prob.params.omega > 0.7:
            d["need"] = prob.fail_at
            d["breaks"] = True
        return d

    def batch(self, prepared):
        return FakeBatchBreak(self, list(prepared))


class FakeBatchBreak(FakeBatch):
    def steps(self, k):
        flags, stats = super().steps(k)
        return flags, [(it, -4 if item.get("breaks") and not f else st, res)
                       for (it, st, res), f, item in zip(stats, flags, self.items)]


def test_a_broken_down_request_is_retried_once_at_the_smaller_weight():
    ft = FakeTime()
    eng = FakeEngineBreak(ft)
    reqs = [_req(0, BreakingProb(10, 7, 3, _W(0.8)), 0.0), _req(1, FakeProb(10, 4), 0.0),
            _req(2, BreakingProb(10, 5, 2, _W(0.6)), 0.0)]
    rep = Server(eng, hbm_budget=10**6, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    r0, r1, r2 = rep.results
    assert (r0.status, r0.iters, r0.retries) == (0, 7, 1)     # retried at 0.6, then converged
    assert (r1.status, r1.retries) == (0, 0)
    assert (r2.status, r2.iters, r2.retries) == (0, 5, 0)     # already at 0.6: never broke
    s = rep.summary()
    assert s["retried"] == 1 and s["converged"]
    off = Server(eng, hbm_budget=10**6, steps_per_tick=1, retry_omega=None).run(
        [_req(0, BreakingProb(10, 7, 3, _W(0.8)), ft.t)], clock=ft.clock, sleep=ft.sleep)
    assert off.results[0].status == -4 and off.results[0].retries == 0


def test_2d_lanes_are_capped_while_1d_requests_run():
    """Three 2D workers and lanes_2d_busy = 1: while a 1D request iterates only one 2D solve runs
    at a time; once it is done, up to three run together.  Without the cap all three start."""
    ft = FakeTime()
    eng = FakeEngine2D(ft, tick=1e-3, k=4, chunk_time=5e-3)
    eng.workers_2d = 3
    reqs = [_req(0, FakeProb(10, 12), 0.0)] + [_req(i, FakeProb2D(8, 4, 4), 0.0) for i in range(1, 7)]
    rep = Server(eng, hbm_budget=10**6, steps_per_tick=1, lanes_2d_busy=1).run(
        reqs, clock=ft.clock, sleep=ft.sleep)
    r = rep.results
    t1d = r[0].finished

    def running(t):
        return sum(1 for x in r[1:] if x.admitted <= t < x.finished)

    assert max(running(x.admitted) for x in r[1:] if x.admitted < t1d) == 1
    assert max(running(x.admitted) for x in r[1:]) == 3
    many = Server(eng, hbm_budget=10**6, steps_per_tick=1).run(
        [_req(0, FakeProb(10, 30), ft.t)] + [_req(i, FakeProb2D(8, 4, 4), ft.t) for i in range(1, 4)],
        clock=ft.clock, sleep=ft.sleep)
    assert len({round(x.admitted, 9) for x in many.results}) == 1
