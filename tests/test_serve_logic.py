"""Scheduling logic of the continuous-batching server, on the CPU with a stand-in engine.

The stand-in engine converges request r after a known number of Newton steps and records what
the server asks of it, so the tests check admission by footprint, arrival order, re-planning
with carried step counts, retirement and the latency statistics without a GPU.
"""
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


def test_replanning_carries_step_counts_and_happens_on_membership_change():
    ft = FakeTime()
    eng = FakeEngine(ft, tick=1e-3)
    # request 1 arrives while request 0 is mid-solve
    reqs = _requests([(0.0, 100, 8), (0.0025, 100, 4)])
    rep = Server(eng, hbm_budget=10**9, steps_per_tick=1).run(reqs, clock=ft.clock, sleep=ft.sleep)
    # plans: {0}, {0,1} after the arrival, {0} after 1 retires
    assert rep.plans == 3
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
