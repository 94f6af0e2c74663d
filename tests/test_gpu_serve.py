"""The continuous-batching server on the GPU: requests that arrive while others are iterating
are admitted as memory frees up, share every launch with them, and each result equals the same
problem solved alone, bit for bit, and the FP64 oracle's solution within the parity bar."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.mark.parametrize("prec_name", ["fp64", "fp32mg"])
def test_served_results_equal_solo_solves(prec_name):
    from paper_2505_10857_amd import _abi as A
    from paper_2505_10857_amd.serve import GpuEngine, Server, stream
    from paper_2505_10857_amd.solver import BatchSolver1D
    prec = A.NMG_FP64 if prec_name == "fp64" else A.NMG_FP32_MG
    import dataclasses
    # requests iterated to the round-off floor (res < 1e-13), where the parity bars are defined
    reqs = [dataclasses.replace(r, prob=dataclasses.replace(r.prob, params=dataclasses.replace(
                r.prob.params, tol=1e-13, n_max=5000)))
            for r in stream(12, rate=3000.0, seed=1, n_min=512, n_max=4096)]
    eng = GpuEngine(DEV, precision=prec)
    fps = [eng.footprint(r.prob) for r in reqs]
    budget = sum(fps) // 2                      # admission has to wait for retirements
    rep = Server(eng, hbm_budget=budget, steps_per_tick=2, keep_states=True).run(reqs)
    eng.close()
    s = rep.summary()
    print(prec_name, {k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()})
    assert s["completed"] == 12 and s["converged"]
    assert 1 < rep.max_batch < 12 and rep.plans > 2
    assert rep.peak_bytes <= budget
    for r, q in zip(rep.results, reqs):
        solo = BatchSolver1D([q.prob], device=DEV, precision=prec)
        U = solo.states()
        (it, st, res), = solo.solve(U, use_graph=False)
        assert it == r.iters and st == r.status == 0
        assert torch.equal(U[0], r.state), f"request {r.rid}: served state differs from solo"
    # every request (512 to 4096 cells) against the FP64 oracle's solution of the same problem,
    # both at the round-off floor
    from concurrent.futures import ThreadPoolExecutor
    bar = 1e-10 if prec == A.NMG_FP64 else 1e-9
    oracle.lib()
    with ThreadPoolExecutor(max_workers=12) as ex:
        ref = list(ex.map(lambda r: oracle.Oracle1D(reqs[r.rid].prob).newton_solve(), rep.results))
    assert all(x[2] < 1e-13 for x in ref)
    for r, (Uo, ito, reso, _) in zip(rep.results, ref):
        err = np.abs(r.state.cpu().numpy() - Uo).max()
        print(f"request {r.rid} (N={r.n}): |U - U_oracle| = {err:.2e}, steps {r.iters} vs {ito}")
        assert err <= bar


def test_a_request_that_breaks_down_is_retried_and_matches_the_oracle():
    """A served channel (N = 2432, strongly varying width) whose V-cycle diverges at the SOR
    weight 0.8: the GPU and the oracle both break down at Newton step 6; the server retries it
    at 0.6 and the result equals the oracle's solution at 0.6 (FP64, within 1e-10)."""
    import dataclasses
    from paper_2505_10857_amd import _abi as A
    from paper_2505_10857_amd.serve import GpuEngine, Request, Server
    from swe_workloads import served_request

    def floor(p):                                  # iterated to the round-off floor (res < 1e-13)
        return dataclasses.replace(p, params=dataclasses.replace(p.params, tol=1e-13, n_max=5000))

    bad, ok = floor(served_request(398, 5)), floor(served_request(3, 5))
    _, it_bad, res_bad, _ = oracle.Oracle1D(bad).newton_solve()
    assert not np.isfinite(res_bad)
    eng = GpuEngine(DEV, precision=A.NMG_FP64)
    reqs = [Request(0, bad, 0.0), Request(1, ok, 0.0)]
    rep = Server(eng, hbm_budget=1 << 32, steps_per_tick=2, keep_states=True).run(reqs)
    r0, r1 = rep.results
    print(f"retried: status {r0.status}, {r0.iters} steps, res {r0.res:.2e}; oracle broke down at {it_bad}")
    assert (r0.status, r0.retries) == (0, 1) and (r1.status, r1.retries) == (0, 0)
    again = dataclasses.replace(bad, params=dataclasses.replace(bad.params, omega=0.6))
    Uo, ito, reso, _ = oracle.Oracle1D(again).newton_solve()
    assert abs(r0.iters - ito) <= 1
    assert np.abs(r0.state.cpu().numpy() - Uo).max() <= 1e-10
    off = Server(eng, hbm_budget=1 << 32, steps_per_tick=2, retry_omega=None).run([Request(0, bad, 0.0)])
    assert off.results[0].status == A.NMG_ENONFINITE and off.results[0].iters == it_bad
    eng.close()
