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
