"""The server's 2D lane on the GPU: 2D requests (the wedge on served grids) run on their own
stream beside the 1D batch; each 2D result equals the same problem solved alone by
nmg_newton_solve bit for bit (same precision), every 1D result its solo solve, and the
stepwise 2D entry points equal the one-call solve."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_stepwise_2d_equals_the_one_call_solve():
    from paper_2505_10857_amd import _abi as A
    from paper_2505_10857_amd.solver import Solver2D, Stepper2D
    from swe_workloads import wedge_problem
    prob = wedge_problem(64, 32, seed=3)
    ref = Solver2D(prob, device=DEV, precision=A.NMG_FP32_MG, check_every=4)
    Ur = ref.state()
    st, _ = ref.newton_solve(Ur)
    side = torch.cuda.Stream(DEV)
    stp = Stepper2D(prob, device=DEV, precision=A.NMG_FP32_MG, stream=side)
    stp.begin()
    chunks = 0
    while True:
        stp.launch(3)
        stp.wait()
        chunks += 1
        act, iters, status, res = stp.state()
        if not act:
            break
    print(f"solo {st.iters} steps; stepwise {iters} steps in {chunks} chunks", flush=True)
    assert status == 0 and iters == st.iters and res == st.res
    assert torch.equal(stp.U, Ur)


def test_mixed_stream_results_equal_solo_solves():
    from paper_2505_10857_amd import _abi as A
    from paper_2505_10857_amd.serve import GpuEngine, Server, stream_mixed
    from paper_2505_10857_amd.solver import BatchSolver1D, Solver2D
    from swe_workloads import SERVED_2D_GRIDS
    reqs = stream_mixed(40, rate=400.0, frac_2d=0.3, seed=2, n_min=512, n_max=4096)
    # keep the 2D requests on the two smaller served grids for a short test
    small = {g for g in SERVED_2D_GRIDS[:2]}
    reqs = [r for r in reqs if not hasattr(r.prob, "ny") or (r.prob.nx, r.prob.ny) in small]
    n2 = sum(hasattr(r.prob, "ny") for r in reqs)
    assert n2 >= 3
    eng = GpuEngine(DEV, precision=A.NMG_FP32_MG)
    rep = Server(eng, hbm_budget=4 << 30, steps_per_tick=2, keep_states=True).run(reqs)
    eng.close()
    s = rep.summary()
    print({k: (round(v, 3) if isinstance(v, float) else v) for k, v in s.items()}, flush=True)
    assert s["completed"] == len(reqs) and s["converged"] and s["completed_2d"] == n2
    for r, q in zip(rep.results, reqs):
        if r.dim == 2:
            solo = Solver2D(q.prob, device=DEV, precision=A.NMG_FP32_MG, check_every=4)
            U = solo.state()
            st, _ = solo.newton_solve(U)
            assert st.iters == r.iters and st.status == r.status == 0
            assert torch.equal(U, r.state), f"2D request {r.rid} differs from its solo solve"
        else:
            solo = BatchSolver1D([q.prob], device=DEV, precision=A.NMG_FP32_MG)
            U = solo.states()
            (it, st1, res), = solo.solve(U, use_graph=False)
            assert it == r.iters and st1 == r.status == 0
            assert torch.equal(U[0], r.state)
