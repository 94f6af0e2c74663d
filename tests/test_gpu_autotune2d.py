"""The 2D launch schedules (pass forms, streaming hints, bottom threshold) and their autotuner on
the GPU: every schedule gives the same V-cycle bit for bit, on the cross and the full stencil,
in FP64 and with FP32 multigrid, on a hierarchy with launched levels of both kinds; the
autotuner returns the fastest of its timings, and a Newton solve under it equals the default's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from swe_workloads import wedge_problem  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _operator(prob, jac):
    from paper_2505_10857_amd import Solver2D
    s = Solver2D(prob, device=DEV, jac=jac)
    rng = np.random.default_rng(3)
    U = s.state(prob.initial_guess() * (1.0 + 0.02 * rng.uniform(-1, 1, (3, prob.ny, prob.nx))))
    R, rn, _ = s.residual(U)
    return s.jacobian(U, R, rn), R


@pytest.mark.parametrize("jac", [9, 21])
@pytest.mark.parametrize("prec_name", ["fp64", "fp32mg"])
def test_every_schedule_gives_the_same_vcycle(jac, prec_name):
    from paper_2505_10857_amd import Solver2D
    from paper_2505_10857_amd import _abi as A
    prec, dt = (A.NMG_FP64, torch.float64) if prec_name == "fp64" else (A.NMG_FP32_MG, torch.float32)
    prob = wedge_problem(192, 96, levels=6)          # launched levels 192x96 .. 24x12 (and 48x24)
    J, R = _operator(prob, jac)
    ref = None
    for c in range(A.NMG_TUNE2D_CANDIDATES):
        s = Solver2D(prob, device=DEV, precision=prec, jac=jac, schedule=c, nu1=3, nu2=3)
        rhs = R.to(dt).contiguous()
        dU = torch.zeros((3, prob.ny, prob.nx), dtype=dt, device=DEV)
        s.vcycle(J, rhs, dU, setup=True)
        s.vcycle(None, rhs, dU, setup=False)
        if ref is None:
            ref = dU.clone()
        else:
            assert torch.equal(dU, ref), f"schedule {c} differs"


def test_autotune_picks_its_fastest_and_the_solve_is_unchanged():
    from paper_2505_10857_amd import Solver2D
    from paper_2505_10857_amd import _abi as A
    prob = wedge_problem(64, 32)
    J, R = _operator(prob, 9)
    s = Solver2D(prob, device=DEV, precision=A.NMG_FP32_MG)
    best, times = s.autotune(J, R.float().contiguous(), cycles=2)
    print("2D schedule times (ms per V-cycle):", {k: round(v, 3) for k, v in times.items()}, "best", best, flush=True)
    assert len(times) == A.NMG_TUNE2D_CANDIDATES and all(t > 0 for t in times.values())
    assert best == min(times, key=times.get)
    U0 = Solver2D(prob, device=DEV, precision=A.NMG_FP32_MG, check_every=4)
    Ua = U0.state()
    sa, _ = U0.newton_solve(Ua)
    sb_ = Solver2D(prob, device=DEV, precision=A.NMG_FP32_MG, check_every=4, schedule=best)
    Ub = sb_.state()
    sb, _ = sb_.newton_solve(Ub)
    assert sa.iters == sb.iters and torch.equal(Ua, Ub)
