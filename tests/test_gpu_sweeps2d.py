"""The paper's directional sweeps D1-D4 (section 4.2) as the 2D multigrid smoother on the GPU
(linear = NMG_LINEAR_MG_SWEEPS), against the oracle's lexicographic sweeps (smoother 1): V-cycles
within 1e-12 (reported bitwise: the hyperplane schedule performs the sequential sweep's operations
in its dependency order), on the cross, the five-point and the full 21-cell stencils, in the
one-workgroup bottom and on launched levels; Newton trajectories to the oracle's state."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.swe2d import Oracle2D, vcycles2d  # noqa: E402
from swe_workloads import wedge_problem  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _solver(prob, **kw):
    from paper_2505_10857_amd import Solver2D
    from paper_2505_10857_amd import _abi as A
    return Solver2D(prob, device=DEV, linear=A.NMG_LINEAR_MG_SWEEPS, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("jac", [9, 21])
@pytest.mark.parametrize("nx,ny,levels", [(16, 8, 2), (32, 16, 3), (160, 96, 6)])
def test_sweeps_vcycle_parity(nx, ny, levels, jac):
    prob = wedge_problem(nx, ny, levels=levels)
    o = Oracle2D(prob)
    rng = np.random.default_rng([5, nx])
    U0 = prob.initial_guess() * (1.0 + 0.02 * rng.uniform(-1.0, 1.0, (3, ny, nx)))
    R, rn, _ = o.residual(U0)
    Jo = o.jacobian(U0, R=R, rn=rn, which=jac)
    p = prob.params
    s = _solver(prob, levels=levels, nu1=2, nu2=2, jac=jac)
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(R, dtype=torch.float64, device=DEV)
    dU = torch.zeros((3, ny, nx), dtype=torch.float64, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    rhs_o = np.ascontiguousarray(R.transpose(1, 2, 0))
    d1 = vcycles2d(Jo, rhs_o, levels=levels, ncycles=1, omega=p.omega, nu1=2, nu2=2, smoother=1)
    g1 = dU.cpu().numpy().transpose(1, 2, 0)
    s.vcycle(None, rhs, dU, setup=False)
    d2 = vcycles2d(Jo, rhs_o, levels=levels, ncycles=2, omega=p.omega, nu1=2, nu2=2, smoother=1)
    e1, e2 = _rel(g1, d1), _rel(dU.cpu().numpy().transpose(1, 2, 0), d2)
    print(f"{nx}x{ny} J{jac} levels={levels}: sweeps V-cycle rel err {e1:.2e}, {e2:.2e} "
          f"(bitwise {np.array_equal(g1, d1)})", flush=True)
    assert e1 <= 1e-12 and e2 <= 1e-12


@pytest.mark.parametrize("jac", [9, 21])
def test_sweeps_newton_matches_the_oracle(jac):
    """The wedge, 32 x 16, NMGM with the directional sweeps to res < 1e-10: the oracle's step
    count (within one) and state (within 1e-10); five-step res histories within 1e-10."""
    prob = wedge_problem(32, 16)
    s = _solver(prob, check_every=4, jac=jac)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, it, reso, _ = Oracle2D(prob).newton_solve(which=jac, smoother=1)
    e = _rel(U.cpu().numpy(), Uo)
    print(f"J{jac}: GPU {st.iters} steps res {st.res:.2e}; oracle {it}; rel err {e:.2e}", flush=True)
    assert st.status == 0 and abs(st.iters - it) <= 1
    assert e <= 1e-10
    s5 = _solver(prob, check_every=1, n_max=5, jac=jac)
    U5 = s5.state()
    _, h = s5.newton_solve(U5, max_hist=5)
    _, _, _, ho = Oracle2D(prob).newton_solve(which=jac, smoother=1, n_max=5)
    assert np.all(np.abs(h - ho) <= 1e-10 * np.abs(ho))
