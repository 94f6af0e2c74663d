"""GPU parity at the two ends of the 1D sizes the C ABI accepts, against the CPU oracle.

Smallest: N = 4 cells on one level.  The hierarchy is then the direct coarsest solve, and no
cell has the interior stencil that the Jacobian kernel's fast branch handles.  Largest:
N = 256 * 2^15 = 8388608 cells on 16 levels, whose coarsest level has the maximum 256 cells,
in one instance.  At that size the residual is compared element by element and the Jacobian
on sampled rows; the oracle differences each sampled row's columns one by one, since its
full form costs the square of the cell count.  Two V-cycles run on a seeded synthetic operator
of that size, and a Newton solve is checked through the oracle's residual of the state it
returns.  The bars are those of the other 1D parity tests: R and J within 1e-12, a V-cycle
within 1e-12 relative, Newton states within 1e-10.

The Newton solve at the largest size uses the full five-block Jacobian.  With the simplified
three-block one, Newton on this workload converges in about 20 steps up to 2^19 cells.  From
2^21 cells it ends non-finite, also with 20 V-cycles per step.  A Newton iteration built from
the separately checked residual, Jacobian and V-cycle entry points has the same residual
history as the batched step, digit for digit.  So the failure belongs to the iteration with
the simplified Jacobian at such resolutions, not to the kernels.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, Params, Problem1D, config2,  # noqa: E402
                           gaussian_bump, synthetic_operator_1d, unit_width)

DEV = "cuda:0"
N_MAX = 256 << 15


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _solver(prob, **kw):
    from paper_2505_10857_amd import Solver1D
    return Solver1D(prob, device=DEV, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _smallest():
    return Problem1D("min4", 0.0, 1.0, 4, 1, gaussian_bump(0.05, 0.5, 0.05), unit_width,
                     BC(BC_DISCHARGE, q=0.5), BC(BC_DEPTH, h=1.0), Params(eps=0.1),
                     surface0=1.0, q0=0.5)


def test_smallest_grid_residual_jacobian_vcycle_and_newton():
    prob = _smallest()
    o = oracle.Oracle1D(prob)
    s = _solver(prob)
    U0 = prob.initial_guess()
    U = s.state(U0)
    R, rn, res = s.residual(U)
    Ro, rno, reso = o.residual(U0)
    assert np.abs(R.cpu().numpy() - Ro).max() <= 1e-12 * max(np.abs(Ro).max(), 1.0)
    assert abs(float(res) - reso) <= 1e-12 * max(reso, 1.0)
    J = np.transpose(s.jacobian(U, R, rn).cpu().numpy(), (3, 0, 1, 2))
    Jo = o.jacobian(U0, nb=3)
    print(f"N=4: max|dR| {np.abs(R.cpu().numpy() - Ro).max():.2e}, max|dJ| {np.abs(J - Jo).max():.2e}")
    assert np.abs(J - Jo).max() <= 1e-12 * np.abs(Jo).max()
    # one level: each V-cycle is the direct block-tridiagonal solve
    rhs = np.random.default_rng(4).standard_normal((prob.n, 2))
    Jd = torch.tensor(np.ascontiguousarray(np.transpose(Jo, (1, 2, 3, 0))), dtype=torch.float64, device=DEV)
    rhs_d = torch.tensor(np.ascontiguousarray(rhs.T), dtype=torch.float64, device=DEV)
    dU = torch.zeros(2, prob.n, dtype=torch.float64, device=DEV)
    ref = np.zeros((prob.n, 2))
    p = prob.params
    for cyc in range(2):
        s.vcycle(Jd, rhs_d, dU, setup=(cyc == 0))
        ref = oracle.vcycles(Jo, rhs, ref, levels=1, ncycles=1, omega=p.omega, nu1=p.nu1, nu2=p.nu2)
        err = _rel(dU.cpu().numpy().T, ref)
        print(f"N=4: V-cycle {cyc + 1} rel.err {err:.3e}")
        assert err <= 1e-12
    for steps in (3, None):
        over = {"n_max": steps} if steps else {}
        s2 = _solver(prob, check_every=1, **over)
        U = s2.state(U0)
        st, _ = s2.newton_solve(U)
        Uo, ito, reso, _ = o.newton_solve(**({"n_max": steps} if steps else {}))
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(f"N=4: gpu {st.iters} steps res {st.res:.2e}; oracle {ito} res {reso:.2e}; |dU| {err:.2e}")
        assert st.iters == ito
        assert err <= 1e-10
        if steps is None:
            assert st.status == 0 and st.res < p.tol


def _largest():
    return config2(0, "sub", n=N_MAX, levels=16)


def test_largest_grid_residual_and_sampled_jacobian_rows():
    prob = _largest()
    o = oracle.Oracle1D(prob)
    s = _solver(prob)
    U0 = prob.initial_guess()
    U = s.state(U0)
    R, rn, res = s.residual(U)
    Ro, rno, reso = o.residual(U0)
    dR = np.abs(R.cpu().numpy() - Ro).max()
    print(f"N={N_MAX}: max|dR| {dR:.2e} (|R| {np.abs(Ro).max():.2e}); res {float(res):.6e} vs {reso:.6e}")
    assert dR <= 1e-12 * max(np.abs(Ro).max(), 1.0)
    assert abs(float(res) - reso) <= 1e-12 * max(reso, 1.0)
    # rows at both ends, at tile edges (256 cells) and inside, plus seeded random rows
    n = N_MAX
    rows = [0, 1, 2, 255, 256, n // 2 - 1, n // 2, n - 257, n - 3, n - 2, n - 1]
    rows += sorted(int(r) for r in np.random.default_rng(5).integers(3, n - 3, 4))
    Jg = s.jacobian(U, R, rn)
    idx = torch.tensor(rows, dtype=torch.long, device=DEV)
    J = np.transpose(Jg.index_select(3, idx).cpu().numpy(), (3, 0, 1, 2))
    del Jg
    Jo = o.jacobian_rows(U0, rows, nb=3, R=Ro, rn=rno)
    err = np.abs(J - Jo).max()
    print(f"N={N_MAX}: {len(rows)} sampled Jacobian rows, max|dJ| {err:.2e} / |J| {np.abs(Jo).max():.2e}")
    assert err <= 1e-12 * np.abs(Jo).max()


def test_largest_grid_vcycles_on_a_synthetic_operator():
    prob = _largest()
    s = _solver(prob)
    p = prob.params
    Jo, rhs = synthetic_operator_1d(N_MAX, nb=3, seed=0, dominance=1.0, spread=0.2)
    J = torch.tensor(np.ascontiguousarray(np.transpose(Jo, (1, 2, 3, 0))), dtype=torch.float64, device=DEV)
    rhs_d = torch.tensor(np.ascontiguousarray(rhs.T), dtype=torch.float64, device=DEV)
    dU = torch.zeros(2, N_MAX, dtype=torch.float64, device=DEV)
    ref = np.zeros((N_MAX, 2))
    for cyc in range(2):
        s.vcycle(J, rhs_d, dU, setup=(cyc == 0))
        ref = oracle.vcycles(Jo, rhs, ref, levels=16, ncycles=1, omega=p.omega, nu1=p.nu1, nu2=p.nu2)
        err = _rel(dU.cpu().numpy().T, ref)
        print(f"N={N_MAX}: V-cycle {cyc + 1} rel.err {err:.3e}")
        assert err <= 1e-12


def test_largest_grid_newton_solve_converges_by_the_oracles_residual():
    prob = _largest()
    s = _solver(prob, jac=5)
    U = s.state()
    st, _ = s.newton_solve(U)
    _, _, reso = oracle.Oracle1D(prob).residual(U.cpu().numpy())
    print(f"N={N_MAX}: {st.iters} Newton steps, status {st.status}, res {st.res:.3e}; "
          f"oracle's res of the returned state {reso:.3e}")
    assert st.status == 0 and st.res < prob.params.tol
    assert reso < prob.params.tol
    # the entries of R near convergence are differences of O(10) fluxes, each rounded at about
    # 1e-15, so the two sums of |R| over the same state agree to about that, absolutely
    assert abs(reso - st.res) <= 1e-13
