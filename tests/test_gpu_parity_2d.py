"""GPU parity of the 2D hot path against the CPU oracle, through the C ABI.

Bar (FP64): residual and J9 within 1e-12 relative (the arithmetic is written to be
bit-identical, which these tests report), V-cycles within 1e-12 relative, Newton trajectories and
converged states within 1e-10.  FP32 multigrid: converged state within 1e-9 of the FP64 oracle's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.swe2d import Oracle2D, vcycles2d  # noqa: E402
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, BC_WALL, Params, Problem2D,  # noqa: E402
                           parabolic_bump_2d, wedge_problem)

DEV = "cuda:0"

@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _solver(prob, **kw):
    from paper_2505_10857_amd import Solver2D
    return Solver2D(prob, device=DEV, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _noisy(prob, seed, amp=0.02):
    """Initial guess with seeded relative noise on every component (a generic state)."""
    rng = np.random.default_rng([11, seed])
    U = prob.initial_guess()
    return U * (1.0 + amp * rng.uniform(-1.0, 1.0, U.shape))


def _ragged_channel(nx=56, ny=24):
    """Sub-critical channel with walls on both sides and a Gaussian mound: the DISCHARGE and
    DEPTH sides of the 2D boundary set; 56 x 24 spans partial residual tiles in x and y."""
    def bottom(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        e = 0.1 * np.exp(-((x - 2.0) ** 2 + (y - 1.0) ** 2))
        return e, -2.0 * (x - 2.0) * e, -2.0 * (y - 1.0) * e
    return Problem2D("ragged", 0.0, 4.0, 0.0, 2.0, nx, ny, 4, bottom,
                     [BC(BC_DISCHARGE, q=0.8), BC(BC_DEPTH, h=1.0), BC(BC_WALL), BC(BC_WALL)],
                     Params(eps=1e-6, omega=0.1, nu1=4, nu2=4, nu3=2), init_state=(1.0, 0.8, 0.0))


def _closed_basin(nx=40, ny=24):
    """Walls on all four sides over a Gaussian mound, flow along both axes: every face of the
    grid's border takes the wall ghosts; 40 x 24 spans partial residual tiles."""
    def bottom(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        e = 0.1 * np.exp(-((x - 1.3) ** 2 + (y - 0.9) ** 2))
        return e, -2.0 * (x - 1.3) * e, -2.0 * (y - 0.9) * e
    return Problem2D("basin", 0.0, 3.0, 0.0, 2.0, nx, ny, 4, bottom, [BC(BC_WALL)] * 4,
                     Params(eps=1e-6, omega=0.1, nu1=4, nu2=4, nu3=2), init_state=(1.0, 0.2, -0.1))


def _cases():
    yield "wedge32x16", wedge_problem(32, 16)
    yield "wedge64x32", wedge_problem(64, 32, seed=3)
    yield "bump16x8", parabolic_bump_2d(16, 8)
    yield "ragged56x24", _ragged_channel()
    yield "basin40x24", _closed_basin()


CASES = list(_cases())
IDS = [c[0] for c in CASES]


@pytest.mark.parametrize("name,prob", CASES, ids=IDS)
def test_residual_parity(name, prob):
    s = _solver(prob)
    o = Oracle2D(prob)
    for U0 in (prob.initial_guess(), _noisy(prob, 1)):
        U = s.state(U0)
        R, rn, res = s.residual(U)
        Ro, rno, reso = o.residual(U0)
        Rg = R.cpu().numpy()
        scale = max(np.abs(Ro).max(), 1.0)
        err = np.abs(Rg - Ro).max()
        print(f"{name}: residual max|dR| = {err:.3e} (bitwise equal: {np.array_equal(Rg, Ro)})")
        assert err <= 1e-12 * scale
        assert np.abs(rn.cpu().numpy() - rno).max() <= 1e-12 * scale
        assert abs(res.item() - reso) <= 1e-12 * max(reso, 1e-300)


@pytest.mark.parametrize("name,prob", CASES, ids=IDS)
def test_jacobian_parity(name, prob):
    s = _solver(prob)
    o = Oracle2D(prob)
    U0 = _noisy(prob, 2)
    U = s.state(U0)
    R, rn, _ = s.residual(U)
    J = s.jacobian(U, R, rn).cpu().numpy()              # [9, 3, 3, ny, nx]
    Jo = o.jacobian(U0)                                  # [ny, nx, 9, 3, 3]
    Jo_t = np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1))
    err = np.abs(J - Jo_t).max()
    print(f"{name}: J9 max|dJ| = {err:.3e} (bitwise equal: {np.array_equal(J, Jo_t)})")
    assert err <= 1e-12 * np.abs(Jo).max()


def _operator(prob, seed=4):
    o = Oracle2D(prob)
    U0 = _noisy(prob, seed)
    R, rn, _ = o.residual(U0)
    Jo = o.jacobian(U0, R=R, rn=rn)
    return Jo, R


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_vcycle_parity(levels):
    """One and two V-cycles (Algorithm 2) from dU = 0 on an oracle operator; levels = 1 is the
    dense coarsest solve applied to the nine-block operator itself."""
    prob = wedge_problem(8 << (levels - 1), 4 << (levels - 1))
    Jo, R = _operator(prob)
    p = prob.params
    s = _solver(prob, levels=levels, nu1=3, nu2=3)
    ny, nx = prob.ny, prob.nx
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(R, dtype=torch.float64, device=DEV)               # [3, ny, nx]
    dU = torch.zeros((3, ny, nx), dtype=torch.float64, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    rhs_o = np.ascontiguousarray(R.transpose(1, 2, 0))                    # [ny, nx, 3]
    d1 = vcycles2d(Jo, rhs_o, levels=levels, ncycles=1, omega=p.omega, nu1=3, nu2=3)
    g1 = dU.cpu().numpy().transpose(1, 2, 0)
    e1 = _rel(g1, d1)
    s.vcycle(None, rhs, dU, setup=False)
    d2 = vcycles2d(Jo, rhs_o, levels=levels, ncycles=2, omega=p.omega, nu1=3, nu2=3)
    e2 = _rel(dU.cpu().numpy().transpose(1, 2, 0), d2)
    print(f"levels={levels}: V-cycle rel err {e1:.3e}, {e2:.3e} (bitwise: {np.array_equal(g1, d1)})")
    assert e1 <= 1e-12 and e2 <= 1e-12


def test_vcycle_ragged_hierarchy():
    """56 x 24 with four levels (7 x 3 coarsest): every level has a partial workgroup."""
    prob = _ragged_channel()
    Jo, R = _operator(prob, seed=5)
    s = _solver(prob)
    p = prob.params
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(R, dtype=torch.float64, device=DEV)
    dU = torch.zeros((3, prob.ny, prob.nx), dtype=torch.float64, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    d1 = vcycles2d(Jo, np.ascontiguousarray(R.transpose(1, 2, 0)), levels=prob.levels, ncycles=1,
                   omega=p.omega, nu1=p.nu1, nu2=p.nu2)
    e = _rel(dU.cpu().numpy().transpose(1, 2, 0), d1)
    print(f"ragged V-cycle rel err {e:.3e}")
    assert e <= 1e-12


def test_vcycle_fp32_mg_tracks_fp64():
    """FP32 operator, right-hand side and correction (aF1): two V-cycles stay within single-
    precision rounding (1e-4 relative) of the FP64 oracle's."""
    from paper_2505_10857_amd import _abi as A
    prob = wedge_problem(32, 16)
    Jo, R = _operator(prob, seed=6)
    p = prob.params
    s = _solver(prob, precision=A.NMG_FP32_MG)
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(R, dtype=torch.float32, device=DEV)
    dU = torch.zeros((3, prob.ny, prob.nx), dtype=torch.float32, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    s.vcycle(None, rhs, dU, setup=False)
    d2 = vcycles2d(Jo, np.ascontiguousarray(R.transpose(1, 2, 0)), levels=prob.levels, ncycles=2,
                   omega=p.omega, nu1=p.nu1, nu2=p.nu2)
    e = _rel(dU.double().cpu().numpy().transpose(1, 2, 0), d2)
    print(f"FP32-MG V-cycles rel err {e:.3e}")
    assert e <= 1e-4


@pytest.mark.parametrize("name,prob", [CASES[0], CASES[3]], ids=[IDS[0], IDS[3]])
def test_newton_trajectory(name, prob):
    """Five Newton steps (Algorithm 1): state and res history within 1e-10."""
    s = _solver(prob, n_max=5, check_every=1)
    o = Oracle2D(prob)
    U = s.state()
    st, hist = s.newton_solve(U, max_hist=5)
    Uo, it, reso, hist_o = o.newton_solve(n_max=5)
    e = _rel(U.cpu().numpy(), Uo)
    print(f"{name}: 5 steps, state rel err {e:.3e}; res {hist} vs {hist_o}")
    assert st.iters == it == 5
    assert e <= 1e-10
    assert np.all(np.abs(hist - hist_o) <= 1e-10 * np.maximum(np.abs(hist_o), 1e-300) + 1e-14)


def test_newton_converges_like_oracle_wedge():
    """Jump over a wedge, 32 x 16, to res < 1e-10: same step count (+-1), state within 1e-10."""
    prob = wedge_problem(32, 16)
    s = _solver(prob, check_every=4)
    o = Oracle2D(prob)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, it, reso, _ = o.newton_solve()
    e = _rel(U.cpu().numpy(), Uo)
    print(f"GPU {st.iters} steps res {st.res:.3e}; oracle {it} steps res {reso:.3e}; rel err {e:.3e}")
    assert st.status == 0 and st.res < prob.params.tol
    assert abs(st.iters - it) <= 1
    assert e <= 1e-10


def test_fp32_mg_converges_to_fp64_solution():
    """FP32 Jacobian and multigrid, FP64 residual/update/test: converged state within 1e-9."""
    from paper_2505_10857_amd import _abi as A
    prob = wedge_problem(32, 16)
    s = _solver(prob, precision=A.NMG_FP32_MG, check_every=4)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, it, reso, _ = Oracle2D(prob).newton_solve()
    e = _rel(U.cpu().numpy(), Uo)
    print(f"FP32-MG: {st.iters} steps (oracle FP64 {it}), res {st.res:.3e}, rel err {e:.3e}")
    assert st.status == 0 and st.res < prob.params.tol
    assert e <= 1e-9


def test_full_size_sampled_rows():
    """1024 x 512 wedge at a generic state: the whole residual against the oracle's, and J9 rows
    of sampled grid lines (first, last, interior) against the oracle's rows."""
    prob = wedge_problem(1024, 512, seed=7)
    s = _solver(prob)
    o = Oracle2D(prob)
    U0 = _noisy(prob, 9, amp=0.01)
    U = s.state(U0)
    R, rn, res = s.residual(U)
    Ro, rno, reso = o.residual(U0)
    assert _rel(R.cpu().numpy(), Ro) <= 1e-12
    assert abs(res.item() - reso) <= 1e-12 * reso
    J = s.jacobian(U, R, rn)
    for j0 in (0, 1, 255, 510, 511):
        Jo = o.jacobian(U0, rows=(j0, j0 + 1), R=Ro, rn=rno)
        Jg = J[:, :, :, j0, :].cpu().numpy()
        Jt = np.ascontiguousarray(Jo[j0].transpose(1, 2, 3, 0))
        assert np.abs(Jg - Jt).max() <= 1e-12 * np.abs(Jt).max(), j0


def test_full_size_newton_step_reduces_res():
    """1024 x 512 wedge, the launch configuration of the benchmark: three Newton steps in FP64
    and in FP32-MG lower res below its value at the uniform inflow guess and stay finite."""
    from paper_2505_10857_amd import _abi as A
    prob = wedge_problem(1024, 512)
    for prec in (A.NMG_FP64, A.NMG_FP32_MG):
        s = _solver(prob, precision=prec, n_max=3, check_every=1)
        U = s.state()
        st, hist = s.newton_solve(U, max_hist=3)
        R0 = Oracle2D(prob).residual(prob.initial_guess())[2]
        print(f"prec {prec}: res0 {R0:.3e} -> {hist}")
        assert st.iters == 3 and np.all(np.isfinite(hist))
        assert hist[2] < R0
        assert torch.isfinite(U).all()


def test_rejects_bad_2d_descriptors():
    from paper_2505_10857_amd import _abi as A
    prob = wedge_problem(32, 16)
    with pytest.raises(A.NmgError):
        _solver(prob, levels=2).workspace()            # coarsest 16 x 8 > 40 cells
    with pytest.raises(A.NmgError):
        _solver(prob, levels=7).workspace()            # 32 not divisible by 64


def test_full_size_vcycle_on_the_wedge_grid():
    """1024 x 512, 8 levels, nu = 20, omega = 0.05 (the wedge's launch configuration): one
    V-cycle on a seeded J9-shaped operator equals the oracle's."""
    from swe_workloads import synthetic_operator_2d
    prob = wedge_problem(1024, 512)
    Jo, rhs_o = synthetic_operator_2d(1024, 512, seed=1)
    p = prob.params
    s = _solver(prob)
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(np.ascontiguousarray(rhs_o.transpose(2, 0, 1)), dtype=torch.float64, device=DEV)
    dU = torch.zeros((3, 512, 1024), dtype=torch.float64, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    d1 = vcycles2d(Jo, rhs_o, levels=prob.levels, ncycles=1, omega=p.omega, nu1=p.nu1, nu2=p.nu2)
    e = _rel(dU.cpu().numpy().transpose(1, 2, 0), d1)
    print(f"1024x512 V-cycle rel err {e:.3e}")
    assert e <= 1e-12


def test_repeated_vcycles_match_oracle():
    """Four V-cycle calls in a row on one workspace, with other device work and host
    synchronisation between them, each equal to the oracle's k-th V-cycle; then the same on a
    fresh workspace."""
    prob = wedge_problem(32, 16)
    Jo, R = _operator(prob, seed=9)
    p = prob.params
    rhs_o = np.ascontiguousarray(R.transpose(1, 2, 0))
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(R, dtype=torch.float64, device=DEV)
    for trial in range(2):
        s = _solver(prob, nu1=2, nu2=2)
        dU = torch.zeros((3, prob.ny, prob.nx), dtype=torch.float64, device=DEV)
        for k in range(1, 5):
            s.vcycle(J if k == 1 else None, rhs, dU, setup=(k == 1))
            junk = (dU * 2.0).sum()                        # other work on the stream in between
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            dk = vcycles2d(Jo, rhs_o, levels=prob.levels, ncycles=k, omega=p.omega, nu1=2, nu2=2)
            e = _rel(dU.cpu().numpy().transpose(1, 2, 0), dk)
            print(f"workspace {trial}, V-cycle {k}: rel err {e:.3e}")
            assert e <= 1e-12


@pytest.mark.parametrize("prec_name", ["fp64", "fp32mg"])
def test_vcycle_launched_levels_above_workgroup_bottom(prec_name):
    """160 x 96, six levels: levels 0 to 2 (15360, 3840 and 960 cells) run as separate launches,
    the levels from 20 x 12 down to the 5 x 3 coarsest in one workgroup; partial wavefronts on
    every level.  Two V-cycles against the oracle's (FP64 within 1e-12, FP32 multigrid within 1e-4)."""
    from paper_2505_10857_amd import _abi as A
    from swe_workloads import synthetic_operator_2d
    prob = wedge_problem(160, 96)
    Jo, rhs_o = synthetic_operator_2d(160, 96, seed=4)
    p = prob.params
    prec, dt, bar = ((A.NMG_FP64, torch.float64, 1e-12) if prec_name == "fp64"
                     else (A.NMG_FP32_MG, torch.float32, 1e-4))
    s = _solver(prob, levels=6, precision=prec)
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(np.ascontiguousarray(rhs_o.transpose(2, 0, 1)), dtype=dt, device=DEV)
    dU = torch.zeros((3, 96, 160), dtype=dt, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    s.vcycle(None, rhs, dU, setup=False)
    d2 = vcycles2d(Jo, rhs_o, levels=6, ncycles=2, omega=p.omega, nu1=p.nu1, nu2=p.nu2)
    e = _rel(dU.double().cpu().numpy().transpose(1, 2, 0), d2)
    print(f"160x96 {prec_name}: two V-cycles rel err {e:.3e}")
    assert e <= bar
