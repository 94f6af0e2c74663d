"""NMGM-21 on the GPU against the CPU oracle, through the C ABI: the full 21-cell Jacobian of
section 4.1 (desc.jac = 21), the nine-colour block SOR on its level (the coarse levels keep the
five-point operators of eq. 24), and the Newton iteration built on them.

Bars as for NMGM-9: J21 and V-cycles within 1e-12 relative (the arithmetic is written to be
bit-identical, which the tests report), Newton trajectories and converged states within 1e-10,
FP32 multigrid within 1e-9 of the FP64 oracle's converged state.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.swe2d import Oracle2D, vcycles2d  # noqa: E402
from swe_workloads import parabolic_bump_2d, wedge_problem  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _solver(prob, **kw):
    from paper_2505_10857_amd import Solver2D
    return Solver2D(prob, device=DEV, jac=21, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _noisy(prob, seed, amp=0.02):
    rng = np.random.default_rng([11, seed])
    U = prob.initial_guess()
    return U * (1.0 + amp * rng.uniform(-1.0, 1.0, U.shape))


def _ragged():
    from test_gpu_parity_2d import _ragged_channel
    return _ragged_channel()


CASES = [("wedge32x16", lambda: wedge_problem(32, 16)), ("wedge64x32", lambda: wedge_problem(64, 32, seed=3)),
         ("bump16x8", lambda: parabolic_bump_2d(16, 8)), ("ragged56x24", _ragged),
         ("wedge8x4", lambda: wedge_problem(8, 4, levels=1))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_j21_parity(name, make):
    """Every one of the 21 blocks of every row, interior rows (partially recomputed face states)
    and rows within two cells of a side (full re-evaluation with ghosts), at a generic state."""
    prob = make()
    s = _solver(prob)
    o = Oracle2D(prob)
    U0 = _noisy(prob, 2)
    U = s.state(U0)
    R, rn, _ = s.residual(U)
    J = s.jacobian(U, R, rn).cpu().numpy()                       # [21, 3, 3, ny, nx]
    Jo = o.jacobian(U0, which=21)                                 # [ny, nx, 21, 3, 3]
    Jo_t = np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1))
    err = np.abs(J - Jo_t).max()
    print(f"{name}: J21 max|dJ| = {err:.3e} (bitwise equal: {np.array_equal(J, Jo_t)})", flush=True)
    assert err <= 1e-12 * np.abs(Jo).max()
    # the cross blocks are J9's
    from paper_2505_10857_amd import Solver2D
    s9 = Solver2D(prob, device=DEV)
    J9 = s9.jacobian(U, R, rn).cpu().numpy()
    assert np.array_equal(J9, J[:9])


def _operator21(prob, seed=4):
    o = Oracle2D(prob)
    U0 = _noisy(prob, seed)
    R, rn, _ = o.residual(U0)
    return o.jacobian(U0, R=R, rn=rn, which=21), R


@pytest.mark.parametrize("nx,ny,levels", [(8, 4, 1), (16, 8, 2), (32, 16, 3), (160, 96, 6)])
def test_j21_vcycle_parity(nx, ny, levels):
    """One and two V-cycles from dU = 0 on an oracle J21: levels = 1 is the dense solve of the
    21-block operator; 16 x 8 and 32 x 16 run whole in the one-workgroup bottom (nine-colour
    passes with barriers); 160 x 96 launches the nine-colour passes on its finest level."""
    prob = wedge_problem(nx, ny, levels=levels)
    Jo, R = _operator21(prob)
    p = prob.params
    s = _solver(prob, levels=levels, nu1=3, nu2=3)
    J = torch.tensor(np.ascontiguousarray(Jo.transpose(2, 3, 4, 0, 1)), dtype=torch.float64, device=DEV)
    rhs = torch.tensor(R, dtype=torch.float64, device=DEV)
    dU = torch.zeros((3, ny, nx), dtype=torch.float64, device=DEV)
    s.vcycle(J, rhs, dU, setup=True)
    rhs_o = np.ascontiguousarray(R.transpose(1, 2, 0))
    d1 = vcycles2d(Jo, rhs_o, levels=levels, ncycles=1, omega=p.omega, nu1=3, nu2=3)
    g1 = dU.cpu().numpy().transpose(1, 2, 0)
    e1 = _rel(g1, d1)
    s.vcycle(None, rhs, dU, setup=False)
    d2 = vcycles2d(Jo, rhs_o, levels=levels, ncycles=2, omega=p.omega, nu1=3, nu2=3)
    e2 = _rel(dU.cpu().numpy().transpose(1, 2, 0), d2)
    print(f"{nx}x{ny} levels={levels}: J21 V-cycle rel err {e1:.3e}, {e2:.3e} "
          f"(bitwise: {np.array_equal(g1, d1)})", flush=True)
    assert e1 <= 1e-12 and e2 <= 1e-12


def test_nmgm21_newton_trajectory():
    """Five Newton steps of NMGM-21 on the wedge, 32 x 16: state and res history within 1e-10."""
    prob = wedge_problem(32, 16)
    s = _solver(prob, n_max=5, check_every=1)
    U = s.state()
    st, hist = s.newton_solve(U, max_hist=5)
    Uo, it, reso, hist_o = Oracle2D(prob).newton_solve(n_max=5, which=21)
    e = _rel(U.cpu().numpy(), Uo)
    print(f"NMGM-21 5 steps: state rel err {e:.3e}; res {hist} vs {hist_o}", flush=True)
    assert st.iters == it == 5
    assert e <= 1e-10
    assert np.all(np.abs(hist - hist_o) <= 1e-10 * np.maximum(np.abs(hist_o), 1e-300) + 1e-14)


@pytest.mark.parametrize("nx,ny", [(32, 16), (64, 32)])
def test_nmgm21_converges_like_the_oracle_and_like_nmgm9(nx, ny):
    """Wedge to res < 1e-10: NMGM-21 takes the oracle's step count (within one) to the oracle's
    state (within 1e-10), and the same step count as NMGM-9 (section 5.2)."""
    prob = wedge_problem(nx, ny)
    s = _solver(prob, check_every=4)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, it, reso, _ = Oracle2D(prob).newton_solve(which=21)
    e = _rel(U.cpu().numpy(), Uo)
    from paper_2505_10857_amd import Solver2D
    s9 = Solver2D(prob, device=DEV, check_every=4)
    U9 = s9.state()
    st9, _ = s9.newton_solve(U9)
    print(f"{nx}x{ny}: NMGM-21 GPU {st.iters} steps, oracle {it}; NMGM-9 GPU {st9.iters}; rel err {e:.3e}",
          flush=True)
    assert st.status == 0 and st.res < prob.params.tol
    assert abs(st.iters - it) <= 1
    assert e <= 1e-10
    assert st9.status == 0 and abs(st9.iters - st.iters) <= max(1, st.iters // 10)


def test_nmgm21_fp32_mg_converges_to_the_fp64_solution():
    from paper_2505_10857_amd import _abi as A
    prob = wedge_problem(32, 16)
    s = _solver(prob, precision=A.NMG_FP32_MG, check_every=4)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, it, reso, _ = Oracle2D(prob).newton_solve(which=21)
    e = _rel(U.cpu().numpy(), Uo)
    print(f"NMGM-21 FP32-MG: {st.iters} steps (oracle {it}), res {st.res:.3e}, rel err {e:.3e}", flush=True)
    assert st.status == 0 and st.res < prob.params.tol
    assert e <= 1e-9


def test_j21_full_size_sampled_rows():
    """1024 x 512 wedge at a generic state: J21 rows of sampled grid lines (both bands of the
    bottom and top sides, an interior line) against the oracle's rows."""
    prob = wedge_problem(1024, 512, seed=7)
    s = _solver(prob)
    o = Oracle2D(prob)
    U0 = _noisy(prob, 9, amp=0.01)
    U = s.state(U0)
    R, rn, _ = s.residual(U)
    Ro, rno, _ = o.residual(U0)
    J = s.jacobian(U, R, rn)
    for j0 in (0, 1, 255, 510, 511):
        Jo = o.jacobian(U0, rows=(j0, j0 + 1), R=Ro, rn=rno, which=21)
        Jg = J[:, :, :, j0, :].cpu().numpy()
        Jt = np.ascontiguousarray(Jo[j0].transpose(1, 2, 3, 0))
        err = np.abs(Jg - Jt).max()
        print(f"row {j0}: J21 max|dJ| {err:.3e}", flush=True)
        assert err <= 1e-12 * np.abs(Jt).max(), j0
