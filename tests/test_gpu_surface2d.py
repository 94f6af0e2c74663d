"""The 2D surface reconstruction (recon = NMG_RECON_SURFACE) on the GPU against the oracle's, through
the C ABI: residual, J9 and J21 within 1e-12 (reported bitwise), still water steady to rounding
on a non-flat bottom, Newton to the oracle's converged state within 1e-10 (FP32 multigrid within
1e-9), and the full 1024 x 512 wedge grid (whole residual, sampled Jacobian rows)."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from oracle.swe2d import Oracle2D  # noqa: E402
from swe_workloads import lake_at_rest_2d, wedge_problem  # noqa: E402

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
    rng = np.random.default_rng([11, seed])
    U = prob.initial_guess()
    return U * (1.0 + amp * rng.uniform(-1.0, 1.0, U.shape))


def _ragged():
    from test_gpu_parity_2d import _ragged_channel
    return dataclasses.replace(_ragged_channel(), recon=1)


CASES = [("wedge32x16", lambda: dataclasses.replace(wedge_problem(32, 16), recon=1)),
         ("ragged56x24", _ragged),
         ("lake32x16", lambda: lake_at_rest_2d(32, 16)),
         ("lake_mixed48x24", lambda: lake_at_rest_2d(48, 24, sides="mixed", levels=4))]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_surface_residual_and_jacobians(name, make):
    prob = make()
    o = Oracle2D(prob)
    for jac in (9, 21):
        s = _solver(prob, jac=jac)
        U0 = _noisy(prob, 3)
        U = s.state(U0)
        R, rn, res = s.residual(U)
        Ro, rno, reso = o.residual(U0)
        eR = np.abs(R.cpu().numpy() - Ro).max()
        assert eR <= 1e-12 * max(np.abs(Ro).max(), 1.0)
        assert abs(res.item() - reso) <= 1e-12 * reso
        J = s.jacobian(U, R, rn).cpu().numpy()
        Jo = np.ascontiguousarray(o.jacobian(U0, which=jac).transpose(2, 3, 4, 0, 1))
        eJ = np.abs(J - Jo).max()
        print(f"{name} J{jac}: |dR| {eR:.2e} (bitwise {np.array_equal(R.cpu().numpy(), Ro)}), "
              f"|dJ| {eJ:.2e} (bitwise {np.array_equal(J, Jo)})", flush=True)
        assert eJ <= 1e-12 * np.abs(Jo).max()


@pytest.mark.parametrize("sides", ["walls", "mixed"])
def test_lake_at_rest_is_steady_on_the_gpu(sides):
    """Still water over a mound and a ripple: the surface variant's residual vanishes to rounding
    (the paper's scheme leaves O(1) on the same bottom).  In the closed basin, Newton from the
    still state ends after one step without moving it (with extrapolating ends the surface level
    is free, the Jacobian singular and the regularisation as small as the residual, so that step
    is not taken: the oracle's and this step both end non-finite)."""
    prob = lake_at_rest_2d(64, 32, levels=4, sides=sides)
    s = _solver(prob, check_every=1)
    U = s.state()
    R, _, res = s.residual(U)
    print(f"{sides}: max|R| {R.abs().max().item():.2e}, res {res.item():.2e}", flush=True)
    assert R.abs().max().item() < 1e-12
    R0, _, _ = _solver(dataclasses.replace(prob, recon=0)).residual(U)
    assert R0.abs().max().item() > 0.1
    if sides == "walls":
        U0 = U.clone()
        st, _ = s.newton_solve(U)
        assert st.status == 0 and st.iters == 1 and st.res < 1e-12
        assert (U - U0).abs().max().item() < 1e-12


@pytest.mark.parametrize("prec_name", ["fp64", "fp32mg"])
def test_surface_newton_matches_the_oracle(prec_name):
    """The wedge (seeded bumps on the bottom), 32 x 16, surface variant: the oracle's step count
    (within one) and converged state (FP64 within 1e-10; FP32 multigrid within 1e-9)."""
    from paper_2505_10857_amd import _abi as A
    prec, bar = (A.NMG_FP64, 1e-10) if prec_name == "fp64" else (A.NMG_FP32_MG, 1e-9)
    prob = dataclasses.replace(wedge_problem(32, 16), recon=1)
    s = _solver(prob, precision=prec, check_every=4)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, it, reso, _ = Oracle2D(prob).newton_solve()
    e = _rel(U.cpu().numpy(), Uo)
    print(f"{prec_name}: GPU {st.iters} steps res {st.res:.2e}; oracle {it} steps; rel err {e:.2e}", flush=True)
    assert st.status == 0 and abs(st.iters - it) <= 1
    assert e <= bar


def test_surface_full_size_wedge_grid():
    """1024 x 512 wedge, surface variant, generic state: the whole residual and J9 rows of sampled
    grid lines against the oracle's."""
    prob = dataclasses.replace(wedge_problem(1024, 512, seed=7), recon=1)
    s = _solver(prob)
    o = Oracle2D(prob)
    U0 = _noisy(prob, 9, amp=0.01)
    U = s.state(U0)
    R, rn, res = s.residual(U)
    Ro, rno, reso = o.residual(U0)
    assert _rel(R.cpu().numpy(), Ro) <= 1e-12
    J = s.jacobian(U, R, rn)
    for j0 in (0, 1, 300, 511):
        Jo = o.jacobian(U0, rows=(j0, j0 + 1), R=Ro, rn=rno)
        Jg = J[:, :, :, j0, :].cpu().numpy()
        Jt = np.ascontiguousarray(Jo[j0].transpose(1, 2, 3, 0))
        assert np.abs(Jg - Jt).max() <= 1e-12 * np.abs(Jt).max(), j0
