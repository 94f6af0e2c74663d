"""The surface reconstruction (NMG_RECON_SURFACE, constant width) on the GPU against the
oracle: residual and Jacobian element by element (1e-12 relative), Newton trajectories (1e-10),
the still surface over a bump kept to rounding through the whole Newton path, batches equal to
their instances alone, and a plan mixing reconstructions rejected."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, BC_WALL, Params, Problem1D,  # noqa: E402
                           bottom_faces_and_averages, config1, gaussian_bump, lake_at_rest,
                           unit_width)

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _solver(prob, **kw):
    from paper_2505_10857_amd import Solver1D
    return Solver1D(prob, device=DEV, **kw)


def _still(prob, surface=1.0):
    _, za = bottom_faces_and_averages(prob)
    return np.stack([surface - za[2:-2], np.zeros(prob.n)])


def _cases():
    yield "cfg1", dataclasses.replace(config1(2), recon=1)
    yield "lake-wall-ragged", lake_at_rest(328, amp=0.4, centre=0.4, levels=3)
    yield "lake-depth", lake_at_rest(256, amp=0.3, right="depth", levels=4)
    yield "tiny", Problem1D("tiny", 0.0, 1.0, 8, 2, gaussian_bump(0.05, 0.5, 0.05), unit_width,
                            BC(BC_DISCHARGE, q=0.5), BC(BC_DEPTH, h=1.0), Params(eps=0.1),
                            surface0=1.0, q0=0.5, recon=1)


def _states(prob):
    """A generic state (flat-surface guess with seeded noise) and, for flows, a mid-solve one."""
    rng = np.random.default_rng([31, prob.n])
    U0 = prob.initial_guess()
    U1 = U0 + np.stack([0.02 * rng.uniform(-1, 1, prob.n), 0.05 * rng.uniform(-1, 1, prob.n)])
    out = [U1]
    if prob.q0 != 0.0:
        out.append(oracle.Oracle1D(prob).newton_solve(n_max=5)[0])
    return out


@pytest.mark.parametrize("name,prob", list(_cases()), ids=[c[0] for c in _cases()])
def test_residual_parity(name, prob):
    s = _solver(prob)
    o = oracle.Oracle1D(prob)
    for U0 in _states(prob):
        R, rn, res = s.residual(s.state(U0))
        Ro, rno, reso = o.residual(U0)
        Rg = R.cpu().numpy()
        scale = max(np.abs(Ro).max(), 1.0)
        err = np.abs(Rg - Ro).max()
        print(f"{name}: max|dR| = {err:.3e} (bitwise equal: {np.array_equal(Rg, Ro)})")
        assert err <= 1e-12 * scale
        assert np.abs(rn.cpu().numpy() - rno).max() <= 1e-12 * scale
        assert abs(res.item() - reso) <= 2e-12 * scale


@pytest.mark.parametrize("nb", [3, 5])
@pytest.mark.parametrize("name,prob", list(_cases()), ids=[c[0] for c in _cases()])
def test_jacobian_parity(name, prob, nb):
    s = _solver(prob, jac=nb)
    o = oracle.Oracle1D(prob)
    for U0 in _states(prob):
        U = s.state(U0)
        R, rn, _ = s.residual(U)
        Jg = np.transpose(s.jacobian(U, R, rn).cpu().numpy(), (3, 0, 1, 2))
        Jo = o.jacobian(U0, nb=nb)
        err = np.abs(Jg - Jo).max()
        print(f"{name} J{nb}: max|dJ| = {err:.3e} / |J| {np.abs(Jo).max():.3e}")
        assert err <= 1e-12 * np.abs(Jo).max()


def test_still_surface_is_kept_by_the_gpu_path():
    """Residual at rounding on the still surface over a bump against a wall, and a Newton solve
    from it ends after its first step with the surface unchanged to rounding."""
    prob = lake_at_rest(512, amp=0.5, centre=1.0, levels=5)
    s = _solver(prob, check_every=1)
    U = s.state(_still(prob))
    R, _, res = s.residual(U)
    assert float(R.abs().max()) < 1e-13 and res.item() < 1e-14
    U0 = U.clone()
    st, _ = s.newton_solve(U)
    assert st.status == 0 and st.iters == 1
    assert float((U - U0).abs().max()) < 1e-13


def test_newton_trajectory_parity():
    prob = dataclasses.replace(config1(3), recon=1)
    o = oracle.Oracle1D(prob)
    for steps in (3, 20):
        s = _solver(prob, check_every=1, n_max=steps)
        U = s.state()
        st, _ = s.newton_solve(U)
        Uo, ito, _, _ = o.newton_solve(n_max=steps)
        assert st.iters == ito
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(f"after {steps} steps |U_gpu - U_oracle| = {err:.3e}")
        assert err <= 1e-10


def test_batch_equals_solo_and_mixed_plans_are_rejected():
    from paper_2505_10857_amd import BatchSolver1D
    from paper_2505_10857_amd import _abi as A
    probs = [dataclasses.replace(config1(i), recon=1) for i in range(3)]
    mix = BatchSolver1D(probs, device=DEV)
    Us = mix.states()
    rs = mix.solve(Us, use_graph=True)
    for k, p in enumerate(probs):
        solo = BatchSolver1D([p], device=DEV)
        Uk = solo.states()
        r = solo.solve(Uk, use_graph=False)
        assert rs[k][:2] == r[0][:2] and rs[k][1] == 0
        assert torch.equal(Us[k], Uk[0])
    with pytest.raises(A.NmgError):
        BatchSolver1D([probs[0], config1(0)], device=DEV)
