"""Pins of the oracle's optional surface reconstruction (recon = 1): WENO3 on h + b with the
split source, for channels of constant width.  The paper's scheme (recon = 0) is not well
balanced; this option keeps a still surface steady to round-off on any bottom and stays third
order on smooth flow."""
import dataclasses
import math

import numpy as np
import pytest

from oracle import Oracle1D, blocks_to_dense
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, BC_WALL, G, bottom_faces_and_averages,
                           config1, e1_bottom, e1_problem, lake_at_rest)


def _still(prob, surface=1.0):
    _, za = bottom_faces_and_averages(prob)
    return np.stack([surface - za[2:-2], np.zeros(prob.n)])


@pytest.mark.parametrize("n,amp,right,centre", [(16, 0.3, "wall", 10.0), (64, 0.3, "wall", 10.0),
                                                (64, 0.6, "depth", 10.0), (256, 0.1, "depth", 10.0),
                                                (64, 0.4, "wall", 0.3), (64, 0.4, "wall", 24.5)])
def test_lake_at_rest_is_steady_to_roundoff(n, amp, right, centre):
    """Bumps in the middle and against either wall (where the ghosts must copy the surface)."""
    p = lake_at_rest(n, amp=amp, right=right, centre=centre)
    R, rn, res = Oracle1D(p).residual(_still(p))
    # fluxes are O(g h^2 / 2) ~ 5: round-off of their differences
    assert np.abs(R).max() < 50 * np.finfo(float).eps * 5.0, np.abs(R).max()
    # the paper's reconstruction leaves a truncation error on the same state
    R0, _, _ = Oracle1D(dataclasses.replace(p, recon=0)).residual(_still(p))
    assert np.abs(R0).max() > 1e3 * np.abs(R).max()


def test_surface_reconstruction_equals_the_paper_on_a_flat_bottom():
    """b = 0: eta = H, the split source vanishes like the paper's, so the two residuals agree to
    rounding on any state."""
    p = dataclasses.replace(config1(0), bottom=lambda x: (0.0 * np.asarray(x), 0.0 * np.asarray(x)))
    rng = np.random.default_rng([21, 0])
    U = p.initial_guess() * (1.0 + 0.05 * rng.uniform(-1.0, 1.0, (2, p.n)))
    R0, _, _ = Oracle1D(p).residual(U)
    R1, _, _ = Oracle1D(dataclasses.replace(p, recon=1)).residual(U)
    assert np.abs(R1 - R0).max() < 1e-13 * np.abs(R0).max()


def _exact_e1_h(x):
    b, _ = e1_bottom(x)
    u = np.ones_like(x)
    for _ in range(60):
        f = u ** 3 + (2 * G * b - 2 * G - 1) * u + 2 * G
        u = u - f / (3 * u ** 2 + (2 * G * b - 2 * G - 1))
    return 1.0 / u


def _cell_avg(f, x0, dx, n, npts=6):
    t, w = np.polynomial.legendre.leggauss(npts)
    xc = x0 + (np.arange(n) + 0.5) * dx
    return sum(wi * f(xc + ti * dx / 2) for ti, wi in zip(t, w)) / 2


def test_truncation_order_on_the_exact_e1_solution():
    """Section 5.1.1's smooth flow (constant width, hu = 1, exact h from the Bernoulli relation):
    R on the exact cell averages decays at least at third order with the surface reconstruction,
    as with the paper's."""
    errs = []
    for n in (96, 192, 384, 768):
        p = dataclasses.replace(e1_problem(n), recon=1)
        U = np.stack([_cell_avg(_exact_e1_h, p.x0, p.dx, n), np.ones(n)])
        errs.append(Oracle1D(p).residual(U)[2])
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert min(orders[1:]) > 3.0, orders


def test_jacobian_entries_equal_brute_force_global_fd():
    """Tiny walled channel over a bump: every kept entry of J3 / J5 is the forward difference of
    the global residual (ghosts that copy the surface included)."""
    n, eps = 8, 0.02
    p = lake_at_rest(n, amp=0.3)
    p = dataclasses.replace(p, x1=8.0, bc_right=BC(BC_DEPTH, h=1.0))
    o = Oracle1D(p)
    rng = np.random.default_rng([22, 0])
    U = _still(p) + np.stack([0.1 * rng.random(n), 0.3 * rng.random(n)])
    R0, _, _ = o.residual(U)
    dense = np.zeros((2 * n, 2 * n))
    for i in range(n):
        for m in range(2):
            Up = U.copy()
            Up[m, i] += eps
            dense[:, 2 * i + m] = ((o.residual(Up)[0] - R0) / eps).T.reshape(-1)
    for nb in (3, 5):
        A = blocks_to_dense(o.jacobian(U, eps=eps, alpha=0.0, nb=nb))
        band = np.abs(np.subtract.outer(np.arange(2 * n) // 2, np.arange(2 * n) // 2)) <= nb // 2
        assert np.array_equal(A[band], dense[band])


def test_newton_keeps_the_still_surface_and_solves_a_flow():
    """Algorithm 1 (which always takes a first step) from the still state stays there; from the
    flat-surface guess it converges on a subcritical flow over a bump, conserving discharge and
    Bernoulli energy to discretisation accuracy."""
    p = lake_at_rest(64, amp=0.3)
    o = Oracle1D(p)
    U0 = _still(p)
    U, it, res, _ = o.newton_solve(U0=U0)
    assert it == 1 and res < 1e-13
    assert np.abs(U - U0).max() < 1e-13
    pf = dataclasses.replace(config1(1), recon=1)
    Uf, it, res, _ = Oracle1D(pf).newton_solve()
    assert res < 1e-10 and it < 1000
    q = pf.meta["q"]
    assert np.max(np.abs(Uf[1] - q)) < 2e-3 * q
    b, _ = pf.bottom(pf.centres())
    E = (Uf[1] / Uf[0]) ** 2 / 2 + G * (Uf[0] + b)
    assert (E.max() - E.min()) / E.mean() < 2e-3
