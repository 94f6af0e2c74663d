"""Pins of the oracle's nested iteration (Algorithm 3) and its Appendix A interpolation."""
import math

import numpy as np
import pytest

import oracle
from swe_workloads import G, config2, nested_grids


def _cell_averages(f_antideriv, x0, dx, n):
    x = x0 + np.arange(n + 1) * dx
    F = f_antideriv(x)
    return (F[1:] - F[:-1]) / dx


def test_interpolation_is_conservative_everywhere():
    rng = np.random.default_rng(5)
    Uc = rng.uniform(0.5, 2.0, (2, 37))
    Uf = oracle.interp_a2(Uc)
    assert np.allclose(0.5 * (Uf[:, 0::2] + Uf[:, 1::2]), Uc, rtol=0, atol=1e-15)


def test_interpolation_reproduces_quadratics_including_the_end_cells():
    """Cell averages of a quadratic on the coarse grid give the exact fine-grid averages (A.1 is
    the quadratic through three cell averages; the end-cell reading keeps that property)."""
    a, b, c = 0.7, -1.3, 0.45
    F = lambda x: a * x + b * x ** 2 / 2 + c * x ** 3 / 3          # noqa: E731
    nc, x0, dxc = 23, -1.0, 0.13
    Uc = np.vstack([_cell_averages(F, x0, dxc, nc), 2.0 * _cell_averages(F, x0, dxc, nc)])
    Uf = oracle.interp_a2(Uc)
    exact = _cell_averages(F, x0, dxc / 2, 2 * nc)
    assert np.abs(Uf[0] - exact).max() < 1e-13
    assert np.abs(Uf[1] - 2.0 * exact).max() < 1e-13


def test_interior_weights_are_those_of_eq_a2():
    Uc = np.zeros((2, 9))
    Uc[0, 4] = 1.0                   # a unit coarse average at cell 4
    Uf = oracle.interp_a2(Uc)[0]
    # children of cell 3 see it as the right neighbour, of cell 5 as the left one
    assert Uf[6] == -1.0 / 8 and Uf[7] == 1.0 / 8
    assert Uf[8] == 1.0 and Uf[9] == 1.0
    assert Uf[10] == 1.0 / 8 and Uf[11] == -1.0 / 8


def test_nested_grids_follow_the_hierarchy():
    p = config2(0, "sub", n=800, levels=4)
    gs = nested_grids(p)
    assert [g.n for g in gs] == [800, 400, 200, 100]
    assert [g.levels for g in gs] == [4, 3, 2, 1]
    assert gs[0].params.eps == p.params.eps and gs[-1].params.eps == 0.2
    assert [g.params.alpha for g in gs] == [p.params.alpha] * 3 + [5.0]


def test_nested_solve_reaches_the_same_discrete_solution():
    """Subcritical hump, 800 cells: nested iteration and plain Newton from the flat surface end
    at the same solution of the discrete equations (both driven to res < 1e-13)."""
    p = config2(1, "sub", n=800, levels=4)
    U, rep = oracle.nested_solve(p, tol=1e-13)
    assert all(r[2] < 1e-13 for r in rep)
    Up, it, res, _ = oracle.Oracle1D(p).newton_solve(tol=1e-13)
    assert res < 1e-13
    assert np.abs(U - Up).max() < 1e-10


def test_nested_solve_reaches_the_transcritical_flow():
    """Transcritical hump (q = 1.53, h_out = 0.66), 800 cells: plain Newton from the flat surface
    breaks down, the nested iteration converges on every grid to a flow that is subcritical
    upstream and supercritical downstream with the discharge q throughout."""
    p = config2(0, "trans", n=800, levels=4)
    _, it, res, _ = oracle.Oracle1D(p).newton_solve(n_max=300)
    assert not (res < p.params.tol)
    U, rep = oracle.nested_solve(p)
    assert all(r[2] < p.params.tol for r in rep), rep
    H, Q = U
    q = p.meta["q"]
    assert np.abs(Q - q).max() < 0.01 * q
    fr = np.abs(Q / H) / np.sqrt(G * H)      # unit width: h = H
    assert fr[:50].max() < 1.0 < fr[-50:].min()
