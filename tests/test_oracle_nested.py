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


# ---- two dimensions: eq. (A.3) and Algorithm 3 on a 2D problem -----------------------------

def test_interpolation_2d_is_conservative_everywhere():
    """Every coarse average is the mean of its four children, corners and edges included."""
    from oracle import swe2d
    rng = np.random.default_rng(6)
    Uc = rng.uniform(0.5, 2.0, (3, 9, 13))
    Uf = swe2d.interp_a3(Uc)
    assert Uf.shape == (3, 18, 26)
    quarters = Uf.reshape(3, 9, 2, 13, 2).mean(axis=(2, 4))
    assert np.abs(quarters - Uc).max() < 1e-15


def test_interpolation_2d_reproduces_biquadratics_including_the_borders():
    """Coarse cell averages of any product of quadratics in x and y give the exact fine averages
    in every cell, the border rows and columns and the corners included (eq. A.3 is the tensor
    product of the quadratics A.1)."""
    from oracle import swe2d
    fx = lambda x: 0.3 * x - 0.8 * x ** 2 / 2 + 1.1 * x ** 3 / 3     # noqa: E731  antiderivatives
    fy = lambda y: 1.0 * y + 0.4 * y ** 2 / 2 - 0.6 * y ** 3 / 3     # noqa: E731
    gx = lambda x: 2.0 * x + 0.5 * x ** 2 / 2                         # noqa: E731
    gy = lambda y: -0.2 * y ** 3 / 3 + 0.7 * y                        # noqa: E731
    nx, ny, x0, y0, dx, dy = 7, 5, -0.4, 0.2, 0.17, 0.23

    def averages(ax, ay, nx, ny, dx, dy):
        return np.outer(_cell_averages(ay, y0, dy, ny), _cell_averages(ax, x0, dx, nx))

    Uc = np.stack([averages(fx, fy, nx, ny, dx, dy), averages(gx, gy, nx, ny, dx, dy),
                   averages(fx, fy, nx, ny, dx, dy) + averages(gx, gy, nx, ny, dx, dy)])
    Uf = swe2d.interp_a3(Uc)
    exact = [averages(fx, fy, 2 * nx, 2 * ny, dx / 2, dy / 2), averages(gx, gy, 2 * nx, 2 * ny, dx / 2, dy / 2)]
    exact.append(exact[0] + exact[1])
    for c in range(3):
        assert np.abs(Uf[c] - exact[c]).max() < 1e-13


def test_interpolation_2d_interior_weights_are_products_of_eq_a2():
    """A unit average in an interior coarse cell spreads over its 3 x 3 neighbourhood with the
    products of the one-dimensional weights of eq. (A.2): 1 on its own children's rows and columns,
    -1/8 and +1/8 towards and away from it in the neighbours' children."""
    from oracle import swe2d
    Uc = np.zeros((3, 7, 9))
    Uc[1, 3, 4] = 1.0
    Uf = swe2d.interp_a3(Uc)[1]
    w = {(-1, 0): -1 / 8, (-1, 1): 1 / 8, (0, 0): 1.0, (0, 1): 1.0, (1, 0): 1 / 8, (1, 1): -1 / 8}
    for dj in (-1, 0, 1):
        for hy in (0, 1):
            for di in (-1, 0, 1):
                for hx in (0, 1):
                    want = w[(di, hx)] * w[(dj, hy)]
                    assert Uf[2 * (3 + dj) + hy, 2 * (4 + di) + hx] == want
    mask = np.ones_like(Uf, dtype=bool)
    mask[4:10, 6:12] = False
    assert not Uf[mask].any()


def test_interpolation_2d_reduces_to_the_1d_one():
    """A state that does not vary along y (x) is refined by eq. (A.2) along x (y) in every row
    (column): the 1D interpolation of the oracle's 1D solver, a separate implementation."""
    from oracle import swe2d
    rng = np.random.default_rng(8)
    row = rng.uniform(0.5, 2.0, 11)
    col = rng.uniform(0.5, 2.0, 6)
    Ux = swe2d.interp_a3(np.broadcast_to(row, (3, 6, 11)).copy())
    Uy = swe2d.interp_a3(np.broadcast_to(col[:, None], (3, 6, 11)).copy())
    rx = oracle.interp_a2(np.vstack([row, row]))[0]
    ry = oracle.interp_a2(np.vstack([col, col]))[0]
    assert np.abs(Ux - rx[None, None, :]).max() < 1e-15
    assert np.abs(Uy - ry[None, :, None]).max() < 1e-15


def test_nested_grids_2d_follow_the_hierarchy():
    from swe_workloads import nested_grids_2d, wedge_problem
    p = wedge_problem(64, 32, seed=0)
    gs = nested_grids_2d(p)
    assert [(g.nx, g.ny, g.levels) for g in gs] == [(64, 32, 4), (32, 16, 3), (16, 8, 2), (8, 4, 1)]
    assert [g.params.nu1 for g in gs] == [20, 15, 10, 10]
    assert all(g.params.omega == p.params.omega and g.params.eps == p.params.eps for g in gs)
    with pytest.raises(ValueError):
        nested_grids_2d(wedge_problem(48, 24, levels=5))


def test_nested_solve_2d_reaches_the_discrete_solution_of_plain_newton():
    """Wedge, 32 x 16 cells, three nested grids (8 x 4 direct, 16 x 8 and 32 x 16 multigrid),
    omega = 0.03: every grid converges, the finest in fewer Newton steps than plain Newton from
    the inflow state, and both end at the same solution of the discrete equations."""
    from oracle import swe2d
    from swe_workloads import wedge_problem
    p = wedge_problem(32, 16, seed=0)
    U, rep = swe2d.nested_solve2d(p, omega=0.03, tol=1e-12)
    assert [(r[0], r[1]) for r in rep] == [(8, 4), (16, 8), (32, 16)]
    assert all(r[3] < 1e-12 for r in rep)
    Up, it, res, _ = swe2d.Oracle2D(p).newton_solve(omega=0.03, tol=1e-12)
    assert res < 1e-12 and rep[-1][2] < it
    assert np.abs(U - Up).max() < 1e-10
