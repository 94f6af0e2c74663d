"""Pins of the 2D CPU oracle (section 4) against closed forms, symmetries, brute force, exact
cell averages of the differential operator and dense linear algebra."""
import math

import numpy as np
import pytest

import oracle
from oracle.swe2d import (Oracle2D, blocks_to_dense2d, coarse_operators, smooth2d,
                          stencil_offsets, vcycles2d)
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, BC_EXTRAP, BC_STATE, BC_WALL, G, Params,
                           Problem2D, wedge_problem)

oracle.lib()


def flat2(x, y):
    x = np.asarray(x, dtype=np.float64)
    return np.zeros_like(x * y), np.zeros_like(x * y), np.zeros_like(x * y)


def _prob(nx=12, ny=8, bottom=flat2, bc=None, x0=0.0, x1=3.0, y0=0.0, y1=2.0, levels=2, wall_x=0.0,
          eps=1e-6):
    bc = bc or [BC(BC_EXTRAP)] * 4
    return Problem2D("t", x0, x1, y0, y1, nx, ny, levels, bottom, bc, Params(eps=eps, omega=0.1),
                     wall_x=wall_x)


def smooth_bottom(a=0.1):
    def f(x, y):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        return (a * np.sin(x) * np.sin(y), a * np.cos(x) * np.sin(y), a * np.sin(x) * np.cos(y))
    return f


def smooth_state(x, y):
    h = 1.0 + 0.1 * np.sin(x) * np.cos(y)
    u = 0.5 + 0.1 * np.cos(x + y)
    v = 0.3 + 0.1 * np.sin(x - y)
    return np.stack([h, h * u, h * v])


def cell_avg2(f, p, npts=6):
    t, w = np.polynomial.legendre.leggauss(npts)
    xc = p.x0 + (np.arange(p.nx) + 0.5) * p.dx
    yc = p.y0 + (np.arange(p.ny) + 0.5) * p.dy
    acc = 0.0
    for ti, wi in zip(t, w):
        for tj, wj in zip(t, w):
            X, Y = np.meshgrid(xc + ti * p.dx / 2, yc + tj * p.dy / 2)
            acc = acc + wi * wj * f(X, Y)
    return acc / 4.0


# ---------------------------------------------------------------------------------------
# residual
# ---------------------------------------------------------------------------------------

def test_constant_state_flat_bottom_is_steady():
    for st in [(1.0, 0.5, -0.2), (2.0, 0.0, 0.0), (0.7, 3.0, 1.0)]:
        p = _prob(bc=[BC(BC_EXTRAP), BC(BC_EXTRAP), BC(BC_STATE, h=st[0], u=st[1] / st[0], v=st[2] / st[0]),
                      BC(BC_EXTRAP)])
        U = np.empty((3, p.ny, p.nx))
        for c in range(3):
            U[c] = st[c]
        R = Oracle2D(p).residual(U)[0]
        assert np.abs(R).max() < 1e-12 * (1 + G * st[0] ** 2) / p.dx


def test_transposition_symmetry():
    rng = np.random.default_rng(0)
    nx, ny = 10, 8
    bot = smooth_bottom(0.05)
    p = _prob(nx, ny, bottom=bot, x1=2.5, y1=2.0,
              bc=[BC(BC_DISCHARGE, q=0.7), BC(BC_DEPTH, h=1.0), BC(BC_WALL), BC(BC_EXTRAP)])
    U = np.stack([1.0 + 0.1 * rng.random((ny, nx)), 0.5 + 0.1 * rng.random((ny, nx)),
                  0.2 + 0.1 * rng.random((ny, nx))])
    R = Oracle2D(p).residual(U)[0]
    botT = lambda x, y: (lambda b: (b[0], b[2], b[1]))(bot(y, x))
    pT = _prob(ny, nx, bottom=botT, x1=2.0, y1=2.5,
               bc=[BC(BC_WALL), BC(BC_EXTRAP), BC(BC_DISCHARGE, q=0.7), BC(BC_DEPTH, h=1.0)])
    UT = np.stack([U[0].T, U[2].T, U[1].T]).copy()
    RT = Oracle2D(pT).residual(UT)[0]
    ref = np.stack([R[0].T, R[2].T, R[1].T])
    assert np.allclose(RT, ref, rtol=1e-13, atol=1e-13 * np.abs(R).max())


def test_mirror_symmetry_in_x():
    rng = np.random.default_rng(1)
    nx, ny = 12, 6
    bot = smooth_bottom(0.05)
    L = 3.0
    p = _prob(nx, ny, bottom=bot, x1=L, bc=[BC(BC_WALL), BC(BC_EXTRAP), BC(BC_WALL), BC(BC_WALL)])
    U = np.stack([1.0 + 0.1 * rng.random((ny, nx)), 0.3 * rng.standard_normal((ny, nx)),
                  0.3 * rng.standard_normal((ny, nx))])
    R = Oracle2D(p).residual(U)[0]
    botM = lambda x, y: (lambda b: (b[0], -b[1], b[2]))(bot(L - np.asarray(x), y))
    pM = _prob(nx, ny, bottom=botM, x1=L, bc=[BC(BC_EXTRAP), BC(BC_WALL), BC(BC_WALL), BC(BC_WALL)])
    UM = np.stack([U[0][:, ::-1], -U[1][:, ::-1], U[2][:, ::-1]]).copy()
    RM = Oracle2D(pM).residual(UM)[0]
    ref = np.stack([R[0][:, ::-1], -R[1][:, ::-1], R[2][:, ::-1]])
    assert np.allclose(RM, ref, rtol=1e-11, atol=1e-11 * np.abs(R).max())


def test_y_invariant_flow_between_walls():
    nx, ny = 16, 6
    bot = lambda x, y: (0.1 * np.exp(-(np.asarray(x) - 2.0) ** 2) + 0 * np.asarray(y),
                        -0.2 * (np.asarray(x) - 2.0) * np.exp(-(np.asarray(x) - 2.0) ** 2) + 0 * np.asarray(y),
                        0 * np.asarray(x) * np.asarray(y))
    p = _prob(nx, ny, bottom=bot, x1=4.0, bc=[BC(BC_DISCHARGE, q=0.8), BC(BC_DEPTH, h=1.0), BC(BC_WALL), BC(BC_WALL)])
    xc = (np.arange(nx) + 0.5) * p.dx
    U = np.stack([np.tile(1.0 + 0.1 * np.cos(xc), (ny, 1)), np.tile(0.8 + 0.05 * np.sin(xc), (ny, 1)), np.zeros((ny, nx))])
    R = Oracle2D(p).residual(U)[0]
    assert np.all(R[2] == 0.0)
    for c in (0, 1):
        assert np.all(R[c] == R[c][0:1, :])


def _basin_bottom(x, y):
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    e = 0.1 * np.exp(-((x - 1.3) ** 2 + (y - 0.9) ** 2))
    return e, -2.0 * (x - 1.3) * e, -2.0 * (y - 0.9) * e


def test_mass_rows_telescope_in_a_closed_basin():
    """Eq. (20) is a flux difference per cell: summed over a grid closed by walls on all four
    sides (mirrored ghosts, so the mass flux through every wall face is zero), the mass rows
    R^h_ij dx dy cancel to rounding for any state, on any bottom (the mass equation has no
    source).  With the right side open the same sum is the outflow through it, far from zero,
    so the identity is not met by accident.  A flux taken from the wrong face, a sign, or a
    face length applied to one side only breaks the cancellation."""
    rng = np.random.default_rng(5)
    nx, ny = 20, 12
    U = np.stack([1.0 + 0.2 * rng.uniform(-1, 1, (ny, nx)), 0.3 * rng.uniform(-1, 1, (ny, nx)),
                  0.3 * rng.uniform(-1, 1, (ny, nx))])
    closed = _prob(nx, ny, bottom=_basin_bottom, bc=[BC(BC_WALL)] * 4)
    R = Oracle2D(closed).residual(U)[0]
    assert abs(R[0].sum()) <= 1e-13 * np.abs(R[0]).sum()
    open_right = _prob(nx, ny, bottom=_basin_bottom, bc=[BC(BC_WALL), BC(BC_EXTRAP), BC(BC_WALL), BC(BC_WALL)])
    Ro = Oracle2D(open_right).residual(U)[0]
    assert abs(Ro[0].sum()) >= 1e-3 * np.abs(Ro[0]).sum()


@pytest.mark.parametrize("recon", [0, 1])
def test_residual_converges_to_cell_average_of_the_pde(recon):
    """R_ij -> (1/|I_ij|) int (F_x + G_y - S) at third order (interior cells, away from ghosts),
    for the paper's reconstruction and for the surface variant: the exact average is computed by
    the divergence theorem with Gauss rules on the edges and a tensor Gauss rule for the
    source."""
    import dataclasses
    bot = smooth_bottom(0.1)
    errs = []
    for n in (16, 32, 64):
        p = dataclasses.replace(_prob(n, n, bottom=bot, x0=0.0, x1=2.0, y0=0.0, y1=2.0), recon=recon)
        U = cell_avg2(smooth_state, p)
        R = Oracle2D(p).residual(U)[0]
        t, w = np.polynomial.legendre.leggauss(6)
        xf = p.x0 + np.arange(n + 1) * p.dx
        yf = p.y0 + np.arange(n + 1) * p.dy
        xc = p.x0 + (np.arange(n) + 0.5) * p.dx
        yc = p.y0 + (np.arange(n) + 0.5) * p.dy

        def F(x, y, d):
            s = smooth_state(x, y)
            h, u, v = s[0], s[1] / s[0], s[2] / s[0]
            if d == 0:
                return np.stack([h * u, h * u * u + 0.5 * G * h * h, h * u * v])
            return np.stack([h * v, h * u * v, h * v * v + 0.5 * G * h * h])

        ex = np.zeros((3, n, n))
        for ti, wi in zip(t, w):
            Yg, Xf = np.meshgrid(yc + ti * p.dy / 2, xf, indexing="ij")
            fx = F(Xf, Yg, 0)                                   # [3, n, n+1]
            ex += wi / 2 * (fx[:, :, 1:] - fx[:, :, :-1]) / p.dx
            Yf, Xg = np.meshgrid(yf, xc + ti * p.dx / 2, indexing="ij")
            gy = F(Xg, Yf, 1)                                   # [3, n+1, n]
            ex += wi / 2 * (gy[:, 1:, :] - gy[:, :-1, :]) / p.dy
        src = lambda X, Y: np.stack([0 * X, -G * smooth_state(X, Y)[0] * bot(X, Y)[1],
                                     -G * smooth_state(X, Y)[0] * bot(X, Y)[2]])
        ex -= cell_avg2(src, p)
        errs.append(np.abs(R - ex)[:, 3:-3, 3:-3].max())
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert orders[-1] > 2.5, (errs, orders)


# ---------------------------------------------------------------------------------------
# the surface variant (reading S1): still water on any bottom
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("sides", ["walls", "mixed"])
def test_surface_variant_keeps_a_lake_at_rest(sides):
    """Still water over a mound and a ripple: the surface variant's residual vanishes to
    rounding (walls all round, or extrapolation left and right), the paper's reconstruction
    leaves an O(1) residual on the same bottom."""
    from swe_workloads import lake_at_rest_2d
    p1 = lake_at_rest_2d(32, 16, recon=1, sides=sides)
    U = p1.initial_guess()
    R1 = Oracle2D(p1).residual(U)[0]
    assert np.abs(R1).max() < 1e-12
    import dataclasses
    R0 = Oracle2D(dataclasses.replace(p1, recon=0)).residual(U)[0]
    assert np.abs(R0).max() > 0.1


def test_surface_variant_is_the_paper_scheme_on_a_flat_bottom():
    """With b = 0 the surface is the depth, the split source vanishes like the paper's, and
    the ghosts copy the same values: the residual is the paper's bit for bit, at a generic state
    with every boundary kind of the wedge."""
    import dataclasses
    p0 = wedge_problem(32, 16, n_bumps=0)
    rng = np.random.default_rng(1)
    U = p0.initial_guess() * (1 + 0.02 * rng.uniform(-1, 1, (3, 16, 32)))
    R0 = Oracle2D(p0).residual(U)[0]
    R1 = Oracle2D(dataclasses.replace(p0, recon=1)).residual(U)[0]
    assert np.array_equal(R0, R1)


def test_surface_variant_newton_stays_at_rest_and_reaches_a_flow():
    """Newton from the still state ends after its first step with res at rounding level; on
    the wedge (its seeded bumps on the bottom) the surface variant converges in the steps of the
    paper's scheme, to a solution that differs from it at truncation level."""
    from swe_workloads import lake_at_rest_2d
    p = lake_at_rest_2d(16, 8, recon=1, levels=2)
    U, it, res, _ = Oracle2D(p).newton_solve()
    assert it == 1 and res < 1e-12
    assert np.abs(U - p.initial_guess()).max() < 1e-12
    import dataclasses
    pw = dataclasses.replace(wedge_problem(32, 16), recon=1)
    U1, it1, r1, _ = Oracle2D(pw).newton_solve()
    U0, it0, r0, _ = Oracle2D(dataclasses.replace(pw, recon=0)).newton_solve()
    assert r1 < 1e-10 and r0 < 1e-10
    assert abs(it1 - it0) <= max(2, it0 // 5)
    d = np.abs(U1 - U0).max()
    assert 1e-6 < d < 0.1, d


# ---------------------------------------------------------------------------------------
# Jacobian (eq. 12, 13, 21)
# ---------------------------------------------------------------------------------------

def _flux_jac(U, d):
    h, u, v = U[0], U[1] / U[0], U[2] / U[0]
    if d == 0:
        return np.array([[0, 1, 0], [G * h - u * u, 2 * u, 0], [-u * v, v, u]])
    return np.array([[0, 0, 1], [-u * v, v, u], [G * h - v * v, 0, 2 * v]])


def test_j9_matches_closed_form_at_constant_state():
    """At a constant state on a flat bottom the WENO weights are stationary and the
    characteristic projection cancels, the two Gauss points' slope terms cancel, and LLF
    linearises to (A + aI)/2 and (A - aI)/2: the Jacobian is a sum of 1D third-order stencils in
    x and y, and the blocks the simplification drops vanish."""
    st = np.array([1.2, 0.6, -0.3])
    p = _prob(12, 10, x1=3.0, y1=2.5)
    U = np.empty((3, p.ny, p.nx))
    for c in range(3):
        U[c] = st[c]
    o = Oracle2D(p)
    J = o.jacobian(U, eps=1e-7, alpha=0.0, which=21)
    wm = {-1: -1 / 6, 0: 5 / 6, 1: 1 / 3}
    wp = {-1: 1 / 3, 0: 5 / 6, 1: -1 / 6}
    ref = {}
    for d, hd in ((0, p.dx), (1, p.dy)):
        A = _flux_jac(st, d)
        a = abs(st[1 + d] / st[0]) + math.sqrt(G * st[0])
        dL, dR = (A + a * np.eye(3)) / 2, (A - a * np.eye(3)) / 2
        for off in range(-2, 3):
            B = dL * wm.get(off, 0.0) + dR * wp.get(off - 1, 0.0) - dL * wm.get(off + 1, 0.0) - dR * wp.get(off, 0.0)
            key = (off, 0) if d == 0 else (0, off)
            ref[key] = ref.get(key, 0) + B / hd
    i, j = 6, 5
    for b, (di, dj) in enumerate(stencil_offsets(21)):
        exp = ref.get((di, dj), np.zeros((3, 3)))
        assert np.allclose(J[j, i, b], exp, atol=3e-5 * np.abs(exp).max() + 1e-6), (di, dj, J[j, i, b], exp)


@pytest.mark.parametrize("recon", [0, 1])
def test_j9_is_j21_on_the_cross_and_brute_force_fd(recon):
    """J21 holds every nonzero of the global difference quotient (brute force over all unknowns),
    J9 is its cross, for the paper's reconstruction and the surface variant, with every boundary
    kind but DISCHARGE in play."""
    import dataclasses
    rng = np.random.default_rng(2)
    nx, ny, eps = 7, 6, 1e-4
    p = _prob(nx, ny, bottom=smooth_bottom(0.05), x1=1.75, y1=1.5, wall_x=0.6,
              bc=[BC(BC_STATE, h=1.0, u=2.0, v=-0.3), BC(BC_EXTRAP), BC(BC_WALL), BC(BC_DEPTH, h=1.1)])
    p = dataclasses.replace(p, recon=recon)
    U = np.stack([1.0 + 0.1 * rng.random((ny, nx)), 1.5 + 0.1 * rng.random((ny, nx)),
                  -0.2 + 0.1 * rng.random((ny, nx))])
    o = Oracle2D(p)
    R0, _, _ = o.residual(U)
    J9 = o.jacobian(U, eps=eps, alpha=0.0, which=9)
    J21 = o.jacobian(U, eps=eps, alpha=0.0, which=21)
    assert np.array_equal(J9, J21[:, :, :9])
    n = nx * ny
    dense = np.zeros((3 * n, 3 * n))
    for j in range(ny):
        for i in range(nx):
            for m in range(3):
                Up = U.copy()
                Up[m, j, i] = U[m, j, i] + eps
                dense[:, (j * nx + i) * 3 + m] = ((o.residual(Up)[0] - R0) / eps).transpose(1, 2, 0).reshape(-1)
    A21 = blocks_to_dense2d(J21)
    mask = A21 != 0
    assert np.allclose(A21[mask], dense[mask], rtol=0, atol=1e-12 * np.abs(dense).max())
    # the full stencil holds every nonzero of the global difference quotient
    assert np.abs(dense[~mask]).max() == 0.0


def test_dropped_blocks_are_small_on_the_wedge():
    """Section 4.1, jump over a wedge: every block the simplification drops stays below 0.5 and
    most kept blocks exceed 1 (the paper's fractions -- all kept blocks above 0.5, 98% of the
    dropped ones below 1e-6 -- are not reproduced on this rescaled domain: here a few kept
    blocks far from the jump are small and the dropped ones are ~1e-3 of the kept ones)."""
    p = wedge_problem(16, 8)
    o = Oracle2D(p)
    U, it, res, _ = o.newton_solve(n_max=200)
    assert res < 1e-10
    J = o.jacobian(U, which=21)
    mag = np.abs(J).sum(axis=(3, 4))
    kept, drop = mag[:, :, :9], mag[:, :, 9:]
    kept = kept[kept > 0]           # blocks whose column cell lies inside the grid
    assert np.mean(kept > 1.0) > 0.75
    assert drop.max() < 0.5
    assert np.median(drop) < 1e-3 * np.median(kept)


# ---------------------------------------------------------------------------------------
# multigrid (section 4.2, eq. 22-25)
# ---------------------------------------------------------------------------------------

def _wedge_operator(nx=16, ny=8):
    p = wedge_problem(nx, ny)
    o = Oracle2D(p)
    U = p.initial_guess()
    R, rn, _ = o.residual(U)
    return p, o.jacobian(U), R


def _P2(nx, ny):
    P = np.zeros((3 * nx * ny, 3 * (nx // 2) * (ny // 2)))
    for j in range(ny):
        for i in range(nx):
            for c in range(3):
                P[(j * nx + i) * 3 + c, ((j // 2) * (nx // 2) + i // 2) * 3 + c] = 1
    return P


def test_coarse_operators_are_galerkin_and_five_point():
    p, J, _ = _wedge_operator(16, 8)
    A = blocks_to_dense2d(J)
    Jc = coarse_operators(J, 3)
    P = _P2(16, 8)
    Ac = P.T @ A @ P
    assert np.allclose(blocks_to_dense2d(Jc[0]), Ac, rtol=1e-14, atol=1e-12)
    # the Galerkin product has no entries outside the five-point stencil (the text after eq. 24)
    five = blocks_to_dense2d(Jc[0]) != 0
    assert np.abs(Ac[~five]).max() < 1e-12
    P2 = _P2(8, 4)
    assert np.allclose(blocks_to_dense2d(Jc[1]), P2.T @ Ac @ P2, rtol=1e-14, atol=1e-12)


def test_smoother_fixed_point_and_two_level_exactness():
    p, J, R = _wedge_operator(16, 8)
    A = blocks_to_dense2d(J)
    rhs = np.transpose(R, (1, 2, 0)).reshape(-1)
    x = np.linalg.solve(A, -rhs)
    for sm in (0, 1):
        y = smooth2d(J, rhs, x, iters=1, omega=0.7, smoother=sm).reshape(-1)
        assert np.allclose(y, x, rtol=1e-11, atol=1e-13)
    rng = np.random.default_rng(3)
    x0 = rng.standard_normal(A.shape[0]) * 1e-3
    P = _P2(16, 8)
    ref = x0 + P @ np.linalg.solve(P.T @ A @ P, P.T @ (-rhs - A @ x0))
    y = vcycles2d(J, rhs, x0, levels=2, ncycles=1, nu1=0, nu2=0).reshape(-1)
    assert np.allclose(y, ref, rtol=1e-11, atol=1e-14)


@pytest.mark.parametrize("smoother", [0, 1])
def test_vcycles_converge_to_dense_solve_on_wedge_operator(smoother):
    p, J, R = _wedge_operator(32, 16)
    A = blocks_to_dense2d(J)
    rhs = np.transpose(R, (1, 2, 0)).reshape(-1)
    x = np.linalg.solve(A, -rhs)
    y = vcycles2d(J, rhs, None, levels=3, ncycles=12, omega=0.05, nu1=10, nu2=10, smoother=smoother).reshape(-1)
    assert np.abs(y - x).max() < 1e-7 * np.abs(x).max()


def _colour(i, j, nb):
    return i % 3 + 3 * (j % 3) if nb == 21 else (i + j) % (2 if nb == 5 else 3)


@pytest.mark.parametrize("which", [9, 21])
def test_colourings_leave_no_coupling_within_a_colour(which):
    """The cross stencil under (i + j) mod 3 and the full stencil under (i mod 3) + 3 (j mod 3):
    no offset of the stencil joins two cells of one colour; (i + j) mod 3 would not do for the
    full stencil, whose diagonal (1, -1) keeps i + j."""
    for di, dj in stencil_offsets(which)[1:]:
        for i in range(3):
            for j in range(3):
                assert _colour(i, j, which) != _colour(i + di, j + dj, which), (di, dj)
    assert any((di + dj) % 3 == 0 for di, dj in stencil_offsets(21)[1:])


@pytest.mark.parametrize("which", [9, 21])
def test_colour_sweeps_are_block_jacobi_updates_of_the_dense_system(which):
    """One smoothing iteration of the oracle equals, on the dense matrix of the operator, the
    schedule of colour updates (colours forward, backward, forward, backward), each a
    simultaneous block-Jacobi relaxation of the cells of that colour: x_c <- (1 - w) x_c -
    w D_c^-1 (rhs_c + sum of the off-diagonal blocks times x)."""
    p, J9, R = _wedge_operator(12, 9)
    o = Oracle2D(p)
    U = p.initial_guess()
    Rr, rn, _ = o.residual(U)
    J = o.jacobian(U, R=Rr, rn=rn, which=which)
    A = blocks_to_dense2d(J)
    nx, ny = p.nx, p.ny
    rng = np.random.default_rng(4)
    rhs = rng.standard_normal(3 * nx * ny)
    x0 = rng.standard_normal(3 * nx * ny) * 0.1
    omega = 0.7
    C = 9 if which == 21 else 3
    col = np.array([_colour(i, j, which) for j in range(ny) for i in range(nx)])
    D = np.zeros_like(A)
    for k in range(nx * ny):
        D[3 * k:3 * k + 3, 3 * k:3 * k + 3] = A[3 * k:3 * k + 3, 3 * k:3 * k + 3]
    Dinv = np.zeros_like(A)
    for k in range(nx * ny):
        Dinv[3 * k:3 * k + 3, 3 * k:3 * k + 3] = np.linalg.inv(A[3 * k:3 * k + 3, 3 * k:3 * k + 3])
    off = A - D
    x = x0.copy()
    order = (list(range(C)) + list(range(C - 1, -1, -1))) * 2
    for c in order:
        sel = np.repeat(col == c, 3)
        t = Dinv @ (rhs + off @ x)
        x[sel] = (1 - omega) * x[sel] - omega * t[sel]
    y = smooth2d(J, rhs, x0, iters=1, omega=omega, smoother=0).reshape(-1)
    assert np.abs(y - x).max() < 1e-12 * np.abs(x).max()


def test_nmgm21_and_nmgm9_take_the_same_newton_steps():
    """Section 5.2: the full and the simplified Jacobian converge almost alike (the linear solver
    changes, not the discrete equations).  Wedge 16 x 8, 32 x 16: the same Newton step counts,
    and the two solutions agree to the level the stopping test leaves."""
    for nx, ny in ((16, 8), (32, 16)):
        p = wedge_problem(nx, ny)
        o = Oracle2D(p)
        U9, it9, r9, _ = o.newton_solve(which=9)
        U21, it21, r21, _ = o.newton_solve(which=21)
        assert r9 < 1e-10 and r21 < 1e-10
        assert abs(it9 - it21) <= max(1, it9 // 10), (nx, it9, it21)
        assert np.abs(U9 - U21).max() < 1e-8


def test_j21_vcycles_converge_to_dense_solve():
    p = wedge_problem(32, 16)
    o = Oracle2D(p)
    U = p.initial_guess()
    R, rn, _ = o.residual(U)
    J = o.jacobian(U, R=R, rn=rn, which=21)
    A = blocks_to_dense2d(J)
    rhs = np.transpose(R, (1, 2, 0)).reshape(-1)
    x = np.linalg.solve(A, -rhs)
    y = vcycles2d(J, rhs, None, levels=3, ncycles=12, omega=0.05, nu1=10, nu2=10).reshape(-1)
    assert np.abs(y - x).max() < 1e-7 * np.abs(x).max()


def test_coarsest_dense_solve_matches_lapack():
    p, J, R = _wedge_operator(8, 4)
    A = blocks_to_dense2d(J)
    rhs = np.transpose(R, (1, 2, 0)).reshape(-1)
    y = vcycles2d(J, rhs, None, levels=1, ncycles=1).reshape(-1)
    assert np.allclose(y, np.linalg.solve(A, -rhs), rtol=1e-12, atol=1e-15)


# ---------------------------------------------------------------------------------------
# Newton on the jump over a wedge (section 5.2.2, rescaled)
# ---------------------------------------------------------------------------------------

@pytest.mark.parametrize("smoother", [0, 1])
def test_wedge_newton_converges_to_the_oblique_jump(smoother):
    """Jump over a wedge from the uniform inflow state (eq. 31 analogue): converges, and behind
    the jump along the wall the depth reaches the oblique-jump value for Fr = 2.736 and
    deflection 8.95 degrees, h2/h1 = 1.50 (textbook oblique-jump relations)."""
    p = wedge_problem(32, 16)
    o = Oracle2D(p)
    U, it, res, hist = o.newton_solve(n_max=300, smoother=smoother)
    assert res < 1e-10, (it, res)
    assert abs(U[0].max() - 1.50) < 0.02
    xc = p.x0 + (np.arange(p.nx) + 0.5) * p.dx
    assert abs(U[0, 0, xc > 30].mean() - 1.50) < 0.03          # along the wall, well behind the corner
    assert abs(U[0, -1, :8].mean() - 1.0) < 1e-3               # undisturbed inflow, top-left
    assert np.abs(U[2, 0, xc > 30] / U[0, 0, xc > 30]).max() < 0.05 * 8.57   # flow follows the wall


def test_multicolour_smoother_needs_the_smaller_relaxation_on_the_jump():
    """At the converged 16x8 jump the multicolour V-cycle diverges with omega = 0.1 and
    contracts with 0.05, while the paper's directional sweeps contract with 0.1."""
    p = wedge_problem(16, 8)
    o = Oracle2D(p)
    U, it, res, _ = o.newton_solve(n_max=300, smoother=1, omega=0.1)
    R, rn, _ = o.residual(U)
    J = o.jacobian(U, R=R, rn=rn)
    n = 3 * p.nx * p.ny
    rho = {}
    for sm, om in ((0, 0.1), (0, 0.05), (1, 0.1)):
        E = np.zeros((n, n))
        for k in range(n):
            e = np.zeros(n)
            e[k] = 1.0
            E[:, k] = vcycles2d(J, np.zeros(n), e, levels=p.levels, ncycles=1, omega=om, nu1=10,
                                nu2=10, smoother=sm).reshape(-1)
        rho[(sm, om)] = np.abs(np.linalg.eigvals(E)).max()
    assert rho[(0, 0.1)] > 1.0 and rho[(0, 0.05)] < 0.5 and rho[(1, 0.1)] < 0.5, rho


def test_source_quadrature_exact_for_linear_depth_and_bilinear_bottom():
    """Depth linear in x and y, bottom b = x y: the reconstructions are exact on linear data, the
    quadratic through three face averages is exact at the Gauss points, and the tensor Gauss rule
    integrates g h b_x = g h y and g h b_y = g h x exactly, so R(b) - R(flat) equals minus the
    exact cell averages of g h b_x and g h b_y (interior cells)."""
    nx, ny = 10, 8
    bxy = lambda x, y: (np.asarray(x) * np.asarray(y), np.asarray(y) + 0 * np.asarray(x), np.asarray(x) + 0 * np.asarray(y))
    pb = _prob(nx, ny, bottom=bxy, x1=2.5, y1=2.0)
    pf = _prob(nx, ny, x1=2.5, y1=2.0)
    xc = (np.arange(nx) + 0.5) * pb.dx
    yc = (np.arange(ny) + 0.5) * pb.dy
    X, Y = np.meshgrid(xc, yc)
    U = np.stack([1.0 + 0.3 * X + 0.5 * Y, 0.4 + 0 * X, 0.1 + 0 * X])   # cell averages of linear data
    d = Oracle2D(pb).residual(U)[0] - Oracle2D(pf).residual(U)[0]
    # exact averages: (1/|I|) int g (1 + 0.3x + 0.5y) y dxdy and ... x dxdy
    h = lambda x, y: 1.0 + 0.3 * x + 0.5 * y
    ex_x = cell_avg2(lambda x, y: G * h(x, y) * y, pb)
    ex_y = cell_avg2(lambda x, y: G * h(x, y) * x, pb)
    s = (slice(2, -2), slice(2, -2))
    assert np.allclose(d[1][s], ex_x[s], rtol=1e-12)
    assert np.allclose(d[2][s], ex_y[s], rtol=1e-12)
    assert np.abs(d[0]).max() == 0.0
