"""Pins of the 1D CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed forms, invariants,
brute force on tiny inputs, dense linear algebra, or the paper's printed numbers (Table 1).
"""
import ctypes
import math
import os

import numpy as np
import pytest

import oracle
from oracle import Oracle1D, blocks_to_dense, coarsen, smooth, vcycles
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, BC_EXTRAP, BC_WALL, G, Params, Problem1D,
                           config1, e1_bottom, e1_problem, flat, gaussian_bump, sine_width,
                           unit_width)

L = oracle.lib()
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _table(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


def _prob(n=16, bottom=flat, width=unit_width, bcl=None, bcr=None, x0=0.0, x1=1.0, levels=2):
    return Problem1D("t", x0, x1, n, levels, bottom, width,
                     bcl or BC(BC_EXTRAP), bcr or BC(BC_EXTRAP), Params(eps=1e-3))


# ---------------------------------------------------------------------------------------
# WENO3 (eq. 7-8)
# ---------------------------------------------------------------------------------------

def test_weno_constant_and_linear_exact():
    for a, d in [(1.3, 0.0), (0.7, 0.25), (-2.0, 1e-3)]:
        um, u0, up = a - d, a, a + d
        # linear data: both candidates are exact, so the face values are exact
        assert L.or1d_weno_plus(um, u0, up) == pytest.approx(a - d / 2, abs=1e-15)
        assert L.or1d_weno_minus(um, u0, up) == pytest.approx(a + d / 2, abs=1e-15)


def test_weno_equal_indicators_give_third_order_weights():
    # um == up makes beta0 == beta1, so the nonlinear weights equal the linear ones; the
    # third-order combinations are 1/3 um + 5/6 u0 - 1/6 up (plus) and -1/6 um + 5/6 u0 + 1/3 up
    # (minus).  The labels printed in eq. (8) would give -1/6 a + 7/6 b instead.
    a, b = 0.3, 1.1
    assert L.or1d_weno_plus(a, b, a) == pytest.approx(a / 3 + 5 * b / 6 - a / 6, rel=1e-14)
    assert L.or1d_weno_minus(a, b, a) == pytest.approx(-a / 6 + 5 * b / 6 + a / 3, rel=1e-14)


def test_weno_face_values_third_order_on_smooth_data():
    # cell averages of sin(x) over [0, 2 pi] shifted to avoid critical points dominating
    errs = []
    for n in (40, 80, 160, 320):
        dx = 2 * math.pi / n
        xf = np.arange(n + 1) * dx
        F = -np.cos(xf + 0.3)
        avg = (F[1:] - F[:-1]) / dx          # exact averages of sin(x + 0.3)
        e = 0.0
        for j in range(1, n - 1):
            up = L.or1d_weno_minus(avg[j - 1], avg[j], avg[j + 1])   # value at x_{j+1/2}
            e = max(e, abs(up - math.sin(xf[j + 1] + 0.3)))
        errs.append(e)
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert orders[-1] > 2.6, orders


# ---------------------------------------------------------------------------------------
# fluxes and source quadrature
# ---------------------------------------------------------------------------------------

def _hll(UL, UR, sig=1.0):
    F = np.empty(2)
    L.or1d_hll(oracle.ptr(np.array(UL, float)), oracle.ptr(np.array(UR, float)), sig, G,
               oracle.ptr(F))
    return F


def test_hll_consistency_and_upwinding():
    for H, Q, s in [(1.0, 0.5, 1.0), (2.0, 4.4, 1.0), (0.6, -0.3, 0.8), (0.4, 3.0, 1.2)]:
        h, u = H / s, Q / H
        phys = np.array([Q, Q * Q / H + 0.5 * G * s * h * h])
        assert np.allclose(_hll([H, Q], [H, Q], s), phys, rtol=1e-15, atol=0)
    # supercritical rightward states: the flux is the left physical flux
    UL, UR = [0.5, 3.0], [0.55, 3.1]
    hl = 0.5
    assert np.allclose(_hll(UL, UR), [3.0, 9.0 / 0.5 + 0.5 * G * hl * hl], rtol=1e-15)
    # mirror symmetry: reversing the flow and swapping the states negates the mass flux
    a = _hll([1.0, 0.4], [1.2, 0.3])
    b = _hll([1.2, -0.3], [1.0, -0.4])
    assert a[0] == pytest.approx(-b[0], rel=1e-14)
    assert a[1] == pytest.approx(b[1], rel=1e-14)


def test_cubic_gauss_weights_interpolate_cubics():
    W = np.empty(8)
    L.or1d_cubic_gauss_weights(oracle.ptr(W))
    W = W.reshape(2, 4)
    assert np.allclose(W.sum(axis=1), 1.0, atol=1e-15)
    nodes = np.array([-1.5, -0.5, 0.5, 1.5])
    tg = np.array([-1, 1]) / (2 * math.sqrt(3))
    for coeffs in ([1, 0, 0, 0], [0.3, -1.2, 0.7, 2.5], [0, 0, 0, 1]):
        p = np.polynomial.Polynomial(coeffs)
        assert np.allclose(W @ p(nodes), p(tg), rtol=1e-14, atol=1e-14)
    # closed form of the left-point weights
    r3 = math.sqrt(3)
    ref = [-1 / 24 - r3 / 216, 13 / 24 + 13 * r3 / 72, 13 / 24 - 13 * r3 / 72, -1 / 24 + r3 / 216]
    assert np.allclose(W[0], ref, rtol=1e-14)


def test_source_gauss_exact_for_linear_depth_and_slope():
    # H linear in x, constant width, b_x constant: -g h b_x is linear so the two-point rule
    # is exact: S_j = -g b_x h(x_j) dx.
    n, bx = 8, 0.3
    pr = _prob(n=n, bottom=lambda x: (bx * np.asarray(x), bx + 0 * np.asarray(x)))
    o = Oracle1D(pr)
    dx = pr.dx
    j = 3
    xj = pr.x0 + (j + 0.5) * dx
    h = lambda x: 1.0 + 0.4 * x
    Hf = np.array([h(xj + t * dx) for t in (-1.5, -0.5, 0.5, 1.5)])
    S = L.or1d_source(ctypes.byref(o.c), j, oracle.ptr(Hf))
    assert S == pytest.approx(-G * bx * h(xj) * dx, rel=1e-13)


# ---------------------------------------------------------------------------------------
# residual (eq. 10)
# ---------------------------------------------------------------------------------------

def test_residual_zero_for_constant_state_flat_bottom():
    for H, Q in [(1.0, 0.0), (2.0, 4.42), (0.5, 3.0)]:
        pr = _prob(n=32)
        U = np.stack([np.full(32, H), np.full(32, Q)])
        R, rn, res = Oracle1D(pr).residual(U)
        assert np.max(np.abs(R)) <= 1e-13 * (Q * Q / H + G * H * H)


def test_residual_mass_rows_telescope():
    # sum_j R^1_j = F^1_{N-1/2} - F^1_{-1/2}: perturbing cells far from both boundaries
    # leaves the sum unchanged (to round-off).
    rng = np.random.default_rng(5)
    n = 40
    pr = _prob(n=n, bottom=gaussian_bump(0.1, 0.5, 0.01), bcl=BC(BC_DISCHARGE, q=1.0),
               bcr=BC(BC_DEPTH, h=1.0))
    o = Oracle1D(pr)
    U = np.stack([1.0 + 0.1 * rng.random(n), 1.0 + 0.1 * rng.random(n)])
    s0 = o.residual(U)[0][0].sum()
    U2 = U.copy()
    U2[:, 5:n - 5] += 0.05 * rng.standard_normal((2, n - 10))
    s1 = o.residual(U2)[0][0].sum()
    assert abs(s1 - s0) < 1e-13


def test_residual_depends_on_five_cells_only():
    n = 24
    pr = _prob(n=n, bottom=gaussian_bump(0.1, 0.5, 0.02))
    o = Oracle1D(pr)
    rng = np.random.default_rng(1)
    U = np.stack([1.0 + 0.1 * rng.random(n), 0.5 + 0.1 * rng.random(n)])
    R0 = o.residual(U)[0]
    i = 12
    U2 = U.copy()
    U2[0, i] += 0.01
    d = np.abs(o.residual(U2)[0] - R0).max(axis=0)
    assert np.all(d[[j for j in range(n) if abs(j - i) > 2]] == 0.0)
    assert np.all(d[i - 2:i + 3] > 0.0)


def _exact_e1_u(x):
    b, _ = e1_bottom(x)
    u = np.ones_like(x)
    for _ in range(60):
        f = u ** 3 + (2 * G * b - 2 * G - 1) * u + 2 * G
        u = u - f / (3 * u ** 2 + (2 * G * b - 2 * G - 1))
    return u


def _cell_avg(f, x0, dx, n, npts=6):
    t, w = np.polynomial.legendre.leggauss(npts)
    xc = x0 + (np.arange(n) + 0.5) * dx
    return sum(wi * f(xc + ti * dx / 2) for ti, wi in zip(t, w)) / 2


def test_residual_truncation_order_on_exact_solution():
    # R on the exact cell averages of the smooth steady state of eq. (27) decays like dx^4
    # (R is not divided by dx) -- at least third order.
    errs = []
    for n in (96, 192, 384, 768):
        pr = e1_problem(n)
        hbar = _cell_avg(lambda x: 1.0 / _exact_e1_u(x), pr.x0, pr.dx, n)
        U = np.stack([hbar, np.ones(n)])
        errs.append(Oracle1D(pr).residual(U)[2])
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert min(orders[1:]) > 3.0, orders


# ---------------------------------------------------------------------------------------
# Jacobian (eq. 12-13, section 3.3)
# ---------------------------------------------------------------------------------------

def _analytic_const_jac(H, Q, alpha_rn=0.0):
    """Linearisation of R at a constant state on a flat bottom (closed form): the WENO weights
    are stationary there (their derivative multiplies a vanishing difference), so the face
    values are linear with weights -1/6, 5/6, 1/3 (minus) and 1/3, 5/6, -1/6 (plus), and the
    HLL flux linearises to dF/dUL = (SR A - SL SR I)/(SR - SL), dF/dUR = (-SL A + SL SR I)/(SR - SL)
    (or A / 0 when SL >= 0)."""
    h, u = H, Q / H
    c = math.sqrt(G * h)
    A = np.array([[0.0, 1.0], [-u * u + G * h, 2 * u]])
    SL, SR = u - c, u + c
    I = np.eye(2)
    if SL >= 0:
        dL, dR = A, 0 * A
    else:
        dL = (SR * A - SL * SR * I) / (SR - SL)
        dR = (-SL * A + SL * SR * I) / (SR - SL)
    wm = {-1: -1 / 6, 0: 5 / 6, 1: 1 / 3}    # U-_{k+1/2} from cell k: offsets k-1, k, k+1
    wp = {-1: 1 / 3, 0: 5 / 6, 1: -1 / 6}    # U+_{k-1/2} from cell k
    blocks = {}
    for off in range(-2, 3):
        B = np.zeros((2, 2))
        # face j+1/2: left state from cell j, right state from cell j+1
        B += dL * wm.get(off - 0, 0.0) + dR * wp.get(off - 1, 0.0)
        # face j-1/2: left state from cell j-1, right state from cell j
        B -= dL * wm.get(off + 1, 0.0) + dR * wp.get(off - 0, 0.0)
        blocks[off] = B
    return blocks


@pytest.mark.parametrize("H,Q", [(1.0, 0.4), (0.5, 3.0)])  # subcritical, supercritical
def test_jacobian_matches_closed_form_at_constant_state(H, Q):
    n = 12
    pr = _prob(n=n)
    o = Oracle1D(pr)
    U = np.stack([np.full(n, H), np.full(n, Q)])
    J = o.jacobian(U, eps=1e-7, alpha=3.0, nb=5)
    ref = _analytic_const_jac(H, Q)
    j = 6
    for b in range(5):
        assert np.allclose(J[j, b], ref[b - 2], atol=2e-6 * (1 + np.abs(ref[b - 2]).max())), (b, J[j, b], ref[b - 2])


def test_j3_is_j5_without_outer_blocks_and_regularisation():
    n = 16
    pr = _prob(n=n, bottom=gaussian_bump(0.1, 0.5, 0.02), bcl=BC(BC_DISCHARGE, q=1.0),
               bcr=BC(BC_DEPTH, h=1.0))
    o = Oracle1D(pr)
    rng = np.random.default_rng(3)
    U = np.stack([1.0 + 0.1 * rng.random(n), 1.0 + 0.1 * rng.random(n)])
    J3 = o.jacobian(U, eps=0.05, alpha=3.0, nb=3)
    J5 = o.jacobian(U, eps=0.05, alpha=3.0, nb=5)
    assert np.array_equal(J3, J5[:, 1:4])
    _, rn, _ = o.residual(U)
    J0 = o.jacobian(U, eps=0.05, alpha=0.0, nb=3)
    d = J3[:, 1] - J0[:, 1]
    assert np.allclose(d[:, 0, 0], 3.0 * rn, rtol=1e-12) and np.allclose(d[:, 1, 1], 3.0 * rn, rtol=1e-12)
    assert np.all(d[:, 0, 1] == 0) and np.all(d[:, 1, 0] == 0)


@pytest.mark.parametrize("bcl,bcr", [(BC(BC_DISCHARGE, q=1.0), BC(BC_DEPTH, h=1.0)),
                                     (BC(BC_WALL), BC(BC_EXTRAP))])
def test_jacobian_entries_equal_brute_force_global_fd(bcl, bcr):
    # Tiny grid: perturb the whole state vector through the public global residual and
    # difference every row; J3/J5 must hold exactly those entries where the stencil keeps them
    # (ghost-cell dependence included).
    n, eps = 8, 0.02
    pr = _prob(n=n, bottom=gaussian_bump(0.1, 0.5, 0.02), width=sine_width(1, 1.0, 0.1), bcl=bcl, bcr=bcr)
    o = Oracle1D(pr)
    rng = np.random.default_rng(11)
    U = np.stack([1.0 + 0.2 * rng.random(n), 0.6 + 0.2 * rng.random(n)])
    R0, _, _ = o.residual(U)
    dense = np.zeros((2 * n, 2 * n))
    for i in range(n):
        for m in range(2):
            Up = U.copy()
            Up[m, i] = U[m, i] + eps
            dense[:, 2 * i + m] = ((o.residual(Up)[0] - R0) / eps).T.reshape(-1)
    for nb in (3, 5):
        J = o.jacobian(U, eps=eps, alpha=0.0, nb=nb)
        A = blocks_to_dense(J)
        band = np.abs(np.subtract.outer(np.arange(2 * n) // 2, np.arange(2 * n) // 2)) <= nb // 2
        assert np.array_equal(A[band], dense[band])
        assert np.all(A[~band] == 0)
        if nb == 5:   # nothing outside the five-block band in the exact FD either
            assert np.all(dense[~band] == 0)


def test_jacobian_rows_equal_brute_force_global_fd():
    # The sampled-row form (for grids too large to difference every column) against the same
    # brute force through the public global residual, boundary rows included, and with the
    # regularisation bit for bit equal to the full form.
    n, eps = 12, 0.02
    pr = _prob(n=n, bottom=gaussian_bump(0.1, 0.5, 0.02), width=sine_width(1, 1.0, 0.1),
               bcl=BC(BC_DISCHARGE, q=1.0), bcr=BC(BC_WALL))
    o = Oracle1D(pr)
    rng = np.random.default_rng(12)
    U = np.stack([1.0 + 0.2 * rng.random(n), 0.6 + 0.2 * rng.random(n)])
    R0, _, _ = o.residual(U)
    rows = [0, 1, 2, 5, n - 3, n - 2, n - 1]
    for nb in (3, 5):
        Jr = o.jacobian_rows(U, rows, eps=eps, alpha=0.0, nb=nb)
        for k, j in enumerate(rows):
            for b in range(nb):
                i = j + b - nb // 2
                for m in range(2):
                    if not 0 <= i < n:
                        assert np.all(Jr[k, b, :, m] == 0)
                        continue
                    Up = U.copy()
                    Up[m, i] = U[m, i] + eps
                    col = (o.residual(Up)[0][:, j] - R0[:, j]) / eps
                    assert np.array_equal(Jr[k, b, :, m], col)
        Jfull = o.jacobian(U, eps=eps, alpha=0.7, nb=nb)
        assert np.array_equal(o.jacobian_rows(U, rows, eps=eps, alpha=0.7, nb=nb), Jfull[rows])


def test_block_magnitudes_on_e1_96():
    # Section 3.3: on the 96-cell smooth subcritical test, central tridiagonal blocks exceed 1,
    # outermost blocks are below 1, and about 69% of the outermost ones are below 1e-4.
    pr = e1_problem(96)
    o = Oracle1D(pr)
    U, it, res, _ = o.newton_solve()
    J = o.jacobian(U, nb=5)
    mag = np.abs(J).sum(axis=(2, 3))
    cen = np.concatenate([mag[:, 2], mag[1:, 1], mag[:-1, 3]])
    out = np.concatenate([mag[2:, 0], mag[:-2, 4]])
    assert cen.min() > 1.0
    assert out.max() < 1.0
    frac = np.mean(out < 1e-4)
    assert 0.4 < frac < 0.95, frac


# ---------------------------------------------------------------------------------------
# multigrid (section 3.4, eq. 15-19, Algorithm 2)
# ---------------------------------------------------------------------------------------

def _random_blocks(n, nb, rng, diag=6.0):
    J = rng.standard_normal((n, nb, 2, 2))
    hw = nb // 2
    for j in range(n):
        J[j, hw] += diag * np.eye(2)
        for b in range(nb):
            if not 0 <= j + b - hw < n:
                J[j, b] = 0.0
    return J


def _P(n):
    P = np.zeros((2 * n, n))   # injection of eq. (18), component-interleaved
    for j in range(n // 2):
        for k in (2 * j, 2 * j + 1):
            P[2 * k, 2 * j] = P[2 * k + 1, 2 * j + 1] = 1.0
    return P


@pytest.mark.parametrize("nb", [3, 5])
def test_coarse_operator_is_galerkin_with_injection(nb):
    rng = np.random.default_rng(2)
    n = 16
    J = _random_blocks(n, nb, rng)
    Jc = coarsen(J)
    P = _P(n)
    assert np.allclose(blocks_to_dense(Jc), P.T @ blocks_to_dense(J) @ P, rtol=1e-14, atol=1e-14)


def test_smoother_fixed_point_and_block_diagonal_exactness():
    rng = np.random.default_rng(4)
    n = 12
    for nb in (3, 5):
        J = _random_blocks(n, nb, rng)
        rhs = rng.standard_normal(2 * n)
        x = np.linalg.solve(blocks_to_dense(J), -rhs)
        for sm in (0, 1):
            y = smooth(J, rhs, x, steps=1, omega=1.3, smoother=sm).reshape(-1)
            assert np.allclose(y, x, rtol=1e-12, atol=1e-12)
    Jd = _random_blocks(n, 3, rng)
    Jd[:, 0] = 0
    Jd[:, 2] = 0
    rhs = rng.standard_normal(2 * n)
    y = smooth(Jd, rhs, None, steps=1, omega=1.0).reshape(-1)
    assert np.allclose(y, np.linalg.solve(blocks_to_dense(Jd), -rhs), rtol=1e-13)


def test_two_level_cycle_without_smoothing_is_exact_coarse_correction():
    rng = np.random.default_rng(6)
    n = 16
    J = _random_blocks(n, 3, rng)
    rhs = rng.standard_normal(2 * n)
    x0 = rng.standard_normal(2 * n)
    A = blocks_to_dense(J)
    P = _P(n)
    r = -rhs - A @ x0
    ref = x0 + P @ np.linalg.solve(P.T @ A @ P, P.T @ r)
    y = vcycles(J, rhs, x0, levels=2, ncycles=1, nu1=0, nu2=0).reshape(-1)
    assert np.allclose(y, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("nb,sm", [(3, 0), (5, 0), (3, 1)])
def test_vcycles_converge_to_dense_solve(nb, sm):
    rng = np.random.default_rng(7)
    n = 64
    J = _random_blocks(n, nb, rng, diag=8.0)
    rhs = rng.standard_normal(2 * n)
    x = np.linalg.solve(blocks_to_dense(J), -rhs)
    y = vcycles(J, rhs, None, levels=4, ncycles=30, omega=1.0, nu1=2, nu2=2, smoother=sm).reshape(-1)
    assert np.allclose(y, x, rtol=1e-10, atol=1e-10)


def test_coarsest_solve_matches_lapack():
    rng = np.random.default_rng(8)
    n = 10
    J = _random_blocks(n, 3, rng, diag=0.5)   # weak diagonal: needs pivoting
    rhs = rng.standard_normal(2 * n)
    y = vcycles(J, rhs, None, levels=1, ncycles=1).reshape(-1)
    assert np.allclose(y, np.linalg.solve(blocks_to_dense(J), -rhs), rtol=1e-12)


# ---------------------------------------------------------------------------------------
# Newton (Algorithm 1) and the paper's first experiment
# ---------------------------------------------------------------------------------------

def test_e1_orders_and_magnitudes_against_table1():
    """Table 1: third order under refinement.  Magnitudes: the h errors are 2.0-2.5 times the
    printed ones and the hu errors 1.4-1.8 times, at every grid; 70% of the h error sits at the
    bumps (|x| < 5), and prescribing the full state h = 1, hu = 1 in the ghosts of both ends
    instead changes the h errors by less than 6%, so the excess comes from the interior scheme
    the paper leaves open (HLL wave speeds), not the boundary reading.  The bands below hold the
    measured factors with a small margin."""
    rows = _table("e1_table1.txt")
    eh, eq = [], []
    for r in rows:
        n = int(r[0])
        pr = e1_problem(n)
        U, it, res, _ = Oracle1D(pr).newton_solve()
        assert res < 1e-11
        hbar = _cell_avg(lambda x: 1.0 / _exact_e1_u(x), pr.x0, pr.dx, n)
        eh.append(np.mean(np.abs(U[0] - hbar)))
        eq.append(np.mean(np.abs(U[1] - 1.0)))
        assert float(r[1]) / 1.5 < eh[-1] < float(r[1]) * 2.7, (n, eh[-1], r[1])
        assert float(r[3]) / 1.5 < eq[-1] < float(r[3]) * 2.0, (n, eq[-1], r[3])
    oh = [math.log2(eh[k] / eh[k + 1]) for k in range(3)]
    oq = [math.log2(eq[k] / eq[k + 1]) for k in range(3)]
    assert 2.7 < oh[-1] < 3.4 and 2.7 < oq[-1] < 3.6, (oh, oq)
    assert np.mean(oh) > 2.6 and np.mean(oq) > 2.6


def test_newton_counts_j3_equal_j5_on_e1():
    """Table 2: NMGM-3 and NMGM-5 take (nearly) the same number of Newton iterations."""
    for n in (96, 192):
        o = Oracle1D(e1_problem(n))
        _, it3, r3, _ = o.newton_solve(nb=3)
        _, it5, r5, _ = o.newton_solve(nb=5)
        assert r3 < 1e-11 and r5 < 1e-11
        assert abs(it3 - it5) <= max(2, 0.1 * it3), (n, it3, it5)


@pytest.mark.parametrize("i", [0, 1, 2])
def test_config1_discharge_and_bernoulli(i):
    """Smooth subcritical steady state: constant discharge and constant Bernoulli energy
    u^2/2 + g(h + b), both up to the discretisation error, which shrinks at third order."""
    pr = config1(i)
    o = Oracle1D(pr)
    U, it, res, hist = o.newton_solve()
    assert res < 1e-10 and it < 1000
    q = pr.meta["q"]
    assert np.max(np.abs(U[1] - q)) < 2e-3 * q
    x = pr.centres()
    b, _ = pr.bottom(x)
    h = U[0]
    E = (U[1] / h) ** 2 / 2 + G * (h + b)
    assert (E.max() - E.min()) / E.mean() < 2e-3
    # monotone decrease of the residual after the first few steps (linear contraction)
    assert hist[-1] < hist[len(hist) // 2] < hist[5]


def test_e1_invariants_converge_at_third_order():
    dq, dE = [], []
    for n in (192, 384, 768):
        pr = e1_problem(n)
        U, it, res, _ = Oracle1D(pr).newton_solve()
        dq.append(np.max(np.abs(U[1] - 1.0)))
        # energy through exact cell averages (comparing E of averages would show 2nd order)
        hbar = _cell_avg(lambda x: 1.0 / _exact_e1_u(x), pr.x0, pr.dx, n)
        dE.append(np.max(np.abs(U[0] - hbar)))
    assert math.log2(dq[1] / dq[2]) > 2.5 and math.log2(dE[1] / dE[2]) > 2.5


def test_lake_at_rest_roundoff_flat_and_third_order_otherwise():
    # flat bottom: the still state is an exact steady state of the scheme (round-off)
    n = 64
    pr = _prob(n=n, bcl=BC(BC_DISCHARGE, q=0.0), bcr=BC(BC_DEPTH, h=1.0))
    U = np.stack([np.ones(n), np.zeros(n)])
    assert Oracle1D(pr).residual(U)[2] < 1e-14
    # smooth non-flat bottom: the paper's scheme is not well-balanced; the still-water
    # residual is a truncation error that decays at least at third order
    rs = []
    for n in (64, 128, 256):
        pr = _prob(n=n, bottom=gaussian_bump(0.1, 0.5, 0.02), bcl=BC(BC_DISCHARGE, q=0.0),
                   bcr=BC(BC_DEPTH, h=1.0))
        xc = pr.centres()
        bbar = _cell_avg(lambda x: pr.bottom(x)[0], pr.x0, pr.dx, n)
        U = np.stack([1.0 - bbar, np.zeros(n)])
        rs.append(Oracle1D(pr).residual(U)[2])
    assert math.log2(rs[1] / rs[2]) > 3.0, rs


def test_source_width_term_exact_for_linear_width():
    # flat bottom, sigma linear, constant depth h: H = sigma h is linear (the cubic is exact)
    # and the source 1/2 g h^2 sigma_x is constant, so S_j = 1/2 g h^2 sigma_x dx exactly.
    n, sx, h = 8, 0.2, 2.0
    pr = _prob(n=n, width=lambda x: (1.0 + sx * np.asarray(x), sx + 0 * np.asarray(x)))
    o = Oracle1D(pr)
    dx, j = pr.dx, 5
    xj = pr.x0 + (j + 0.5) * dx
    Hf = np.array([(1.0 + sx * (xj + t * dx)) * h for t in (-1.5, -0.5, 0.5, 1.5)])
    S = L.or1d_source(ctypes.byref(o.c), j, oracle.ptr(Hf))
    assert S == pytest.approx(0.5 * G * h * h * sx * dx, rel=1e-13)


def test_still_water_in_varying_channel_converges():
    # Q = 0 and constant depth is an exact steady state of eq. (3) for any width on a flat
    # bottom: the residual of the scheme is a truncation error decaying at high order.
    rs = []
    for n in (64, 128, 256):
        pr = _prob(n=n, width=sine_width(1, 1.0, 0.2), bcl=BC(BC_WALL), bcr=BC(BC_WALL))
        xf = pr.x0 + np.arange(n + 1) * pr.dx
        F = np.array([-math.cos(2 * math.pi * x) / (2 * math.pi) for x in xf])
        sbar = 1.0 + 0.2 * (F[1:] - F[:-1]) / pr.dx     # exact cell averages of the width
        U = np.stack([2.0 * sbar, np.zeros(n)])
        R = Oracle1D(pr).residual(U)[0]
        rs.append(np.abs(R[:, 4:-4]).max())            # away from the walls
    assert math.log2(rs[0] / rs[1]) > 2.8 and math.log2(rs[1] / rs[2]) > 2.8, rs
