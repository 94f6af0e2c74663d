"""ctypes binding of the 2D oracle (``swe2d.c``) -- TEST INFRASTRUCTURE ONLY.

Geometry is sampled here at this oracle's own tensor Gauss points
(x_i -+ dx/(2 sqrt 3), y_j -+ dy/(2 sqrt 3)).
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

_dp = C.POINTER(C.c_double)


class OrProb2D(C.Structure):
    _fields_ = [("Nx", C.c_int), ("Ny", C.c_int), ("dx", C.c_double), ("dy", C.c_double),
                ("g", C.c_double), ("x0", C.c_double), ("y0", C.c_double),
                ("bx_gp", _dp), ("by_gp", _dp),
                ("bc_kind", C.c_int * 4), ("bc_q", C.c_double * 4), ("bc_h", C.c_double * 4),
                ("bc_u", C.c_double * 4), ("bc_v", C.c_double * 4), ("wall_x", C.c_double),
                ("recon", C.c_int), ("zavg", _dp), ("zfx", _dp), ("zfy", _dp)]


class OrParams2D(C.Structure):
    _fields_ = [("alpha", C.c_double), ("tau", C.c_double), ("eps", C.c_double),
                ("omega", C.c_double), ("tol", C.c_double),
                ("nu1", C.c_int), ("nu2", C.c_int), ("nu3", C.c_int), ("n_max", C.c_int),
                ("levels", C.c_int), ("stencil", C.c_int), ("smoother", C.c_int)]


def _declare(L):
    P = C.POINTER(OrProb2D)
    vp = C.c_void_p
    L.or2d_cell.argtypes = [P, _dp, C.c_int, C.c_int, _dp]
    L.or2d_local_residual.argtypes = [P, _dp, C.c_int, C.c_int, _dp]
    L.or2d_residual.argtypes = [P, _dp, _dp, _dp]
    L.or2d_residual.restype = C.c_double
    L.or2d_jacobian.argtypes = [P, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int, _dp]
    L.or2d_jacobian_rows.argtypes = [P, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                     C.c_int, _dp]
    L.or2d_face_state.argtypes = [P, _dp, C.c_int, C.c_int, C.c_int, C.c_int, _dp]
    L.or2d_llf.argtypes = [_dp, _dp, C.c_int, C.c_double, _dp]
    L.or2d_flux.argtypes = [_dp, C.c_int, C.c_double, _dp]
    L.or2d_eigen.argtypes = [_dp, C.c_int, C.c_double, _dp, _dp]
    L.or2d_newton_solve.argtypes = [P, C.POINTER(OrParams2D), _dp, _dp, C.c_int, _dp]
    L.or2d_interp_a3.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.or2d_newton_solve.restype = C.c_int
    L.or2d_vcycles.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, C.c_int,
                               C.c_double, C.c_int, C.c_int, C.c_int]
    L.or2d_smooth_only.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, C.c_int, C.c_double,
                                   C.c_int]
    L.or2d_mg_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
    L.or2d_mg_create.restype = vp
    L.or2d_mg_free.argtypes = [vp]
    L.or2d_mg_setup.argtypes = [vp, _dp]
    for nm in ("or2d_mg_level_J", "or2d_mg_level_rhs", "or2d_mg_level_dU"):
        getattr(L, nm).argtypes = [vp, C.c_int]
        getattr(L, nm).restype = _dp


def _ptr(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def stencil_offsets(which: int = 9):
    """Block order of the Jacobian: the cross of eq. (21), centre first; then the 12 cells of the
    full 21-cell stencil that the simplification drops."""
    off = [(0, 0), (-2, 0), (-1, 0), (1, 0), (2, 0), (0, -2), (0, -1), (0, 1), (0, 2)]
    if which == 21:
        for dj in (-1, 1):
            for di in (-2, -1, 1, 2):
                off.append((di, dj))
        for di in (-1, 1):
            for dj in (-2, 2):
                off.append((di, dj))
    return off


class Oracle2D:
    def __init__(self, prob):
        from . import lib
        self.L = lib()
        self.prob = prob
        nx, ny, dx, dy = prob.nx, prob.ny, prob.dx, prob.dy
        xc = prob.x0 + (np.arange(nx) + 0.5) * dx
        yc = prob.y0 + (np.arange(ny) + 0.5) * dy
        ox = dx / (2.0 * math.sqrt(3.0))
        oy = dy / (2.0 * math.sqrt(3.0))
        bx = np.empty((ny, nx, 2, 2))
        by = np.empty((ny, nx, 2, 2))
        for be, sy in enumerate((-oy, oy)):
            for ga, sx in enumerate((-ox, ox)):
                X, Y = np.meshgrid(xc + sx, yc + sy)
                _, gx, gy = prob.bottom(X, Y)
                bx[:, :, be, ga] = gx
                by[:, :, be, ga] = gy
        self.bx = np.ascontiguousarray(bx)
        self.by = np.ascontiguousarray(by)
        c = OrProb2D()
        c.Nx, c.Ny, c.dx, c.dy, c.g, c.x0, c.y0 = nx, ny, dx, dy, prob.g, prob.x0, prob.y0
        c.bx_gp = _ptr(self.bx)
        c.by_gp = _ptr(self.by)
        for k, bc in enumerate(prob.bc):
            c.bc_kind[k], c.bc_q[k], c.bc_h[k], c.bc_u[k], c.bc_v[k] = bc.kind, bc.q, bc.h, bc.u, bc.v
        c.wall_x = prob.wall_x
        c.recon = getattr(prob, "recon", 0)
        if c.recon == 1:
            from swe_workloads import bottom_samples_2d
            self.zavg, self.zfx, self.zfy = bottom_samples_2d(prob)
            c.zavg, c.zfx, c.zfy = _ptr(self.zavg), _ptr(self.zfx), _ptr(self.zfy)
        self.c = c
        self.nx, self.ny = nx, ny

    def residual(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.empty_like(U)
        rn = np.empty((self.ny, self.nx))
        res = self.L.or2d_residual(C.byref(self.c), _ptr(U), _ptr(R), _ptr(rn))
        return R, rn, res

    def local_residual(self, U, i, j):
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.empty(3)
        self.L.or2d_local_residual(C.byref(self.c), _ptr(U), i, j, _ptr(out))
        return out

    def cell(self, U, i, j):
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.empty(3)
        self.L.or2d_cell(C.byref(self.c), _ptr(U), i, j, _ptr(out))
        return out

    def jacobian(self, U, eps=None, alpha=None, which=9, rows=None, R=None, rn=None):
        """Blocks J[ny, nx, nb, 3, 3] (eq. 12-13, 21).  rows = (j0, j1) restricts the rows."""
        p = self.prob.params
        eps = p.eps if eps is None else eps
        alpha = p.alpha if alpha is None else alpha
        U = np.ascontiguousarray(U, dtype=np.float64)
        if R is None:
            R, rn, _ = self.residual(U)
        nb = len(stencil_offsets(which))
        J = np.zeros((self.ny, self.nx, nb, 3, 3))
        if rows is None:
            self.L.or2d_jacobian(C.byref(self.c), _ptr(U), _ptr(np.ascontiguousarray(R)),
                                 _ptr(np.ascontiguousarray(rn)), eps, alpha, which, _ptr(J))
        else:
            self.L.or2d_jacobian_rows(C.byref(self.c), _ptr(U), _ptr(np.ascontiguousarray(R)),
                                      _ptr(np.ascontiguousarray(rn)), eps, alpha, which, rows[0],
                                      rows[1], _ptr(J))
        return J

    def newton_solve(self, U0=None, which=9, smoother=0, levels=None, max_hist=100000, **over):
        p = self.prob.params
        pp = OrParams2D()
        vals = dict(alpha=p.alpha, tau=p.tau, eps=p.eps, omega=p.omega, tol=p.tol,
                    nu1=p.nu1, nu2=p.nu2, nu3=p.nu3, n_max=p.n_max)
        vals.update(over)
        for k, v in vals.items():
            setattr(pp, k, v)
        pp.levels = self.prob.levels if levels is None else levels
        pp.stencil = which
        pp.smoother = smoother
        U = np.ascontiguousarray(self.prob.initial_guess() if U0 is None else U0, dtype=np.float64).copy()
        hist = np.zeros(max_hist)
        res = C.c_double(0.0)
        it = self.L.or2d_newton_solve(C.byref(self.c), C.byref(pp), _ptr(U), _ptr(hist), max_hist,
                                      C.byref(res))
        return U, it, res.value, hist[:min(it, max_hist)].copy()


def blocks_to_dense2d(J, which=None):
    """Dense (3 n x 3 n) matrix of J[ny, nx, nb, 3, 3] (unknown (j*nx + i)*3 + c)."""
    ny, nx, nb = J.shape[:3]
    off = stencil_offsets(9 if nb == 9 else 21) if nb in (9, 21) else \
        [(0, 0), (-1, 0), (1, 0), (0, -1), (0, 1)]
    A = np.zeros((3 * nx * ny, 3 * nx * ny))
    for j in range(ny):
        for i in range(nx):
            for b, (di, dj) in enumerate(off):
                pi, pj = i + di, j + dj
                if 0 <= pi < nx and 0 <= pj < ny:
                    r = (j * nx + i) * 3
                    c = (pj * nx + pi) * 3
                    A[r:r + 3, c:c + 3] = J[j, i, b]
    return A


def vcycles2d(J, rhs, dU=None, levels=2, ncycles=1, omega=1.0, nu1=1, nu2=1, smoother=0):
    from . import lib
    L = lib()
    J = np.ascontiguousarray(J, dtype=np.float64)
    ny, nx, nb = J.shape[:3]
    which = 9 if nb == 9 else 21
    rhs = np.ascontiguousarray(np.asarray(rhs, dtype=np.float64).reshape(ny, nx, 3))
    dU = np.zeros((ny, nx, 3)) if dU is None else np.ascontiguousarray(dU, dtype=np.float64).reshape(ny, nx, 3).copy()
    L.or2d_vcycles(nx, ny, levels, which, _ptr(J), _ptr(rhs), _ptr(dU), ncycles, omega, nu1, nu2, smoother)
    return dU


def smooth2d(J, rhs, dU=None, iters=1, omega=1.0, smoother=0):
    from . import lib
    L = lib()
    J = np.ascontiguousarray(J, dtype=np.float64)
    ny, nx, nb = J.shape[:3]
    which = 9 if nb == 9 else 21
    rhs = np.ascontiguousarray(np.asarray(rhs, dtype=np.float64).reshape(ny, nx, 3))
    dU = np.zeros((ny, nx, 3)) if dU is None else np.ascontiguousarray(dU, dtype=np.float64).reshape(ny, nx, 3).copy()
    L.or2d_smooth_only(nx, ny, which, _ptr(J), _ptr(rhs), _ptr(dU), iters, omega, smoother)
    return dU


def coarse_operators(J, levels):
    """Five-point operators of levels 1..levels-1 built by the oracle from the fine J."""
    from . import lib
    L = lib()
    J = np.ascontiguousarray(J, dtype=np.float64)
    ny, nx, nb = J.shape[:3]
    which = 9 if nb == 9 else 21
    mg = L.or2d_mg_create(nx, ny, levels, which)
    L.or2d_mg_setup(mg, _ptr(J))
    out = []
    for l in range(1, levels):
        n = (nx >> l) * (ny >> l)
        a = np.ctypeslib.as_array(L.or2d_mg_level_J(mg, l), shape=(n * 5 * 9,))
        out.append(a.reshape(ny >> l, nx >> l, 5, 3, 3).copy())
    L.or2d_mg_free(mg)
    return out


def interp_a3(Uc: np.ndarray) -> np.ndarray:
    """Fine-grid cell averages [3, 2 ny, 2 nx] from a coarse state [3, ny, nx] (Appendix A,
    eq. A.3: the tensor product of eq. A.2, first along x, then along y)."""
    from . import lib
    Uc = np.ascontiguousarray(Uc, dtype=np.float64)
    _, ny, nx = Uc.shape
    if nx < 3 or ny < 3:
        raise ValueError("the interpolation needs at least three coarse cells in each direction")
    Uf = np.empty((3, 2 * ny, 2 * nx))
    lib().or2d_interp_a3(nx, ny, _ptr(Uc), _ptr(Uf))
    return Uf


def nested_solve2d(prob, ngrids=None, which=9, smoother=0, **over):
    """Algorithm 3 in two dimensions: Newton with the dense direct solve on the coarsest of the
    nested grids (a one-level hierarchy) from the problem's initial state there, then on each
    finer grid the Newton multigrid iteration with one more level, started from the eq. (A.3)
    interpolation of the coarser solution.  Returns (U on the finest grid, [(nx, ny, Newton
    steps, res) per grid, coarsest first])."""
    from swe_workloads import nested_grids_2d
    grids = nested_grids_2d(prob, ngrids)
    U = None
    report = []
    for g in range(len(grids) - 1, -1, -1):
        pg = grids[g]
        U0 = pg.initial_guess() if U is None else interp_a3(U)
        Ug, it, res, _ = Oracle2D(pg).newton_solve(U0=U0, which=which, smoother=smoother, **over)
        report.append((pg.nx, pg.ny, it, res))
        U = Ug
    return U, report
