"""CPU oracle for the Newton multigrid shallow-water path -- TEST INFRASTRUCTURE ONLY.

Plain FP64 C (``swe1d.c``, ``swe2d.c``) built with gcc ``-O2 -ffp-contract=off`` and driven
through ctypes.  Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg may import this package; the GPU library never does, and this package never
imports the GPU library.  Both take their problem descriptions from ``swe_workloads``.

Parity status: every exported function is pinned by ``tests/test_oracle_*.py`` against
closed forms, invariants, brute force or the paper's printed numbers, except where a
function's docstring says "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SRCS = [os.path.join(_HERE, "swe1d.c"), os.path.join(_HERE, "swe2d.c")]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math)."""
    srcs = [s for s in _SRCS if os.path.exists(s)]
    if force or not os.path.exists(_LIB) or any(
            os.path.getmtime(s) > os.path.getmtime(_LIB) for s in srcs):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-fopenmp", "-o", tmp] + srcs + ["-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or any(
                os.path.exists(s) and os.path.getmtime(s) > os.path.getmtime(_LIB) for s in _SRCS):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


_dp = C.POINTER(C.c_double)


class OrProb1D(C.Structure):
    _fields_ = [("N", C.c_int), ("dx", C.c_double), ("g", C.c_double),
                ("sig_face", _dp), ("sig_gp", _dp), ("sigx_gp", _dp), ("bx_gp", _dp),
                ("bc_kind", C.c_int * 2), ("bc_q", C.c_double * 2), ("bc_h", C.c_double * 2),
                ("recon", C.c_int), ("z_face", _dp), ("z_avg", _dp)]


class OrParams1D(C.Structure):
    _fields_ = [("alpha", C.c_double), ("tau", C.c_double), ("eps", C.c_double),
                ("omega", C.c_double), ("tol", C.c_double),
                ("nu1", C.c_int), ("nu2", C.c_int), ("nu3", C.c_int), ("n_max", C.c_int),
                ("levels", C.c_int), ("nb", C.c_int), ("smoother", C.c_int),
                ("linear", C.c_int), ("sor_max", C.c_int), ("sor_tol", C.c_double)]


def _declare(L):
    P = C.POINTER(OrProb1D)
    vp = C.c_void_p
    L.or1d_residual.argtypes = [P, _dp, _dp, _dp]
    L.or1d_residual.restype = C.c_double
    L.or1d_fill_ghosts.argtypes = [P, _dp, _dp]
    L.or1d_local_residual.argtypes = [P, _dp, C.c_int, _dp]
    L.or1d_jacobian.argtypes = [P, _dp, _dp, _dp, C.c_double, C.c_double, C.c_int, _dp]
    L.or1d_weno_plus.argtypes = [C.c_double] * 3
    L.or1d_weno_plus.restype = C.c_double
    L.or1d_weno_minus.argtypes = [C.c_double] * 3
    L.or1d_weno_minus.restype = C.c_double
    L.or1d_flux.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, _dp]
    L.or1d_hll.argtypes = [_dp, _dp, C.c_double, C.c_double, _dp]
    L.or1d_cubic_gauss_weights.argtypes = [_dp]
    L.or1d_source.argtypes = [P, C.c_int, _dp]
    L.or1d_source.restype = C.c_double
    L.or1d_coarsen.argtypes = [C.c_int, C.c_int, _dp, _dp]
    L.or1d_newton_solve.argtypes = [P, C.POINTER(OrParams1D), _dp, _dp, C.c_int, _dp]
    L.or1d_newton_solve.restype = C.c_int
    L.or1d_vcycles.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, C.c_int, C.c_double,
                               C.c_int, C.c_int, C.c_int]
    L.or1d_smooth_only.argtypes = [C.c_int, C.c_int, _dp, _dp, _dp, C.c_int, C.c_double, C.c_int]
    L.or1d_mg_create.argtypes = [C.c_int, C.c_int, C.c_int]
    L.or1d_mg_create.restype = vp
    L.or1d_mg_free.argtypes = [vp]
    L.or1d_mg_setup.argtypes = [vp, _dp]
    for nm in ("or1d_mg_level_J", "or1d_mg_level_Dinv", "or1d_mg_level_rhs", "or1d_mg_level_dU"):
        getattr(L, nm).argtypes = [vp, C.c_int]
        getattr(L, nm).restype = _dp
    L.or1d_smooth.argtypes = [vp, C.c_int, C.c_double, C.c_int]
    L.or1d_restrict.argtypes = [vp, C.c_int]
    L.or1d_prolong.argtypes = [vp, C.c_int]
    L.or1d_coarse_solve.argtypes = [vp, C.c_int]
    L.or1d_interp_a2.argtypes = [C.c_int, _dp, _dp]
    L.or1d_vcycle.argtypes = [vp, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int]
    if hasattr(L, "or2d_residual"):
        from . import swe2d as _s2
        _s2._declare(L)


def ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


# ----------------------------------------------------------------------------------------
# 1D problem binding: geometry sampled at this oracle's own Gauss points
# ----------------------------------------------------------------------------------------

class Oracle1D:
    """The oracle for one quasi-1D problem (``swe_workloads.Problem1D``)."""

    def __init__(self, prob):
        self.prob = prob
        n, dx = prob.n, prob.dx
        self.n = n
        # face x_{j-1/2}, j = 0..N
        xf = prob.x0 + np.arange(n + 1) * dx
        # Gauss points x_j -+ dx / (2 sqrt 3) (eq. 9)
        xc = prob.x0 + (np.arange(n) + 0.5) * dx
        off = dx / (2.0 * math.sqrt(3.0))
        xg = np.empty(2 * n)
        xg[0::2] = xc - off
        xg[1::2] = xc + off
        self.sig_face = np.ascontiguousarray(prob.width(xf)[0], dtype=np.float64)
        s, sx = prob.width(xg)
        _, bx = prob.bottom(xg)
        self.sig_gp = np.ascontiguousarray(s, dtype=np.float64)
        self.sigx_gp = np.ascontiguousarray(sx, dtype=np.float64)
        self.bx_gp = np.ascontiguousarray(bx, dtype=np.float64)
        c = OrProb1D()
        c.N = n
        c.dx = dx
        c.g = prob.g
        c.sig_face = ptr(self.sig_face)
        c.sig_gp = ptr(self.sig_gp)
        c.sigx_gp = ptr(self.sigx_gp)
        c.bx_gp = ptr(self.bx_gp)
        c.bc_kind[0], c.bc_kind[1] = prob.bc_left.kind, prob.bc_right.kind
        c.bc_q[0], c.bc_q[1] = prob.bc_left.q, prob.bc_right.q
        c.bc_h[0], c.bc_h[1] = prob.bc_left.h, prob.bc_right.h
        c.recon = getattr(prob, "recon", 0)
        if c.recon:
            from swe_workloads import bottom_faces_and_averages
            self.z_face, self.z_avg = bottom_faces_and_averages(prob)
            c.z_face = ptr(self.z_face)
            c.z_avg = ptr(self.z_avg)
        self.c = c
        lib()

    # -- residual -----------------------------------------------------------------------
    def residual(self, U: np.ndarray):
        """R[2, N], rn[N] = ||R_j||_1 and res = mean(rn) (eq. 10; Algorithm 1)."""
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.empty_like(U)
        rn = np.empty(self.n)
        res = lib().or1d_residual(C.byref(self.c), ptr(U), ptr(R), ptr(rn))
        return R, rn, res

    def ghosts(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        Ug = np.empty((self.n + 4) * 2)
        lib().or1d_fill_ghosts(C.byref(self.c), ptr(U), ptr(Ug))
        return Ug.reshape(self.n + 4, 2)

    def local_residual(self, Ug: np.ndarray, j: int):
        Ug = np.ascontiguousarray(Ug, dtype=np.float64).reshape(-1)
        out = np.empty(2)
        lib().or1d_local_residual(C.byref(self.c), ptr(Ug), j, ptr(out))
        return out

    # -- Jacobian -----------------------------------------------------------------------
    def jacobian(self, U, eps=None, alpha=None, nb=3, R=None, rn=None):
        """Blocks J[N, nb, 2, 2] of the regularised FD Jacobian (eq. 12-13)."""
        p = self.prob.params
        eps = p.eps if eps is None else eps
        alpha = p.alpha if alpha is None else alpha
        U = np.ascontiguousarray(U, dtype=np.float64)
        if R is None:
            R, rn, _ = self.residual(U)
        J = np.empty((self.n, nb, 2, 2))
        lib().or1d_jacobian(C.byref(self.c), ptr(U), ptr(np.ascontiguousarray(R)),
                            ptr(np.ascontiguousarray(rn)), eps, alpha, nb, ptr(J))
        return J

    def jacobian_rows(self, U, rows, eps=None, alpha=None, nb=3, R=None, rn=None):
        """Blocks J[len(rows), nb, 2, 2] of the rows `rows` only (eq. 12-13): each column
        (i, m) of a row is the forward difference of that row's local residual under the
        perturbation of component m of cell i, with the ghosts refilled from the perturbed
        state, plus alpha ||R_j||_1 on the diagonal block.  The same arithmetic as
        ``jacobian`` (which differences every column of the grid), for grids too large for it."""
        p = self.prob.params
        eps = p.eps if eps is None else eps
        alpha = p.alpha if alpha is None else alpha
        U = np.ascontiguousarray(U, dtype=np.float64)
        if R is None:
            R, rn, _ = self.residual(U)
        hw = nb // 2
        out = np.zeros((len(rows), nb, 2, 2))
        for k, j in enumerate(rows):
            for b in range(nb):
                i = j + b - hw
                if i < 0 or i >= self.n:
                    continue
                for m in range(2):
                    Up = U.copy()
                    Up[m, i] = Up[m, i] + eps
                    Rp = self.local_residual(self.ghosts(Up), j)
                    for l in range(2):
                        out[k, b, l, m] = (Rp[l] - R[l, j]) / eps
            for l in range(2):
                out[k, hw, l, l] += alpha * rn[j]
        return out

    # -- Newton ---------------------------------------------------------------------------
    def newton_solve(self, U0=None, nb=3, smoother=0, levels=None, max_hist=100000, **over):
        """Algorithm 1 with nu3 V-cycles per step.  Returns (U, iterations, res, history)."""
        p = self.prob.params
        pp = OrParams1D()
        vals = dict(alpha=p.alpha, tau=p.tau, eps=p.eps, omega=p.omega, tol=p.tol,
                    nu1=p.nu1, nu2=p.nu2, nu3=p.nu3, n_max=p.n_max)
        vals.update(over)
        for k, v in vals.items():
            setattr(pp, k, v)
        pp.levels = self.prob.levels if levels is None else levels
        pp.nb = nb
        pp.smoother = smoother
        U = np.ascontiguousarray(self.prob.initial_guess() if U0 is None else U0,
                                 dtype=np.float64).copy()
        hist = np.zeros(max_hist)
        res = C.c_double(0.0)
        it = lib().or1d_newton_solve(C.byref(self.c), C.byref(pp), ptr(U), ptr(hist), max_hist,
                                     C.byref(res))
        return U, it, res.value, hist[:min(it, max_hist)].copy()


# ----------------------------------------------------------------------------------------
# multigrid helpers on explicit operators (level equation: sum_i J_ji dU_i = -rhs_j)
# ----------------------------------------------------------------------------------------

def coarsen(Jf: np.ndarray) -> np.ndarray:
    """eq. (17) operator part: fine blocks [n, nb, 2, 2] -> coarse [n/2, 3, 2, 2]."""
    Jf = np.ascontiguousarray(Jf, dtype=np.float64)
    n, nb = Jf.shape[0], Jf.shape[1]
    Jc = np.empty((n // 2, 3, 2, 2))
    lib().or1d_coarsen(n, nb, ptr(Jf), ptr(Jc))
    return Jc


def vcycles(J, rhs, dU=None, levels=2, ncycles=1, omega=1.0, nu1=2, nu2=2, smoother=0):
    J = np.ascontiguousarray(J, dtype=np.float64)
    n, nb = J.shape[0], J.shape[1]
    rhs = np.ascontiguousarray(np.asarray(rhs, dtype=np.float64).reshape(n, 2))
    dU = np.zeros((n, 2)) if dU is None else np.ascontiguousarray(dU, dtype=np.float64).reshape(n, 2).copy()
    lib().or1d_vcycles(n, levels, nb, ptr(J), ptr(rhs), ptr(dU), ncycles, omega, nu1, nu2, smoother)
    return dU


def smooth(J, rhs, dU=None, steps=1, omega=1.0, smoother=0):
    J = np.ascontiguousarray(J, dtype=np.float64)
    n, nb = J.shape[0], J.shape[1]
    rhs = np.ascontiguousarray(np.asarray(rhs, dtype=np.float64).reshape(n, 2))
    dU = np.zeros((n, 2)) if dU is None else np.ascontiguousarray(dU, dtype=np.float64).reshape(n, 2).copy()
    lib().or1d_smooth_only(n, nb, ptr(J), ptr(rhs), ptr(dU), steps, omega, smoother)
    return dU


def blocks_to_dense(J: np.ndarray) -> np.ndarray:
    """Dense (2n x 2n) matrix of block rows J[n, nb, 2, 2]."""
    n, nb = J.shape[0], J.shape[1]
    hw = nb // 2
    A = np.zeros((2 * n, 2 * n))
    for j in range(n):
        for b in range(nb):
            i = j + b - hw
            if 0 <= i < n:
                A[2 * j:2 * j + 2, 2 * i:2 * i + 2] = J[j, b]
    return A


def interp_a2(Uc: np.ndarray) -> np.ndarray:
    """Fine-grid cell averages from a coarse solution [2, nc] (Appendix A, eq. A.1-A.2)."""
    Uc = np.ascontiguousarray(Uc, dtype=np.float64)
    nc = Uc.shape[1]
    if nc < 3:
        raise ValueError("the interpolation needs at least three coarse cells")
    Uf = np.empty((2, 2 * nc))
    lib().or1d_interp_a2(nc, ptr(Uc), ptr(Uf))
    return Uf


def nested_solve(prob, ngrids=None, U0=None, nb=3, **over):
    """Algorithm 3: Newton with a direct linear solve on the coarsest grid (N / 2^(ngrids-1)
    cells) from the problem's initial guess there, then on each finer grid l the Newton
    multigrid iteration with ngrids - l levels from the Appendix A interpolation of the coarser
    solution.  Returns (U on the finest grid, [(cells, Newton steps, res) per grid, coarsest
    first])."""
    from swe_workloads import nested_grids
    grids = nested_grids(prob, ngrids)
    ng = len(grids)
    U = grids[-1].initial_guess() if U0 is None else np.ascontiguousarray(U0, dtype=np.float64)
    report = []
    for g in range(ng - 1, -1, -1):
        if g < ng - 1:
            U = interp_a2(U)
        Ug, it, res, _ = Oracle1D(grids[g]).newton_solve(U0=U, nb=nb, levels=ng - g, **over)
        report.append((grids[g].n, it, res))
        U = Ug
    return U, report
