"""Python binding of libnmg: marshals problems and torch device tensors into the C ABI.

Every step of the solver runs in the HIP library; this module only samples the problem's
geometry at the points the discretisation uses, allocates device memory through torch and
passes pointers and the current stream.
"""
from __future__ import annotations

import ctypes as C
import math
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi as A


def _stream_ptr() -> int:
    return torch.cuda.current_stream().cuda_stream


def _dptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def params_struct(p, precision: int = A.NMG_FP64, check_every: int = 4) -> A.nmg_params:
    s = A.nmg_params()
    s.alpha, s.tau, s.eps, s.omega, s.tol = p.alpha, p.tau, p.eps, p.omega, p.tol
    s.nu1, s.nu2, s.nu3, s.n_max = p.nu1, p.nu2, p.nu3, p.n_max
    s.precision = precision
    s.check_every = check_every
    s.linear = getattr(p, "linear", A.NMG_LINEAR_MG)
    s.sor_max = getattr(p, "sor_max", 10)
    s.sor_tol = getattr(p, "sor_tol", 1e-7)
    s.schedule = getattr(p, "schedule", 0)
    return s


class Problem1DDevice:
    """Device-resident description of one quasi-1D problem (eq. 3-4): geometry sampled at the
    faces and at the two Gauss points x_j -/+ dx/(2 sqrt 3) of each cell (eq. 9)."""

    def __init__(self, prob, device="cuda", jac: int = 3):
        self.prob = prob
        n, dx = prob.n, prob.dx
        xf = prob.x0 + np.arange(n + 1) * dx
        xc = prob.x0 + (np.arange(n) + 0.5) * dx
        off = dx / (2.0 * math.sqrt(3.0))
        xg = np.empty(2 * n)
        xg[0::2] = xc - off
        xg[1::2] = xc + off
        s, sx = prob.width(xg)
        _, bx = prob.bottom(xg)
        f64 = dict(dtype=torch.float64, device=device)
        self.sig_face = torch.tensor(np.ascontiguousarray(prob.width(xf)[0]), **f64)
        self.sig_gp = torch.tensor(np.ascontiguousarray(s), **f64)
        self.sigx_gp = torch.tensor(np.ascontiguousarray(sx), **f64)
        self.bx_gp = torch.tensor(np.ascontiguousarray(bx), **f64)
        d = A.nmg_desc()
        d.dim, d.nx, d.ny, d.levels, d.jac = 1, n, 1, prob.levels, jac
        d.x0, d.x1, d.y0, d.y1, d.g = prob.x0, prob.x1, 0.0, 1.0, prob.g
        for k, bc in enumerate((prob.bc_left, prob.bc_right)):
            d.bc[k].kind, d.bc[k].q, d.bc[k].h = bc.kind, bc.q, bc.h
        d.sig_face = self.sig_face.data_ptr()
        d.sig_gp = self.sig_gp.data_ptr()
        d.sigx_gp = self.sigx_gp.data_ptr()
        d.bx_gp = self.bx_gp.data_ptr()
        d.recon = getattr(prob, "recon", A.NMG_RECON_CONSERVED)
        if d.recon == A.NMG_RECON_SURFACE:
            from swe_workloads import bottom_faces_and_averages
            zf, za = bottom_faces_and_averages(prob)
            self.z_face = torch.tensor(zf, **f64)
            self.z_avg = torch.tensor(za, **f64)
            d.z_face = self.z_face.data_ptr()
            d.z_avg = self.z_avg.data_ptr()
        self.desc = d
        self.n = n
        self.device = device

    def with_jac(self, jac: int) -> "Problem1DDevice":
        self.desc.jac = jac
        return self


class Solver1D:
    """Single-instance entry points of the C ABI for one problem."""

    def __init__(self, prob, device="cuda", jac: int = 3, precision: int = A.NMG_FP64,
                 check_every: int = 4, **param_overrides):
        A.load()
        self.dev = Problem1DDevice(prob, device, jac)
        p = prob.params
        if param_overrides:
            import dataclasses
            p = dataclasses.replace(p, **param_overrides)
        self.p = p
        self.params = params_struct(p, precision, check_every)
        self.precision = precision
        self.n = prob.n
        self.jac = jac
        self.device = device
        self._ws = None

    @property
    def L(self):
        return A.load()

    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            nbytes = self.L.nmg_workspace_bytes(C.byref(self.dev.desc), C.byref(self.params))
            if nbytes == 0:
                raise A.NmgError(A.NMG_EINVAL, self.L.nmg_last_error().decode())
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def state(self, U=None) -> torch.Tensor:
        U = self.dev.prob.initial_guess() if U is None else U
        if isinstance(U, torch.Tensor):
            return U.to(device=self.device, dtype=torch.float64).contiguous().clone()
        return torch.tensor(np.ascontiguousarray(U), dtype=torch.float64, device=self.device)

    def residual(self, U: torch.Tensor):
        """R [2, N], rn [N], res (0-d tensor) on the device (eq. 10, Algorithm 1)."""
        R = torch.empty_like(U)
        rn = torch.empty(self.n, dtype=torch.float64, device=self.device)
        res = torch.empty((), dtype=torch.float64, device=self.device)
        A.check(self.L.nmg_residual(C.byref(self.dev.desc), _dptr(U), _dptr(R), _dptr(rn),
                                    _dptr(res), C.c_void_p(_stream_ptr())))
        return R, rn, res

    def jacobian(self, U, R, rn) -> torch.Tensor:
        """Blocks J [nb, 2, 2, N] (eq. 12-13) on the device."""
        J = torch.empty((self.jac, 2, 2, self.n), dtype=torch.float64, device=self.device)
        A.check(self.L.nmg_jacobian_assemble_simplified(
            C.byref(self.dev.desc), C.byref(self.params), _dptr(U), _dptr(R), _dptr(rn), _dptr(J),
            C.c_void_p(_stream_ptr())))
        return J

    def vcycle(self, J: Optional[torch.Tensor], rhs: torch.Tensor, dU: torch.Tensor, setup: bool):
        """One V-cycle for sum_i J_ji dU_i = -rhs_j; dU is updated in place."""
        ws = self.workspace()
        A.check(self.L.nmg_mg_vcycle(C.byref(self.dev.desc), C.byref(self.params), _dptr(ws),
                                     ws.numel(), _dptr(J) if J is not None else None, _dptr(rhs),
                                     _dptr(dU), 1 if setup else 0, C.c_void_p(_stream_ptr())))
        return dU

    def newton_solve(self, U: torch.Tensor, max_hist: int = 0):
        """Algorithm 1 in place on U.  Returns (stats, history ndarray)."""
        ws = self.workspace()
        st = A.nmg_stats()
        hist = (C.c_double * max(1, max_hist))()
        status = self.L.nmg_newton_solve(C.byref(self.dev.desc), C.byref(self.params), _dptr(ws),
                                         ws.numel(), _dptr(U), C.byref(st),
                                         hist if max_hist > 0 else None, max_hist,
                                         C.c_void_p(_stream_ptr()))
        A.check(status, ok=(A.NMG_OK, A.NMG_NOT_CONVERGED, A.NMG_ENONFINITE))
        h = np.array(hist[:min(max_hist, st.iters)]) if max_hist > 0 else np.zeros(0)
        return st, h


class BatchSolver1D:
    """Many independent 1D problems solved together (one launch per kernel per step)."""

    def __init__(self, probs: Sequence, device="cuda", jac: int = 3, precision: int = A.NMG_FP64,
                 check_every: int = 4, jacs: Optional[Sequence[int]] = None,
                 devs: Optional[Sequence[Problem1DDevice]] = None):
        A.load()
        if devs is None:
            devs = [Problem1DDevice(p, device, (jacs[k] if jacs else jac)) for k, p in enumerate(probs)]
        self.devs = list(devs)
        self.probs = list(probs)
        n = len(probs)
        self.descs = (A.nmg_desc * n)(*[d.desc for d in self.devs])
        self.params = (A.nmg_params * n)(*[params_struct(p.params, precision, check_every) for p in probs])
        self.device = device
        self.n = n
        self.plan = C.c_void_p()
        A.check(A.load().nmg_plan_create(self.descs, self.params, n, C.byref(self.plan)))
        self.ws_bytes = A.load().nmg_plan_workspace_bytes(self.plan)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def __del__(self):
        try:
            if self.plan:
                A.load().nmg_plan_destroy(self.plan)
        except Exception:
            pass

    def states(self, Us=None) -> List[torch.Tensor]:
        out = []
        for k, p in enumerate(self.probs):
            U = p.initial_guess() if Us is None else Us[k]
            out.append(torch.tensor(np.ascontiguousarray(U), dtype=torch.float64, device=self.device)
                       if not isinstance(U, torch.Tensor) else U)
        return out

    def solve(self, Us: List[torch.Tensor], use_graph: bool = True):
        ptrs = (C.c_void_p * self.n)(*[u.data_ptr() for u in Us])
        stats = (A.nmg_stats * self.n)()
        st = A.load().nmg_plan_solve(self.plan, _dptr(self.ws), self.ws_bytes, ptrs, stats,
                                     1 if use_graph else 0, C.c_void_p(_stream_ptr()))
        A.check(st, ok=(A.NMG_OK, A.NMG_NOT_CONVERGED, A.NMG_ENONFINITE))
        return [(s.iters, s.status, s.res) for s in stats]

    def begin(self, Us: List[torch.Tensor]):
        self._ptrs = (C.c_void_p * self.n)(*[u.data_ptr() for u in Us])
        A.check(A.load().nmg_plan_begin(self.plan, _dptr(self.ws), self.ws_bytes, self._ptrs,
                                        C.c_void_p(_stream_ptr())))

    def resume(self, Us: List[torch.Tensor], n_done: Sequence[int]):
        """Begin on states that have already taken n_done[k] Newton steps under another plan."""
        self._ptrs = (C.c_void_p * self.n)(*[u.data_ptr() for u in Us])
        counts = (C.c_int32 * self.n)(*[int(v) for v in n_done])
        A.check(A.load().nmg_plan_resume(self.plan, _dptr(self.ws), self.ws_bytes, self._ptrs, counts,
                                         C.c_void_p(_stream_ptr())))

    def set_options(self, bottom_cells: int, smooth_tile: int = 0, split_finest: int = 0,
                    split_residual: int = 0):
        opt = A.nmg_plan_options()
        opt.bottom_cells = bottom_cells
        opt.smooth_tile = smooth_tile
        opt.split_finest = split_finest
        opt.split_residual = split_residual
        A.check(A.load().nmg_plan_set_options(self.plan, C.byref(opt)))

    @staticmethod
    def _opt_dict(opt) -> dict:
        return {"bottom_cells": opt.bottom_cells, "smooth_tile": opt.smooth_tile,
                "split_finest": opt.split_finest, "fused_finest": bool(opt.fused_finest),
                "split_residual": opt.split_residual}

    def options(self) -> dict:
        opt = A.nmg_plan_options()
        A.check(A.load().nmg_plan_get_options(self.plan, C.byref(opt)))
        return self._opt_dict(opt)

    @staticmethod
    def tune_candidate(c: int) -> tuple:
        """(bottom_cells, split_finest, smooth_tile, split_residual) of autotuner candidate c."""
        return 256 << (c % 4), (c // 4) % 2, 256 << ((c // 8) % 2), c // 16

    def autotune(self, Us: List[torch.Tensor], trial_steps: int = 3, use_graph: bool = True):
        """Time every candidate option set on these states (restored afterwards), keep the
        fastest.  Returns (best options, {(bottom_cells, split_finest, smooth_tile, split_residual): ms per
        Newton step})."""
        ptrs = (C.c_void_p * self.n)(*[u.data_ptr() for u in Us])
        best = A.nmg_plan_options()
        times = (C.c_double * A.NMG_TUNE_CANDIDATES)()
        A.check(A.load().nmg_plan_autotune(self.plan, _dptr(self.ws), self.ws_bytes, ptrs, trial_steps,
                                           1 if use_graph else 0, C.byref(best), times,
                                           C.c_void_p(_stream_ptr())))
        return (self._opt_dict(best),
                {self.tune_candidate(c): times[c] for c in range(A.NMG_TUNE_CANDIDATES)})

    def profile(self, kernel: int):
        """Time every later non-graph launch of one kernel (NMG_K_*) with HIP events."""
        A.check(A.load().nmg_plan_profile(self.plan, kernel))

    def profile_read(self):
        """(milliseconds, launches) accumulated since the last read."""
        ms = C.c_double()
        cnt = C.c_int32()
        A.check(A.load().nmg_plan_profile_read(self.plan, C.byref(ms), C.byref(cnt)))
        return ms.value, cnt.value

    def steps(self, k: int, use_graph: bool = True):
        active = (C.c_int32 * self.n)()
        stats = (A.nmg_stats * self.n)()
        A.check(A.load().nmg_plan_steps(self.plan, _dptr(self.ws), k, 1 if use_graph else 0, active,
                                        stats, C.c_void_p(_stream_ptr())))
        return list(active), [(s.iters, s.status, s.res) for s in stats]


class Problem2DDevice:
    """Device-resident description of one 2D problem (eq. 1-2): b_x and b_y sampled at the
    tensor Gauss points (x_i -/+ dx/(2 sqrt 3), y_j -/+ dy/(2 sqrt 3)) of every cell, stored
    [ny][nx][y point][x point]."""

    def __init__(self, prob, device="cuda", jac: int = 9):
        self.prob = prob
        nx, ny, dx, dy = prob.nx, prob.ny, prob.dx, prob.dy
        gx = dx / (2.0 * math.sqrt(3.0))
        gy = dy / (2.0 * math.sqrt(3.0))
        xc = prob.x0 + (np.arange(nx) + 0.5) * dx
        yc = prob.y0 + (np.arange(ny) + 0.5) * dy
        bx = np.empty((ny, nx, 2, 2))
        by = np.empty((ny, nx, 2, 2))
        for b, sy in ((0, -gy), (1, gy)):
            for a, sx in ((0, -gx), (1, gx)):
                X = np.ascontiguousarray(np.broadcast_to((xc + sx)[None, :], (ny, nx)))
                Y = np.ascontiguousarray(np.broadcast_to((yc + sy)[:, None], (ny, nx)))
                _, dbx, dby = prob.bottom(X, Y)
                bx[:, :, b, a] = dbx
                by[:, :, b, a] = dby
        f64 = dict(dtype=torch.float64, device=device)
        self.bx_gp = torch.tensor(np.ascontiguousarray(bx), **f64)
        self.by_gp = torch.tensor(np.ascontiguousarray(by), **f64)
        d = A.nmg_desc()
        d.dim, d.nx, d.ny, d.levels, d.jac = 2, nx, ny, prob.levels, jac
        d.x0, d.x1, d.y0, d.y1, d.g = prob.x0, prob.x1, prob.y0, prob.y1, prob.g
        for k, bc in enumerate(prob.bc):
            d.bc[k].kind, d.bc[k].q, d.bc[k].h, d.bc[k].u, d.bc[k].v = bc.kind, bc.q, bc.h, bc.u, bc.v
        d.wall_x = prob.wall_x
        d.bx_gp = self.bx_gp.data_ptr()
        d.by_gp = self.by_gp.data_ptr()
        d.recon = getattr(prob, "recon", 0)
        if d.recon == A.NMG_RECON_SURFACE:
            from swe_workloads import bottom_samples_2d
            za, zfx, zfy = bottom_samples_2d(prob)
            self.z_avg = torch.tensor(za, **f64)
            self.z_face = torch.tensor(np.concatenate([zfx.ravel(), zfy.ravel()]), **f64)
            d.z_avg = self.z_avg.data_ptr()
            d.z_face = self.z_face.data_ptr()
        self.desc = d
        self.device = device


class Solver2D:
    """Single-instance entry points of the C ABI for one 2D problem (state [3, ny, nx])."""

    def __init__(self, prob, device="cuda", precision: int = A.NMG_FP64, check_every: int = 4,
                 levels: Optional[int] = None, jac: int = 9, **param_overrides):
        A.load()
        self.dev = Problem2DDevice(prob, device, jac)
        self.nb = jac
        if levels is not None:
            self.dev.desc.levels = levels
        p = prob.params
        if param_overrides:
            import dataclasses
            p = dataclasses.replace(p, **param_overrides)
        self.p = p
        self.params = params_struct(p, precision, check_every)
        self.precision = precision
        self.nx, self.ny = prob.nx, prob.ny
        self.device = device
        self._ws = None

    @property
    def L(self):
        return A.load()

    def workspace(self) -> torch.Tensor:
        if self._ws is None:
            nbytes = self.L.nmg_workspace_bytes(C.byref(self.dev.desc), C.byref(self.params))
            if nbytes == 0:
                raise A.NmgError(A.NMG_EINVAL, self.L.nmg_last_error().decode())
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self._ws

    def state(self, U=None) -> torch.Tensor:
        U = self.dev.prob.initial_guess() if U is None else U
        if isinstance(U, torch.Tensor):
            return U.to(device=self.device, dtype=torch.float64).contiguous().clone()
        return torch.tensor(np.ascontiguousarray(U), dtype=torch.float64, device=self.device)

    def residual(self, U: torch.Tensor):
        """R [3, ny, nx], rn [ny, nx], res (0-d tensor) on the device (eq. 20, Algorithm 1)."""
        R = torch.empty_like(U)
        rn = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
        res = torch.empty((), dtype=torch.float64, device=self.device)
        A.check(self.L.nmg_residual(C.byref(self.dev.desc), _dptr(U), _dptr(R), _dptr(rn),
                                    _dptr(res), C.c_void_p(_stream_ptr())))
        return R, rn, res

    def jacobian(self, U, R, rn) -> torch.Tensor:
        """Blocks J [nb, 3, 3, ny, nx] (eq. 12-13, 21; nb = 9 or 21) on the device."""
        J = torch.empty((self.nb, 3, 3, self.ny, self.nx), dtype=torch.float64, device=self.device)
        A.check(self.L.nmg_jacobian_assemble_simplified(
            C.byref(self.dev.desc), C.byref(self.params), _dptr(U), _dptr(R), _dptr(rn), _dptr(J),
            C.c_void_p(_stream_ptr())))
        return J

    def vcycle(self, J: Optional[torch.Tensor], rhs: torch.Tensor, dU: torch.Tensor, setup: bool):
        """One V-cycle for sum J dU = -rhs (rhs, dU [3, ny, nx]); dU is updated in place."""
        ws = self.workspace()
        A.check(self.L.nmg_mg_vcycle(C.byref(self.dev.desc), C.byref(self.params), _dptr(ws),
                                     ws.numel(), _dptr(J) if J is not None else None, _dptr(rhs),
                                     _dptr(dU), 1 if setup else 0, C.c_void_p(_stream_ptr())))
        return dU

    def autotune(self, J: torch.Tensor, rhs: torch.Tensor, cycles: int = 2):
        """Time one V-cycle under every 2D launch schedule (nmg_autotune2d) on this operator;
        returns (the fastest schedule, {schedule: ms per V-cycle}).  Pass the schedule as
        schedule=... to later solvers of this problem (results are the same under every one)."""
        ws = self.workspace()
        best = C.c_int32()
        ms = (C.c_double * A.NMG_TUNE2D_CANDIDATES)()
        A.check(self.L.nmg_autotune2d(C.byref(self.dev.desc), C.byref(self.params), _dptr(ws), ws.numel(),
                                      _dptr(J), _dptr(rhs), cycles, C.byref(best), ms, C.c_void_p(_stream_ptr())))
        return best.value, {c: ms[c] for c in range(A.NMG_TUNE2D_CANDIDATES)}

    def newton_solve(self, U: torch.Tensor, max_hist: int = 0):
        """Algorithm 1 in place on U.  Returns (stats, history ndarray)."""
        ws = self.workspace()
        st = A.nmg_stats()
        hist = (C.c_double * max(1, max_hist))()
        status = self.L.nmg_newton_solve(C.byref(self.dev.desc), C.byref(self.params), _dptr(ws),
                                         ws.numel(), _dptr(U), C.byref(st),
                                         hist if max_hist > 0 else None, max_hist,
                                         C.c_void_p(_stream_ptr()))
        A.check(status, ok=(A.NMG_OK, A.NMG_NOT_CONVERGED, A.NMG_ENONFINITE))
        h = np.array(hist[:min(max_hist, st.iters)]) if max_hist > 0 else np.zeros(0)
        return st, h


class Stepper2D:
    """Algorithm 1 for one 2D problem in pieces on a stream of the caller (nmg_newton2d_begin,
    nmg_newton2d_steps): the state and the workspace stay on the device, each chunk of Newton
    steps ends with a copy of the Newton state into pinned host memory and an event, so the
    caller can poll instead of waiting.  The arithmetic is nmg_newton_solve's."""

    def __init__(self, prob, device="cuda", precision: int = A.NMG_FP32_MG, stream=None, jac: int = 9,
                 **param_overrides):
        self.solver = Solver2D(prob, device=device, precision=precision, jac=jac, **param_overrides)
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        self.U = self.solver.state()
        self.ws = self.solver.workspace()
        self._host = torch.zeros(C.sizeof(A.nmg_newton_state), dtype=torch.uint8).pin_memory()
        self.event = None

    def _call(self, fn, *args):
        d = self.solver.dev.desc
        A.check(fn(C.byref(d), C.byref(self.solver.params), _dptr(self.ws), self.ws.numel(),
                   _dptr(self.U), *args, C.c_void_p(self.stream.cuda_stream)))

    def begin(self):
        # the state and geometry were written on the current stream
        self.stream.wait_stream(torch.cuda.current_stream(self.U.device))
        self._call(A.load().nmg_newton2d_begin)

    def launch(self, steps: int):
        """Enqueue `steps` Newton steps, the state copy and an event (returns at once)."""
        self._call(A.load().nmg_newton2d_steps, steps, C.c_void_p(self._host.data_ptr()))
        self.event = torch.cuda.Event()
        self.event.record(self.stream)

    def ready(self) -> bool:
        return self.event is None or self.event.query()

    def wait(self):
        if self.event is not None:
            self.event.synchronize()

    def state(self):
        """(active, iters, status, res) after the last completed chunk."""
        s = A.nmg_newton_state.from_address(self._host.data_ptr())
        return s.active, s.iters, s.status, s.res


def interp_coarse_to_fine(Uc: torch.Tensor) -> torch.Tensor:
    """Appendix A interpolation of a device state [2, nc] to [2, 2 nc]."""
    Uc = Uc.contiguous()
    Uf = torch.empty((2, 2 * Uc.shape[1]), dtype=torch.float64, device=Uc.device)
    A.check(A.load().nmg_interp_coarse_to_fine(_dptr(Uc), Uc.shape[1], _dptr(Uf), C.c_void_p(_stream_ptr())))
    return Uf


def nested_solve(prob, ngrids: Optional[int] = None, device="cuda", precision: int = A.NMG_FP64,
                 check_every: int = 4):
    """Algorithm 3 on the GPU for a 1D problem: Newton with the direct solve on the coarsest of
    the nested grids (from the problem's initial guess there), then the Newton multigrid
    iteration on every finer grid from the interpolated coarser solution.  Returns (finest
    state [2, N] on the device, [(cells, Newton steps, status, res) per grid, finest first])."""
    from swe_workloads import nested_grids
    grids = nested_grids(prob, ngrids)
    ng = len(grids)
    devs = [Problem1DDevice(g, device, 3) for g in grids]
    descs = (A.nmg_desc * ng)(*[d.desc for d in devs])
    params = (A.nmg_params * ng)(*[params_struct(g.params, precision, check_every) for g in grids])
    Us = [torch.empty((2, g.n), dtype=torch.float64, device=device) for g in grids]
    Us[-1].copy_(torch.tensor(np.ascontiguousarray(grids[-1].initial_guess()), dtype=torch.float64))
    L = A.load()
    nbytes = L.nmg_nested_workspace_bytes(descs, ng, params)
    if nbytes == 0:
        raise A.NmgError(A.NMG_EINVAL, L.nmg_last_error().decode())
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    ptrs = (C.c_void_p * ng)(*[u.data_ptr() for u in Us])
    stats = (A.nmg_stats * ng)()
    st = L.nmg_nested_solve(descs, ng, params, _dptr(ws), nbytes, ptrs, stats, C.c_void_p(_stream_ptr()))
    A.check(st, ok=(A.NMG_OK, A.NMG_NOT_CONVERGED, A.NMG_ENONFINITE))
    return Us[0], [(g.n, s.iters, s.status, s.res) for g, s in zip(grids, stats)]


def interp2d_coarse_to_fine(Uc: torch.Tensor) -> torch.Tensor:
    """Eq. (A.3) interpolation of a device state [3, nyc, nxc] to [3, 2 nyc, 2 nxc]."""
    Uc = Uc.contiguous()
    _, nyc, nxc = Uc.shape
    Uf = torch.empty((3, 2 * nyc, 2 * nxc), dtype=torch.float64, device=Uc.device)
    A.check(A.load().nmg_interp2d_coarse_to_fine(_dptr(Uc), nxc, nyc, _dptr(Uf), C.c_void_p(_stream_ptr())))
    return Uf


def nested_solve2d(prob, ngrids: Optional[int] = None, device="cuda", precision: int = A.NMG_FP64,
                   check_every: int = 1, jac: int = 9, **param_overrides):
    """Algorithm 3 on the GPU for a 2D problem: Newton with the dense direct solve on the
    coarsest grid (one level) from the problem's initial state there, then the Newton multigrid
    iteration on every finer grid from the eq. (A.3) interpolation of the coarser solution.
    param_overrides apply to every grid.  Returns (finest state [3, ny, nx] on the device,
    [(nx, ny, Newton steps, status, res) per grid, finest first])."""
    import dataclasses
    from swe_workloads import nested_grids_2d
    grids = nested_grids_2d(prob, ngrids)
    ng = len(grids)
    A.load()
    devs = [Problem2DDevice(g, device, jac) for g in grids]
    descs = (A.nmg_desc * ng)(*[d.desc for d in devs])
    params = (A.nmg_params * ng)(*[params_struct(dataclasses.replace(g.params, **param_overrides),
                                                 precision, check_every) for g in grids])
    Us = [torch.empty((3, g.ny, g.nx), dtype=torch.float64, device=device) for g in grids]
    Us[-1].copy_(torch.tensor(np.ascontiguousarray(grids[-1].initial_guess()), dtype=torch.float64))
    L = A.load()
    nbytes = L.nmg_nested_workspace_bytes(descs, ng, params)
    if nbytes == 0:
        raise A.NmgError(A.NMG_EINVAL, L.nmg_last_error().decode())
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    ptrs = (C.c_void_p * ng)(*[u.data_ptr() for u in Us])
    stats = (A.nmg_stats * ng)()
    st = L.nmg_nested_solve(descs, ng, params, _dptr(ws), nbytes, ptrs, stats, C.c_void_p(_stream_ptr()))
    A.check(st, ok=(A.NMG_OK, A.NMG_NOT_CONVERGED, A.NMG_ENONFINITE))
    return Us[0], [(g.nx, g.ny, s.iters, s.status, s.res) for g, s in zip(grids, stats)]


class NestedBatch:
    """Algorithm 3 for a batch of 1D problems on the same nested grids: one batched plan per
    grid (every launch covers every instance), the Appendix A interpolation between grids.
    Each instance's result equals its own nested solve (no cross-instance arithmetic)."""

    def __init__(self, probs: Sequence, ngrids: Optional[int] = None, device="cuda",
                 precision: int = A.NMG_FP64, check_every: int = 4, jac: int = 3):
        """jac: 3 or 5 on the grids solved by the Newton multigrid iteration; the coarsest grid,
        solved directly (a one-level hierarchy, block tridiagonal), always takes J3."""
        from swe_workloads import nested_grids
        A.load()
        self.grids = [nested_grids(p, ngrids) for p in probs]      # [instance][grid]
        ng = len(self.grids[0])
        if any(len(g) != ng or g[0].n != self.grids[0][0].n for g in self.grids):
            raise ValueError("all problems of a nested batch need the same grids")
        self.ng = ng
        self.n = len(probs)
        self.device = device
        self.plans = [BatchSolver1D([g[k] for g in self.grids], device=device, precision=precision,
                                    check_every=check_every, jac=(3 if self.grids[0][k].levels == 1 else jac))
                      for k in range(ng)]

    def states(self):
        """Fresh per-grid state buffers with the coarsest initial guesses filled in."""
        Us = [[torch.empty((2, g[k].n), dtype=torch.float64, device=self.device) for g in self.grids]
              for k in range(self.ng)]
        for i, g in enumerate(self.grids):
            Us[-1][i].copy_(torch.tensor(np.ascontiguousarray(g[-1].initial_guess()), dtype=torch.float64))
        return Us

    def solve(self, Us, use_graph: bool = True):
        """Returns per grid (coarsest first) the list of (iters, status, res) per instance;
        Us[0] holds the finest solutions afterwards."""
        out = []
        for k in range(self.ng - 1, -1, -1):
            if k < self.ng - 1:
                for i in range(self.n):
                    A.check(A.load().nmg_interp_coarse_to_fine(
                        _dptr(Us[k + 1][i]), Us[k + 1][i].shape[1], _dptr(Us[k][i]), C.c_void_p(_stream_ptr())))
            out.append(self.plans[k].solve(Us[k], use_graph=use_graph))
        return out
