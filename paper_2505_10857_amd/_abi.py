"""ctypes mirror of include/nmg.h and the loader of the in-tree libnmg.so.

There is no fallback: if the HIP library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnmg.so")

NMG_OK = 0
NMG_NOT_CONVERGED = 1
NMG_EINVAL = -1
NMG_ENOMEM_WS = -2
NMG_EHIP = -3
NMG_ENONFINITE = -4

NMG_BC_DISCHARGE = 0
NMG_BC_DEPTH = 1
NMG_BC_EXTRAP = 2
NMG_BC_WALL = 3
NMG_BC_STATE = 4

NMG_FP64 = 0
NMG_FP32_MG = 1
NMG_RECON_CONSERVED = 0
NMG_RECON_SURFACE = 1

NMG_LINEAR_MG = 0
NMG_LINEAR_SOR = 1
NMG_LINEAR_SOR_LEX = 2
NMG_LINEAR_MG_SWEEPS = 3
NMG_SCHED2D_ALT_FINEST = 1
NMG_SCHED2D_ALT_COARSE = 2
NMG_SCHED2D_NO_STREAM = 4
NMG_SCHED2D_SMALL_BOTTOM = 8
NMG_TUNE2D_CANDIDATES = 16

EXPORTS = [
    "nmg_workspace_bytes", "nmg_residual", "nmg_jacobian_assemble_simplified", "nmg_mg_vcycle",
    "nmg_newton_solve", "nmg_plan_create", "nmg_plan_workspace_bytes", "nmg_plan_solve",
    "nmg_plan_begin", "nmg_plan_steps", "nmg_plan_destroy", "nmg_last_error",
    "nmg_plan_profile", "nmg_plan_profile_read", "nmg_plan_resume", "nmg_plan_set_options",
    "nmg_plan_get_options", "nmg_plan_autotune", "nmg_interp_coarse_to_fine",
    "nmg_nested_workspace_bytes", "nmg_nested_solve", "nmg_newton_solve_static",
    "nmg_interp2d_coarse_to_fine",
    "nmg_newton2d_begin",
    "nmg_newton2d_steps",
    "nmg_autotune2d",
    "nmg_lane_stream_create",
    "nmg_lane_stream_destroy",
]

NMG_STATIC_WS_MIB = 64

NMG_K_NONE = 0
NMG_K_JACOBIAN = 1
NMG_K_SMOOTH_PRE = 2
NMG_K_SMOOTH_POST = 3
NMG_K_RESIDUAL = 4
NMG_K_COARSEN = 5
NMG_K_SMOOTH_FUSED = 6


class nmg_bc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("q", C.c_double), ("h", C.c_double),
                ("u", C.c_double), ("v", C.c_double)]


class nmg_desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("levels", C.c_int32),
                ("jac", C.c_int32), ("recon", C.c_int32),
                ("x0", C.c_double), ("x1", C.c_double), ("y0", C.c_double), ("y1", C.c_double),
                ("g", C.c_double), ("bc", nmg_bc * 4), ("wall_x", C.c_double),
                ("sig_face", C.c_void_p), ("sig_gp", C.c_void_p), ("sigx_gp", C.c_void_p),
                ("bx_gp", C.c_void_p), ("by_gp", C.c_void_p), ("z_face", C.c_void_p),
                ("z_avg", C.c_void_p)]


class nmg_params(C.Structure):
    _fields_ = [("alpha", C.c_double), ("tau", C.c_double), ("eps", C.c_double),
                ("omega", C.c_double), ("tol", C.c_double),
                ("nu1", C.c_int32), ("nu2", C.c_int32), ("nu3", C.c_int32), ("n_max", C.c_int32),
                ("precision", C.c_int32), ("check_every", C.c_int32),
                ("linear", C.c_int32), ("sor_max", C.c_int32), ("sor_tol", C.c_double),
                ("schedule", C.c_int32), ("reserved", C.c_int32)]


class nmg_newton_state(C.Structure):
    _fields_ = [("res", C.c_double), ("iters", C.c_int32), ("active", C.c_int32), ("status", C.c_int32),
                ("reserved", C.c_int32)]


class nmg_stats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("status", C.c_int32), ("res", C.c_double)]


class nmg_plan_options(C.Structure):
    _fields_ = [("bottom_cells", C.c_int32), ("fused_finest", C.c_int32), ("smooth_tile", C.c_int32),
                ("split_finest", C.c_int32), ("split_residual", C.c_int32), ("reserved", C.c_int32 * 3)]


NMG_TUNE_CANDIDATES = 32


class NmgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libnmg status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libnmg.so (built by ``paper_2505_10857_amd.build``).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libnmg.so not found at {path}: build it with "
                           "`python -m paper_2505_10857_amd.build` (there is no CPU fallback)")
    # the library binds the HIP runtime by its soname; torch ships its own copy, and importing
    # torch after the library would put a second runtime in the process (with no devices of its
    # own to share with the first): torch first, so that the library binds to torch's runtime
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = C.CDLL(path)
    vp, sz = C.c_void_p, C.c_size_t
    P = C.POINTER
    L.nmg_workspace_bytes.argtypes = [P(nmg_desc), P(nmg_params)]
    L.nmg_workspace_bytes.restype = sz
    L.nmg_residual.argtypes = [P(nmg_desc), vp, vp, vp, vp, vp]
    L.nmg_jacobian_assemble_simplified.argtypes = [P(nmg_desc), P(nmg_params), vp, vp, vp, vp, vp]
    L.nmg_mg_vcycle.argtypes = [P(nmg_desc), P(nmg_params), vp, sz, vp, vp, vp, C.c_int32, vp]
    L.nmg_newton_solve.argtypes = [P(nmg_desc), P(nmg_params), vp, sz, vp, P(nmg_stats),
                                   P(C.c_double), C.c_int32, vp]
    L.nmg_newton_solve_static.argtypes = [P(nmg_desc), P(nmg_params), vp, P(nmg_stats), P(C.c_double),
                                          C.c_int32, vp]
    L.nmg_plan_create.argtypes = [P(nmg_desc), P(nmg_params), C.c_int32, P(vp)]
    L.nmg_plan_workspace_bytes.argtypes = [vp]
    L.nmg_plan_workspace_bytes.restype = sz
    L.nmg_plan_solve.argtypes = [vp, vp, sz, P(vp), P(nmg_stats), C.c_int32, vp]
    L.nmg_plan_begin.argtypes = [vp, vp, sz, P(vp), vp]
    L.nmg_plan_steps.argtypes = [vp, vp, C.c_int32, C.c_int32, P(C.c_int32), P(nmg_stats), vp]
    L.nmg_plan_resume.argtypes = [vp, vp, sz, P(vp), P(C.c_int32), vp]
    L.nmg_interp_coarse_to_fine.argtypes = [vp, C.c_int32, vp, vp]
    L.nmg_interp2d_coarse_to_fine.argtypes = [vp, C.c_int32, C.c_int32, vp, vp]
    L.nmg_newton2d_begin.argtypes = [P(nmg_desc), P(nmg_params), vp, sz, vp, vp]
    L.nmg_newton2d_steps.argtypes = [P(nmg_desc), P(nmg_params), vp, sz, vp, C.c_int32, vp, vp]
    L.nmg_autotune2d.argtypes = [P(nmg_desc), P(nmg_params), vp, sz, vp, vp, C.c_int32, P(C.c_int32),
                                 P(C.c_double), vp]
    L.nmg_lane_stream_create.argtypes = [P(vp)]
    L.nmg_lane_stream_destroy.argtypes = [vp]
    L.nmg_nested_workspace_bytes.argtypes = [P(nmg_desc), C.c_int32, P(nmg_params)]
    L.nmg_nested_workspace_bytes.restype = sz
    L.nmg_nested_solve.argtypes = [P(nmg_desc), C.c_int32, P(nmg_params), vp, sz, P(vp), P(nmg_stats), vp]
    L.nmg_plan_set_options.argtypes = [vp, P(nmg_plan_options)]
    L.nmg_plan_get_options.argtypes = [vp, P(nmg_plan_options)]
    L.nmg_plan_autotune.argtypes = [vp, vp, sz, P(vp), C.c_int32, C.c_int32, P(nmg_plan_options),
                                    P(C.c_double), vp]
    L.nmg_plan_destroy.argtypes = [vp]
    L.nmg_plan_destroy.restype = None
    L.nmg_plan_profile.argtypes = [vp, C.c_int32]
    L.nmg_plan_profile.restype = C.c_int32
    L.nmg_plan_profile_read.argtypes = [vp, P(C.c_double), P(C.c_int32)]
    L.nmg_plan_profile_read.restype = C.c_int32
    L.nmg_last_error.argtypes = []
    L.nmg_last_error.restype = C.c_char_p
    for nm in ("nmg_residual", "nmg_jacobian_assemble_simplified", "nmg_mg_vcycle",
               "nmg_newton_solve", "nmg_newton_solve_static", "nmg_plan_create", "nmg_plan_solve", "nmg_plan_begin",
               "nmg_plan_steps", "nmg_plan_resume", "nmg_plan_set_options", "nmg_plan_get_options",
               "nmg_plan_autotune", "nmg_interp_coarse_to_fine", "nmg_interp2d_coarse_to_fine",
               "nmg_nested_solve", "nmg_newton2d_begin", "nmg_newton2d_steps", "nmg_autotune2d",
               "nmg_lane_stream_create", "nmg_lane_stream_destroy"):
        getattr(L, nm).restype = C.c_int32
    _lib = L
    return L


def check(status: int, ok=(NMG_OK,)) -> int:
    if status in ok:
        return status
    raise NmgError(status, load().nmg_last_error().decode())
