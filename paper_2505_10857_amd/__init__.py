"""MI355X-native Newton multigrid solver for steady shallow water equations.

The solver (third-order WENO finite volumes, simplified finite-difference block Jacobian,
geometric multigrid with multicolour block SOR) runs in hand-written HIP kernels for gfx950
behind the C ABI of ``include/nmg.h`` (libnmg.so).  This package is the thin Python binding.
"""
from ._abi import (NMG_BC_DEPTH, NMG_BC_DISCHARGE, NMG_BC_EXTRAP, NMG_BC_STATE, NMG_BC_WALL,
                   NMG_EHIP, NMG_EINVAL, NMG_ENOMEM_WS, NMG_ENONFINITE, NMG_FP32_MG, NMG_FP64,
                   NMG_NOT_CONVERGED, NMG_OK, NmgError, load)

__all__ = ["load", "NmgError", "NMG_FP64", "NMG_FP32_MG", "Solver1D", "BatchSolver1D", "Solver2D"]


def __getattr__(name):
    # the binding imports torch; keep `import paper_2505_10857_amd` light for the build step
    if name in ("Solver1D", "BatchSolver1D", "Problem1DDevice", "Solver2D", "Problem2DDevice"):
        from . import solver
        return getattr(solver, name)
    raise AttributeError(name)
