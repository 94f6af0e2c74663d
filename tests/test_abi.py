"""The C-ABI library loads and exports every entry point include/nmg.h declares (CPU only:
no compute call is made without a GPU); host-side argument checks reject bad input."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nmg.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(nmg_\w+)\s*\(", txt)))


def _lib():
    from paper_2505_10857_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        pytest.skip("libnmg.so not built (run __graft_entry__.build())")
    return _abi, _abi.load()


def test_header_declares_the_four_paper_calls():
    names = _declared()
    for n in ("nmg_residual", "nmg_jacobian_assemble_simplified", "nmg_mg_vcycle", "nmg_newton_solve"):
        assert n in names


def test_library_exports_every_declared_symbol():
    abi, L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(abi.EXPORTS) <= set(_declared())


def test_struct_sizes_match_header_layout():
    abi, _ = _lib()
    assert ctypes.sizeof(abi.nmg_bc) == 40
    assert ctypes.sizeof(abi.nmg_desc) == 24 + 40 + 4 * 40 + 8 + 7 * 8
    assert ctypes.sizeof(abi.nmg_params) == 5 * 8 + 8 * 4 + 8 + 2 * 4
    assert ctypes.sizeof(abi.nmg_plan_options) == 8 * 4
    assert abi.NMG_TUNE_CANDIDATES == 32


def _desc(abi, nx=64, levels=3, jac=3):
    d = abi.nmg_desc()
    d.dim, d.nx, d.ny, d.levels, d.jac = 1, nx, 1, levels, jac
    d.x0, d.x1, d.g = 0.0, 1.0, 9.812
    d.sig_face = d.sig_gp = d.sigx_gp = d.bx_gp = 8   # non-null placeholders; never dereferenced
    p = abi.nmg_params()
    p.alpha, p.tau, p.eps, p.omega, p.tol = 3.0, 0.6, 0.01, 1.0, 1e-10
    p.nu1 = p.nu2 = p.nu3 = 2
    p.n_max = 100
    p.check_every = 1
    return d, p


def test_workspace_query_and_argument_checks():
    abi, L = _lib()
    d, p = _desc(abi)
    assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) > 0
    bad = [dict(nx=60, levels=4),      # not divisible by 2^(levels-1)
           dict(nx=4096, levels=2),    # coarsest level too large
           dict(jac=4), dict(levels=0),
           dict(levels=1, jac=5)]      # the direct one-level solve is block-tridiagonal
    for kw in bad:
        d2, p2 = _desc(abi, **kw)
        assert L.nmg_workspace_bytes(ctypes.byref(d2), ctypes.byref(p2)) == 0
        assert L.nmg_last_error()
    d1, p1 = _desc(abi, nx=128, levels=1)   # one level: Newton with the direct solve
    assert L.nmg_workspace_bytes(ctypes.byref(d1), ctypes.byref(p1)) > 0
    d3, p3 = _desc(abi)
    p3.eps = 0.0
    assert L.nmg_workspace_bytes(ctypes.byref(d3), ctypes.byref(p3)) == 0
    # residual with a null state pointer fails on the host before any launch
    assert L.nmg_residual(ctypes.byref(d), None, None, None, None, None) == abi.NMG_EINVAL
    # workspace too small
    st = abi.nmg_stats()
    assert L.nmg_newton_solve(ctypes.byref(d), ctypes.byref(p), ctypes.c_void_p(256), 16,
                              ctypes.c_void_p(512), ctypes.byref(st), None, 0, None) == abi.NMG_ENOMEM_WS


def test_plan_rejects_mixed_precision():
    abi, L = _lib()
    d1, p1 = _desc(abi)
    d2, p2 = _desc(abi, nx=128, levels=4)
    p2.precision = abi.NMG_FP32_MG
    descs = (abi.nmg_desc * 2)(d1, d2)
    params = (abi.nmg_params * 2)(p1, p2)
    plan = ctypes.c_void_p()
    assert L.nmg_plan_create(descs, params, 2, ctypes.byref(plan)) == abi.NMG_EINVAL
    params[1].precision = abi.NMG_FP64
    assert L.nmg_plan_create(descs, params, 2, ctypes.byref(plan)) == abi.NMG_OK
    assert L.nmg_plan_workspace_bytes(plan) > L.nmg_workspace_bytes(ctypes.byref(d1), ctypes.byref(p1))
    L.nmg_plan_destroy(plan)


def test_nested_solve_argument_checks():
    """Grid g of the nested iteration must have half the cells of grid g-1 and ngrids - g levels;
    the checks run on the host before any launch."""
    abi, L = _lib()
    grids = [_desc(abi, nx=256 >> g, levels=3 - g) for g in range(3)]
    descs = (abi.nmg_desc * 3)(*[g[0] for g in grids])
    params = (abi.nmg_params * 3)(*[g[1] for g in grids])
    ws = L.nmg_nested_workspace_bytes(descs, 3, params)
    assert ws == max(L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) for d, p in grids)
    U = (ctypes.c_void_p * 3)(256, 512, 768)
    st = (abi.nmg_stats * 3)()
    descs[1].levels = 3
    assert L.nmg_nested_solve(descs, 3, params, ctypes.c_void_p(1024), ws, U, st, None) == abi.NMG_EINVAL
    descs[1].levels = 2
    descs[2].nx = 48
    assert L.nmg_nested_solve(descs, 3, params, ctypes.c_void_p(1024), ws, U, st, None) == abi.NMG_EINVAL
    descs[2].nx = 64
    assert L.nmg_nested_solve(descs, 3, params, ctypes.c_void_p(1024), 16, U, st, None) == abi.NMG_ENOMEM_WS
    assert L.nmg_interp_coarse_to_fine(ctypes.c_void_p(256), 2, ctypes.c_void_p(512), None) == abi.NMG_EINVAL
    assert L.nmg_interp2d_coarse_to_fine(ctypes.c_void_p(256), 4, 2, ctypes.c_void_p(512), None) == abi.NMG_EINVAL
    assert L.nmg_interp2d_coarse_to_fine(None, 4, 4, ctypes.c_void_p(512), None) == abi.NMG_EINVAL
    descs[1].dim = 2                 # grids of one nested iteration share their dimension
    assert L.nmg_nested_solve(descs, 3, params, ctypes.c_void_p(1024), ws, U, st, None) == abi.NMG_EINVAL
    assert b"same dim" in L.nmg_last_error()


def test_reconstruction_field_is_checked():
    """recon must be NMG_RECON_CONSERVED or NMG_RECON_SURFACE (1D); 2D takes only the first."""
    abi, L = _lib()
    d, p = _desc(abi)
    d.recon = abi.NMG_RECON_SURFACE
    assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) > 0
    d.recon = 2
    assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) == 0
    assert b"recon" in L.nmg_last_error()


def test_size_limits_and_empty_batch():
    """The accepted 1D sizes end exactly where the header says, and an empty batch is refused."""
    abi, L = _lib()
    ok = [dict(nx=4, levels=1), dict(nx=256 << 15, levels=16), dict(nx=256, levels=1)]
    bad = [dict(nx=3, levels=1),               # fewer than four cells
           dict(nx=256 << 16, levels=16),      # coarsest level of 512 cells
           dict(nx=257 << 15, levels=16),      # not divisible by 2^15
           dict(nx=512, levels=1),             # one level of more than 256 cells
           dict(nx=256 << 16, levels=17)]      # more than 16 levels
    for kw in ok:
        d, p = _desc(abi, **kw)
        assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) > 0, kw
    for kw in bad:
        d, p = _desc(abi, **kw)
        assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) == 0, kw
        assert L.nmg_last_error()
    d, p = _desc(abi)
    descs = (abi.nmg_desc * 1)(d)
    params = (abi.nmg_params * 1)(p)
    plan = ctypes.c_void_p()
    for n in (0, -1):
        assert L.nmg_plan_create(descs, params, n, ctypes.byref(plan)) == abi.NMG_EINVAL
        assert L.nmg_last_error()


def test_static_newton_solve_rejects_on_the_host():
    """nmg_newton_solve_static refuses null arguments and problems whose workspace exceeds its
    NMG_STATIC_WS_MIB static array before it touches the device."""
    abi, L = _lib()
    d, p = _desc(abi)
    st = abi.nmg_stats()
    assert L.nmg_newton_solve_static(None, ctypes.byref(p), ctypes.c_void_p(256), ctypes.byref(st), None, 0,
                                     None) == abi.NMG_EINVAL
    assert L.nmg_newton_solve_static(ctypes.byref(d), ctypes.byref(p), None, ctypes.byref(st), None, 0,
                                     None) == abi.NMG_EINVAL
    big, pb = _desc(abi, nx=256 << 12, levels=13)            # about 300 MiB of workspace
    assert L.nmg_workspace_bytes(ctypes.byref(big), ctypes.byref(pb)) > abi.NMG_STATIC_WS_MIB << 20
    assert L.nmg_newton_solve_static(ctypes.byref(big), ctypes.byref(pb), ctypes.c_void_p(256),
                                     ctypes.byref(st), None, 0, None) == abi.NMG_ENOMEM_WS
    assert b"static workspace" in L.nmg_last_error()
    bad, pbad = _desc(abi, nx=60, levels=4)
    assert L.nmg_newton_solve_static(ctypes.byref(bad), ctypes.byref(pbad), ctypes.c_void_p(256),
                                     ctypes.byref(st), None, 0, None) == abi.NMG_EINVAL


def test_2d_surface_reconstruction_needs_its_bottom_samples():
    """recon = NMG_RECON_SURFACE in 2D needs z_avg and z_face; the check runs on the host before
    any launch.  Other recon values are rejected."""
    abi, L = _lib()
    d = abi.nmg_desc()
    d.dim, d.nx, d.ny, d.levels, d.jac, d.recon = 2, 32, 16, 3, 9, abi.NMG_RECON_SURFACE
    d.x0, d.x1, d.y0, d.y1, d.g = 0.0, 4.0, 0.0, 2.0, 9.81
    for k in range(4):
        d.bc[k].kind = abi.NMG_BC_WALL
    d.bx_gp = d.by_gp = 4096
    U = ctypes.c_void_p(8192)
    assert L.nmg_residual(ctypes.byref(d), U, U, U, None, None) == abi.NMG_EINVAL
    assert b"z_face and z_avg" in L.nmg_last_error()
    d.recon = 2
    assert L.nmg_residual(ctypes.byref(d), U, U, U, None, None) == abi.NMG_EINVAL
    assert b"recon" in L.nmg_last_error()


def test_linear_solver_choices_per_dimension():
    """NMG_LINEAR_MG_SWEEPS is 2D only and limited to 65536 cells; the Newton-SOR solvers are 1D
    only.  Checked on the host before any launch."""
    abi, L = _lib()
    d, p = _desc(abi)
    p.linear = abi.NMG_LINEAR_MG_SWEEPS
    assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) == 0
    d2 = abi.nmg_desc()
    d2.dim, d2.nx, d2.ny, d2.levels, d2.jac = 2, 32, 16, 3, 9
    d2.x0, d2.x1, d2.y0, d2.y1, d2.g = 0.0, 4.0, 0.0, 2.0, 9.81
    for k in range(4):
        d2.bc[k].kind = abi.NMG_BC_WALL
    p2 = abi.nmg_params()
    p2.eps, p2.nu1, p2.nu2, p2.nu3, p2.n_max = 1e-6, 2, 2, 1, 10
    p2.linear = abi.NMG_LINEAR_MG_SWEEPS
    assert L.nmg_workspace_bytes(ctypes.byref(d2), ctypes.byref(p2)) > 0
    p2.linear = abi.NMG_LINEAR_SOR
    assert L.nmg_workspace_bytes(ctypes.byref(d2), ctypes.byref(p2)) == 0
    p2.linear = abi.NMG_LINEAR_MG_SWEEPS
    d2.nx, d2.ny, d2.levels = 512, 256, 7
    assert L.nmg_workspace_bytes(ctypes.byref(d2), ctypes.byref(p2)) == 0
    assert b"65536" in L.nmg_last_error()


def test_2d_schedule_is_checked():
    abi, L = _lib()
    d = abi.nmg_desc()
    d.dim, d.nx, d.ny, d.levels, d.jac = 2, 32, 16, 3, 9
    d.x0, d.x1, d.y0, d.y1, d.g = 0.0, 4.0, 0.0, 2.0, 9.81
    for k in range(4):
        d.bc[k].kind = abi.NMG_BC_WALL
    p = abi.nmg_params()
    p.eps, p.nu1, p.nu2, p.nu3, p.n_max = 1e-6, 2, 2, 1, 10
    for c in range(abi.NMG_TUNE2D_CANDIDATES):
        p.schedule = c
        assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) > 0
    p.schedule = abi.NMG_TUNE2D_CANDIDATES
    assert L.nmg_workspace_bytes(ctypes.byref(d), ctypes.byref(p)) == 0
    p.schedule = 0
    best = ctypes.c_int32()
    ms = (ctypes.c_double * abi.NMG_TUNE2D_CANDIDATES)()
    assert L.nmg_autotune2d(ctypes.byref(d), ctypes.byref(p), None, 0, None, None, 1, ctypes.byref(best), ms,
                            None) == abi.NMG_EINVAL
