"""nmg_newton_solve_static (the Newton solve on the library's own static workspace) against
nmg_newton_solve with a caller workspace, through the C ABI: two calls in a row on one GPU, the
second with a smaller problem, each bitwise equal in state, step count, res and history; a
problem larger than the static workspace is rejected before any device work."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from swe_workloads import config1, config2, wedge_problem  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _static_solve(solver, U, max_hist=4000):
    from paper_2505_10857_amd import _abi as A
    L = A.load()
    st = A.nmg_stats()
    hist = (C.c_double * max_hist)()
    status = L.nmg_newton_solve_static(C.byref(solver.dev.desc), C.byref(solver.params),
                                       C.c_void_p(U.data_ptr()), C.byref(st), hist, max_hist, _stream())
    A.check(status, ok=(A.NMG_OK, A.NMG_NOT_CONVERGED))
    return st, np.array(hist[:min(max_hist, st.iters)])


def _compare(solver, label):
    U_ref = solver.state()
    st_ref, h_ref = solver.newton_solve(U_ref, max_hist=4000)
    assert st_ref.status == 0, f"{label}: the workspace call itself did not converge"
    U = solver.state()
    st, h = _static_solve(solver, U)
    torch.cuda.synchronize()
    same = torch.equal(U, U_ref)
    print(f"{label}: {st.iters} steps res {st.res:.3e} (workspace call {st_ref.iters}, {st_ref.res:.3e}); "
          f"state bitwise equal {same}, max|dU| {(U - U_ref).abs().max().item():.1e}", flush=True)
    assert st.status == st_ref.status == 0
    assert st.iters == st_ref.iters and st.res == st_ref.res
    assert same
    assert np.array_equal(h, h_ref)


@pytest.mark.parametrize("prec_name", ["fp64", "fp32mg"])
def test_static_1d_two_calls_second_smaller(prec_name):
    from paper_2505_10857_amd import Solver1D, _abi as A
    prec = A.NMG_FP64 if prec_name == "fp64" else A.NMG_FP32_MG
    big = Solver1D(config2(3), device=DEV, precision=prec)          # 12800 cells, 8 levels
    small = Solver1D(config1(5), device=DEV, precision=prec)        # 200 cells, 3 levels
    _compare(big, f"1D {prec_name} N=12800")
    _compare(small, f"1D {prec_name} N=200 after N=12800")


def test_static_2d_two_calls_second_smaller():
    from paper_2505_10857_amd import Solver2D
    big = Solver2D(wedge_problem(64, 32, seed=2), device=DEV)
    small = Solver2D(wedge_problem(32, 16, seed=5), device=DEV)
    _compare(big, "2D wedge 64x32")
    _compare(small, "2D wedge 32x16 after 64x32")


def test_static_rejects_problems_beyond_the_array():
    from paper_2505_10857_amd import Solver2D, _abi as A
    s = Solver2D(wedge_problem(512, 256), device=DEV)               # about 120 MiB in FP64
    need = A.load().nmg_workspace_bytes(C.byref(s.dev.desc), C.byref(s.params))
    assert need > A.NMG_STATIC_WS_MIB << 20
    U = s.state()
    st = A.nmg_stats()
    status = A.load().nmg_newton_solve_static(C.byref(s.dev.desc), C.byref(s.params), C.c_void_p(U.data_ptr()),
                                              C.byref(st), None, 0, _stream())
    assert status == A.NMG_ENOMEM_WS
    assert b"static workspace" in A.load().nmg_last_error()
