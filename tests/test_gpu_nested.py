"""Nested iteration (Algorithm 3) on the GPU against the oracle: the Appendix A interpolation,
Newton with the direct coarsest solve (one-level hierarchy), and the whole nested solve on the
subcritical and transcritical humps (the latter is out of reach of plain Newton from the flat
surface)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from swe_workloads import config2  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_interpolation_parity():
    from paper_2505_10857_amd.solver import interp_coarse_to_fine
    rng = np.random.default_rng(17)
    for nc in (3, 4, 100, 1603):
        Uc = rng.uniform(0.3, 3.0, (2, nc))
        Uf = interp_coarse_to_fine(torch.tensor(Uc, device=DEV)).cpu().numpy()
        ref = oracle.interp_a2(Uc)
        print(nc, np.abs(Uf - ref).max(), np.array_equal(Uf, ref))
        assert np.abs(Uf - ref).max() <= 1e-15 * np.abs(ref).max()


def test_one_level_newton_is_the_direct_solve():
    from paper_2505_10857_amd import Solver1D
    for variant in ("sub", "trans"):
        prob = config2(0, variant, n=100, levels=1)
        s = Solver1D(prob, device=DEV)
        U = s.state()
        st, _ = s.newton_solve(U)
        Uo, ito, reso, _ = oracle.Oracle1D(prob).newton_solve()
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(variant, st.iters, ito, st.res, err)
        assert st.status == 0 and abs(st.iters - ito) <= 1
        assert err <= 1e-10


@pytest.mark.parametrize("variant,n,levels", [("sub", 800, 4), ("trans", 3200, 6), ("trans", 12800, 8)])
def test_nested_solve_matches_the_oracle(variant, n, levels):
    from paper_2505_10857_amd.solver import nested_solve
    prob = config2(0, variant, n=n, levels=levels)
    U, rep = nested_solve(prob, device=DEV)
    Uo, rep_o = oracle.nested_solve(prob)
    err = np.abs(U.cpu().numpy() - Uo).max()
    print(variant, n, "gpu", [(r[0], r[1]) for r in rep], "oracle", [(r[0], r[1]) for r in rep_o[::-1]],
          f"|dU| {err:.2e}")
    assert all(r[2] == 0 for r in rep)
    for (ng, it, _, _), (no, ito, _) in zip(rep, rep_o[::-1]):
        assert ng == no and abs(it - ito) <= 1
    assert err <= 1e-10


def test_nested_batch_equals_single_nested_solves():
    from paper_2505_10857_amd.solver import NestedBatch, nested_solve
    probs = [config2(i, v, n=800, levels=4) for i, v in ((0, "trans"), (1, "sub"), (2, "trans"))]
    nb = NestedBatch(probs, device=DEV)
    Us = nb.states()
    rep = nb.solve(Us, use_graph=True)
    assert all(x[1] == 0 for x in rep[-1])
    for i, p in enumerate(probs):
        U1, r1 = nested_solve(p, device=DEV)
        assert torch.equal(U1, Us[0][i])
        assert [r[1] for r in r1] == [rep[::-1][k][i][0] for k in range(4)]


def test_interpolation_2d_parity():
    """Eq. (A.3) on the device equals the oracle's bit for bit (same operations in the same
    order, no contraction), on grids from the 3 x 3 minimum to the 1024 x 512 finest grid's
    coarse parent, with ragged sizes that are not multiples of the 256-wide rows of the kernel."""
    from oracle import swe2d
    from paper_2505_10857_amd.solver import interp2d_coarse_to_fine
    rng = np.random.default_rng(19)
    for nyc, nxc in ((3, 3), (4, 5), (37, 130), (256, 512)):
        Uc = rng.uniform(0.3, 3.0, (3, nyc, nxc))
        Uf = interp2d_coarse_to_fine(torch.tensor(Uc, device=DEV)).cpu().numpy()
        ref = swe2d.interp_a3(Uc)
        print(nxc, nyc, np.abs(Uf - ref).max(), flush=True)
        assert np.array_equal(Uf, ref)


def test_nested_solve_2d_matches_the_oracle():
    """Algorithm 3 on the wedge, 32 x 16 cells on three nested grids (8 x 4 by the dense direct
    solve, then 16 x 8 and 32 x 16 by the Newton multigrid iteration), omega = 0.03: the same
    Newton step counts per grid as the oracle's nested solve (within one) and the same finest
    solution."""
    from oracle import swe2d
    from paper_2505_10857_amd.solver import nested_solve2d
    from swe_workloads import wedge_problem
    prob = wedge_problem(32, 16, seed=0)
    U, rep = nested_solve2d(prob, device=DEV, omega=0.03)
    Uo, rep_o = swe2d.nested_solve2d(prob, omega=0.03)
    err = np.abs(U.cpu().numpy() - Uo).max()
    print("gpu", [(r[0], r[1], r[2]) for r in rep], "oracle", [(r[0], r[1], r[2]) for r in rep_o[::-1]],
          f"|dU| {err:.2e}", flush=True)
    assert all(r[3] == 0 for r in rep)
    for (nx, ny, it, _, _), (nxo, nyo, ito, _) in zip(rep, rep_o[::-1]):
        assert (nx, ny) == (nxo, nyo) and abs(it - ito) <= 1
    assert err <= 1e-10


def test_nested_batch_with_the_full_jacobian_matches_the_oracle():
    """Transcritical hump, 800 cells, 4 grids, J5 on the multigrid grids (the coarsest, solved
    directly, keeps J3): the oracle run grid by grid with the same Jacobians gives the same
    Newton steps (within one) and the same finest state."""
    from paper_2505_10857_amd.solver import NestedBatch
    from swe_workloads import nested_grids
    prob = config2(0, "trans", n=800, levels=4)
    nb = NestedBatch([prob], device=DEV, jac=5)
    Us = nb.states()
    rep = nb.solve(Us, use_graph=True)
    grids = nested_grids(prob)
    U = grids[-1].initial_guess()
    steps = []
    for g in range(len(grids) - 1, -1, -1):
        if g < len(grids) - 1:
            U = oracle.interp_a2(U)
        U, it, res, _ = oracle.Oracle1D(grids[g]).newton_solve(U0=U, nb=3 if g == len(grids) - 1 else 5,
                                                               levels=len(grids) - g)
        steps.append(it)
    gpu_steps = [r[0][0] for r in rep]
    err = np.abs(Us[0][0].cpu().numpy() - U).max()
    print("J5 nested: gpu", gpu_steps, "oracle", steps, f"|dU| {err:.2e}", flush=True)
    assert all(r[0][1] == 0 for r in rep)
    assert all(abs(a - b) <= 1 for a, b in zip(gpu_steps, steps))
    assert err <= 1e-10
