"""Newton-SOR (the reference solver of section 5.1.1 / Table 2) on the GPU against the oracle:
the lexicographic symmetric sweep reproduces the oracle's Newton-SOR to the bit budget of the
parity bar, the multicolour variant its trajectory; both inner iterations stop by the l1 change
of dU or the step limit."""
import dataclasses

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from swe_workloads import config1, config4_instance, e1_problem  # noqa: E402

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _sor_problem(prob, linear):
    return dataclasses.replace(prob, params=dataclasses.replace(prob.params, linear=linear, sor_max=10,
                                                                sor_tol=1e-7))


def test_lexicographic_newton_sor_matches_the_oracle():
    """E1 on 96 cells (Table 2's smallest grid): full solve, same step count, same state."""
    from paper_2505_10857_amd import Solver1D
    prob = _sor_problem(e1_problem(96), 2)
    s = Solver1D(prob, device=DEV, check_every=1)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, ito, reso, _ = oracle.Oracle1D(prob).newton_solve(linear=1, smoother=1, sor_max=10, sor_tol=1e-7)
    err = np.abs(U.cpu().numpy() - Uo).max()
    print("lex Newton-SOR:", st.iters, ito, st.res, reso, err)
    assert st.status == 0 and reso < prob.params.tol
    assert abs(st.iters - ito) <= 1
    assert err <= 1e-10


@pytest.mark.parametrize("name,prob", [("cfg1", config1(0)), ("cfg4", config4_instance(5))])
def test_multicolour_newton_sor_trajectory(name, prob):
    """Five Newton-SOR steps with the multicolour symmetric step: state within 1e-10."""
    from paper_2505_10857_amd import Solver1D
    p = _sor_problem(prob, 1)
    s = Solver1D(p, device=DEV, check_every=1, n_max=5)
    U = s.state()
    st, hist = s.newton_solve(U, max_hist=5)
    Uo, ito, reso, hist_o = oracle.Oracle1D(p).newton_solve(linear=1, smoother=0, sor_max=10, sor_tol=1e-7,
                                                            n_max=5)
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    print(name, "mc Newton-SOR 5 steps:", hist, hist_o, err)
    assert st.iters == ito == 5
    assert err <= 1e-10


def test_newton_sor_batch_equals_single():
    from paper_2505_10857_amd import BatchSolver1D
    probs = [_sor_problem(p, 1) for p in (config1(1), config4_instance(9), config1(3))]
    alone = []
    for p in probs:
        b = BatchSolver1D([p], device=DEV)
        Us = b.states()
        r = b.solve(Us, use_graph=False)
        alone.append((Us[0].clone(), r[0]))
    mix = BatchSolver1D(probs, device=DEV)
    Us = mix.states()
    rs = mix.solve(Us, use_graph=True)
    for k in range(len(probs)):
        assert rs[k][0] == alone[k][1][0]
        assert torch.equal(Us[k], alone[k][0])


@pytest.mark.parametrize("n,jac", [(600, 3), (768, 5), (1100, 3)])
def test_lexicographic_newton_sor_over_several_chunks(n, jac):
    """The lexicographic sweep staged through LDS in chunks of 256 cells: grids of two to five
    chunks (ragged last chunks; the five-block stencil carries two cells across each chunk edge);
    eight Newton-SOR steps, state and residual history against the oracle's within 1e-10."""
    from paper_2505_10857_amd import Solver1D
    prob = _sor_problem(e1_problem(n), 2)
    s = Solver1D(prob, device=DEV, jac=jac, check_every=1, n_max=8)
    U = s.state()
    st, hist = s.newton_solve(U, max_hist=8)
    Uo, ito, reso, hist_o = oracle.Oracle1D(prob).newton_solve(nb=jac, linear=1, smoother=1, sor_max=10,
                                                            sor_tol=1e-7, n_max=8)
    err = np.abs(U.cpu().numpy() - Uo).max() / np.abs(Uo).max()
    print(f"lex Newton-SOR N={n} J{jac}: {st.iters} steps, rel err {err:.2e}, res {hist[-1]:.3e} vs {hist_o[-1]:.3e}")
    assert st.iters == ito == 8
    assert err <= 1e-10
    assert np.all(np.abs(hist - hist_o) <= 1e-10 * np.abs(hist_o) + 1e-14)


def test_lexicographic_newton_sor_batch_equals_single():
    """Instances of different sizes (one and four chunks) in one plan: each result equals its
    solve alone, bit for bit."""
    from paper_2505_10857_amd import BatchSolver1D
    probs = [_sor_problem(e1_problem(n), 2) for n in (96, 1000, 384)]
    probs = [dataclasses.replace(p, params=dataclasses.replace(p.params, n_max=6)) for p in probs]
    alone = []
    for p in probs:
        b = BatchSolver1D([p], device=DEV)
        Us = b.states()
        r = b.solve(Us, use_graph=False)
        alone.append((Us[0].clone(), r[0]))
    mix = BatchSolver1D(probs, device=DEV)
    Us = mix.states()
    rs = mix.solve(Us, use_graph=True)
    for k in range(len(probs)):
        assert rs[k][0] == alone[k][1][0]
        assert torch.equal(Us[k], alone[k][0])


@pytest.mark.parametrize("n", [96, 192])
def test_table2_setting_step_counts_match_the_oracle(n):
    """Table 2's setting (E1, the Appendix A start from the steady state on n/2 cells, res <
    1e-11): NMGM-3 with the multicolour smoother and Newton-SOR with the lexicographic sweep take
    the oracle's Newton steps (within one) and reach its state within 1e-10."""
    from paper_2505_10857_amd import Solver1D
    from paper_2505_10857_amd.solver import interp_coarse_to_fine
    sc = Solver1D(e1_problem(n // 2), device=DEV, check_every=1)
    Uc = sc.state()
    sc.newton_solve(Uc)
    U0 = interp_coarse_to_fine(Uc)
    Uc_o, _, rc, _ = oracle.Oracle1D(e1_problem(n // 2)).newton_solve()
    U0_o = oracle.interp_a2(Uc_o)
    assert np.abs(U0.cpu().numpy() - U0_o).max() <= 1e-10
    for lin, kw in ((0, dict(smoother=0)), (2, dict(smoother=1, linear=1, sor_max=10, sor_tol=1e-7))):
        prob = e1_problem(n)
        if lin:
            prob = _sor_problem(prob, lin)
        s = Solver1D(prob, device=DEV, check_every=1)
        U = U0.clone()
        st, _ = s.newton_solve(U)
        Uo, ito, reso, _ = oracle.Oracle1D(prob).newton_solve(U0=U0_o, **kw)
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(f"N={n} linear={lin}: GPU {st.iters} steps, oracle {ito}; |dU| {err:.2e}")
        assert st.status == 0 and reso < 1e-11
        assert abs(st.iters - ito) <= 1
        assert err <= 1e-10
