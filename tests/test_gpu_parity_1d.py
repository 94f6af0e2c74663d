"""GPU parity of the 1D hot path against the CPU oracle, through the C ABI.

Bar (FP64): residual and Jacobian within 1e-12 relative (the kernels evaluate the formulas in
algebraically equal forms with fewer divisions, so agreement is to rounding; the tests report
whether it is also bitwise), one V-cycle within 1e-12 relative, Newton trajectories within
1e-10 at the same step count.  FP32 multigrid: converged state within
1e-9 of the FP64 oracle's.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle  # noqa: E402
from swe_workloads import (BC, BC_DEPTH, BC_DISCHARGE, BC_WALL, Params, Problem1D,  # noqa: E402
                           config1, config2, config4_instance, gaussian_bump, sine_width,
                           unit_width)

DEV = "cuda:0"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_10857_amd import _abi
    _abi.load()


def _solver(prob, **kw):
    from paper_2505_10857_amd import Solver1D
    return Solver1D(prob, device=DEV, **kw)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _mid_state(prob, steps=5):
    """Oracle iterate after a few Newton steps (an interior point of the trajectory)."""
    o = oracle.Oracle1D(prob)
    U, it, res, _ = o.newton_solve(n_max=steps)
    return U


def _cases():
    yield "cfg1", config1(0)
    yield "cfg1-ragged-wall", Problem1D("wall", 0.0, 3.0, 328, 3, gaussian_bump(0.1, 1.5, 0.1),
                                        sine_width(2, 3.0, 0.1), BC(BC_WALL), BC(BC_DEPTH, h=1.0),
                                        Params(eps=0.05), surface0=1.0, q0=0.0)
    yield "cfg4-width", config4_instance(3)
    yield "tiny", Problem1D("tiny", 0.0, 1.0, 8, 2, gaussian_bump(0.05, 0.5, 0.05), unit_width,
                            BC(BC_DISCHARGE, q=0.5), BC(BC_DEPTH, h=1.0), Params(eps=0.1),
                            surface0=1.0, q0=0.5)


@pytest.mark.parametrize("name,prob", list(_cases()), ids=[c[0] for c in _cases()])
def test_residual_parity(name, prob):
    s = _solver(prob)
    o = oracle.Oracle1D(prob)
    for U0 in (prob.initial_guess(), _mid_state(prob)):
        U = s.state(U0)
        R, rn, res = s.residual(U)
        Ro, rno, reso = o.residual(U0)
        Rg = R.cpu().numpy()
        scale = max(np.abs(Ro).max(), 1.0)
        err = np.abs(Rg - Ro).max()
        print(f"{name}: residual max|dR| = {err:.3e} (bitwise equal: {np.array_equal(Rg, Ro)})")
        assert err <= 1e-12 * scale
        assert np.abs(rn.cpu().numpy() - rno).max() <= 1e-12 * scale
        # res is the mean of |R0| + |R1|, so its error is at most twice the largest R error
        assert abs(res.item() - reso) <= 2e-12 * scale


@pytest.mark.parametrize("nb", [3, 5])
@pytest.mark.parametrize("name,prob", list(_cases()), ids=[c[0] for c in _cases()])
def test_jacobian_parity(name, prob, nb):
    s = _solver(prob, jac=nb)
    o = oracle.Oracle1D(prob)
    for U0 in (prob.initial_guess(), _mid_state(prob)):
        U = s.state(U0)
        R, rn, _ = s.residual(U)
        J = s.jacobian(U, R, rn).cpu().numpy()          # [nb, 2, 2, N]
        Jo = o.jacobian(U0, nb=nb)                       # [N, nb, 2, 2]
        Jg = np.transpose(J, (3, 0, 1, 2))
        err = np.abs(Jg - Jo).max()
        print(f"{name} J{nb}: max|dJ| = {err:.3e} / |J| {np.abs(Jo).max():.3e} "
              f"(bitwise equal: {np.array_equal(Jg, Jo)})")
        assert err <= 1e-12 * np.abs(Jo).max()


@pytest.mark.parametrize("name,prob", list(_cases()), ids=[c[0] for c in _cases()])
def test_vcycle_parity(name, prob):
    s = _solver(prob)
    o = oracle.Oracle1D(prob)
    U0 = _mid_state(prob)
    Jo = o.jacobian(U0, nb=3)
    rng = np.random.default_rng(0)
    rhs = rng.standard_normal((prob.n, 2))
    J = torch.tensor(np.ascontiguousarray(np.transpose(Jo, (1, 2, 3, 0))), dtype=torch.float64, device=DEV)
    rhs_d = torch.tensor(np.ascontiguousarray(rhs.T), dtype=torch.float64, device=DEV)
    dU = torch.zeros(2, prob.n, dtype=torch.float64, device=DEV)
    p = prob.params
    ref = np.zeros((prob.n, 2))
    for cyc in range(2):
        s.vcycle(J, rhs_d, dU, setup=(cyc == 0))
        ref = oracle.vcycles(Jo, rhs, ref, levels=prob.levels, ncycles=1, omega=p.omega,
                             nu1=p.nu1, nu2=p.nu2)
        g = dU.cpu().numpy().T
        err = _rel(g, ref)
        print(f"{name}: V-cycle {cyc + 1} rel.err {err:.3e} (bitwise equal: {np.array_equal(g, ref)})")
        assert err <= 1e-12


def _with_params(prob, **kw):
    import dataclasses
    return dataclasses.replace(prob, params=dataclasses.replace(prob.params, **kw))


@pytest.mark.parametrize("nb,nu1,nu2", [(3, 1, 3), (3, 3, 1), (5, 2, 2), (5, 1, 2)])
def test_vcycle_parity_tiled_levels(nb, nu1, nu2):
    """Levels above the bottom-of-cycle threshold (2048 cells) are smoothed in tiles whose halo
    is the reach of the merged colour schedule; N = 8192 puts the two finest levels in 34 and
    17 tiles.  Unequal pre/post counts and the three-colour J5 smoother, two V-cycles, 1e-12."""
    prob = _with_params(config2(0, "sub", n=8192, levels=6), nu1=nu1, nu2=nu2)
    s = _solver(prob, jac=nb)
    o = oracle.Oracle1D(prob)
    U0 = _mid_state(prob, steps=3)
    Jo = o.jacobian(U0, nb=nb)
    rng = np.random.default_rng(1)
    rhs = rng.standard_normal((prob.n, 2))
    J = torch.tensor(np.ascontiguousarray(np.transpose(Jo, (1, 2, 3, 0))), dtype=torch.float64, device=DEV)
    rhs_d = torch.tensor(np.ascontiguousarray(rhs.T), dtype=torch.float64, device=DEV)
    dU = torch.zeros(2, prob.n, dtype=torch.float64, device=DEV)
    ref = np.zeros((prob.n, 2))
    for cyc in range(2):
        s.vcycle(J, rhs_d, dU, setup=(cyc == 0))
        ref = oracle.vcycles(Jo, rhs, ref, levels=prob.levels, ncycles=1, omega=prob.params.omega,
                             nu1=nu1, nu2=nu2)
        err = _rel(dU.cpu().numpy().T, ref)
        print(f"J{nb} nu=({nu1},{nu2}): V-cycle {cyc + 1} rel.err {err:.3e}")
        assert err <= 1e-12


@pytest.mark.parametrize("nu1,nu2", [(1, 3), (2, 2)])
def test_newton_trajectory_fused_smoothing(nu1, nu2):
    """N = 8192, nu3 = 2: the finest level's post-smoothing of the first cycle and the
    pre-smoothing of the second run in one tiled launch (halo for nu2 + nu1 steps).  Three
    Newton steps against the oracle's, within 1e-10."""
    prob = _with_params(config2(1, "sub", n=8192, levels=6), nu1=nu1, nu2=nu2)
    o = oracle.Oracle1D(prob)
    s = _solver(prob, check_every=1, n_max=3)
    U = s.state()
    st, _ = s.newton_solve(U)
    Uo, ito, reso, _ = o.newton_solve(n_max=3)
    assert st.iters == ito == 3
    err = np.abs(U.cpu().numpy() - Uo).max()
    print(f"nu=({nu1},{nu2}): after 3 steps |U_gpu - U_oracle| = {err:.3e}")
    assert err <= 1e-10


@pytest.mark.parametrize("name,prob", list(_cases())[:3], ids=[c[0] for c in _cases()][:3])
def test_newton_trajectory_parity(name, prob):
    """Same number of Newton steps, states within 1e-10 after each checked prefix."""
    o = oracle.Oracle1D(prob)
    for steps in (3, 20):
        s2 = _solver(prob, check_every=1, n_max=steps)
        U = s2.state()
        st, _ = s2.newton_solve(U)
        Uo, ito, reso, _ = o.newton_solve(n_max=steps)
        assert st.iters == ito, (st.iters, st.status, st.res, ito, reso)
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(f"{name}: after {steps} steps |U_gpu - U_oracle| = {err:.3e}")
        assert err <= 1e-10


def test_newton_converged_cfg1_seeds():
    for i in range(4):
        prob = config1(i)
        s = _solver(prob)
        U = s.state()
        st, hist = s.newton_solve(U, max_hist=3000)
        Uo, ito, reso, histo = oracle.Oracle1D(prob).newton_solve()
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(f"cfg1[{i}]: gpu {st.iters} it res {st.res:.2e}; oracle {ito} it; dU {err:.2e}")
        assert st.status == 0 and st.res < 1e-10
        assert abs(st.iters - ito) <= 1
        assert err <= 1e-10
        n = min(len(hist), len(histo))
        assert np.allclose(hist[:n], histo[:n], rtol=1e-9)


def test_config2_full_size_residual_jacobian_and_solve():
    """N = 12800, 8 levels (the benchmark workload): R and J element by element at the
    initial guess, and the converged GPU state against the oracle's."""
    prob = config2(0, "sub")
    s = _solver(prob)
    o = oracle.Oracle1D(prob)
    U0 = prob.initial_guess()
    U = s.state(U0)
    R, rn, _ = s.residual(U)
    Ro, rno, _ = o.residual(U0)
    # R is a difference of fluxes of size O(10): near a steady state its own magnitude is no
    # yardstick for rounding, so the bar is relative to max(|R|, 1) as in the other R tests
    assert np.abs(R.cpu().numpy() - Ro).max() <= 1e-12 * max(np.abs(Ro).max(), 1.0)
    J = np.transpose(s.jacobian(U, R, rn).cpu().numpy(), (3, 0, 1, 2))
    Jo = o.jacobian(U0, nb=3)
    assert np.abs(J - Jo).max() <= 1e-12 * np.abs(Jo).max()
    st, _ = s.newton_solve(U)
    Uo, ito, reso, _ = o.newton_solve()
    err = np.abs(U.cpu().numpy() - Uo).max()
    print(f"cfg2-sub N=12800: gpu {st.iters} it res {st.res:.2e}; oracle {ito} it res {reso:.2e}; "
          f"|dU| {err:.2e}")
    assert st.status == 0 and reso < 1e-10
    assert err <= 1e-10


def test_batch_results_bitwise_equal_alone_and_in_mix():
    from paper_2505_10857_amd import BatchSolver1D
    probs = [config1(0), config4_instance(1), config1(5), config4_instance(2)]
    alone = []
    for p in probs:
        b = BatchSolver1D([p], device=DEV)
        Us = b.states()
        r = b.solve(Us, use_graph=False)
        alone.append((Us[0].cpu().numpy(), r[0]))
    mix = BatchSolver1D(probs, device=DEV)
    Us = mix.states()
    rs = mix.solve(Us, use_graph=True)
    for k in range(len(probs)):
        assert rs[k][0] == alone[k][1][0]
        assert np.array_equal(Us[k].cpu().numpy(), alone[k][0])
        assert rs[k][1] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32mg"])
def test_state_at_roundoff_floor_matches_oracle(precision):
    """Both forms iterated to the round-off floor (tol 1e-13) against the FP64 oracle iterated
    the same way: FP64 within 1e-10, FP32 multigrid within 1e-9."""
    from paper_2505_10857_amd import NMG_FP32_MG, NMG_FP64
    prec = NMG_FP32_MG if precision == "fp32mg" else NMG_FP64
    bar = 1e-9 if precision == "fp32mg" else 1e-10
    for prob in (config1(1), config4_instance(5)):
        s = _solver(prob, precision=prec, tol=1e-13, n_max=5000)
        U = s.state()
        st, _ = s.newton_solve(U)
        # the FP64 oracle iterated to its round-off floor
        o = oracle.Oracle1D(prob)
        Uo, ito, reso, _ = o.newton_solve(tol=1e-13, n_max=5000)
        err = np.abs(U.cpu().numpy() - Uo).max()
        print(f"{prob.name} {precision}: {st.iters} it res {st.res:.2e} vs oracle {ito} it "
              f"res {reso:.2e}: |dU| {err:.2e}")
        assert st.status == 0
        assert err <= bar


def test_nonfinite_state_is_reported():
    from paper_2505_10857_amd import NMG_ENONFINITE
    prob = config1(0)
    s = _solver(prob)
    U = s.state()
    U[0, 50] = -1.0          # negative depth: sqrt of a negative number in the flux
    st, _ = s.newton_solve(U)
    assert st.status == NMG_ENONFINITE


def test_full_batch_newton_steps_equal_solo_and_repeat():
    """The benchmark batch (256 instances of the N = 12800 hump, 8 levels): far more tiles than
    the GPU holds at once, so neighbouring tiles of one launch run at different times.  Two
    Newton steps of the batch, with and without the graph, equal those of each sampled instance
    solved alone, bit for bit, and repeat bit for bit."""
    from paper_2505_10857_amd import BatchSolver1D
    from swe_workloads import config2
    probs = [config2(i, "sub", n=12800, levels=8) for i in range(256)]

    def two_steps(ps, use_graph):
        b = BatchSolver1D(ps, device=DEV)
        Us = b.states()
        b.begin(Us)
        b.steps(2, use_graph=use_graph)
        torch.cuda.synchronize()
        return [u.cpu().numpy() for u in Us]

    a = two_steps(probs, False)
    g = two_steps(probs, True)
    a2 = two_steps(probs, False)
    for k in range(256):
        assert np.array_equal(a[k], a2[k]), f"instance {k}: batch not repeatable"
        assert np.array_equal(a[k], g[k]), f"instance {k}: graph differs from launches"
    for k in (0, 1, 157, 255):
        solo = two_steps([probs[k]], False)[0]
        assert np.array_equal(a[k], solo), f"instance {k}: batch differs from solo"


def _oracle_floor(probs, tol=1e-13):
    """FP64 oracle solutions iterated to the round-off floor, on host threads (the oracle's C
    code runs without the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    oracle.lib()
    with ThreadPoolExecutor(max_workers=min(len(probs), 16)) as ex:
        return list(ex.map(lambda p: oracle.Oracle1D(p).newton_solve(tol=tol, n_max=5000), probs))


@pytest.mark.parametrize("seed", [0, 7])
def test_headline_size_at_roundoff_floor(seed):
    """The benchmark workload (hump, N = 12800, 8 levels) in FP64 and with FP32 multigrid,
    iterated to the round-off floor (res < 1e-13), against the FP64 oracle iterated the same
    way: within 1e-10 (FP64) and 1e-9 (FP32 multigrid).  The difference at the res < 1e-10
    termination of the benchmark is printed beside it."""
    from paper_2505_10857_amd import NMG_FP32_MG, NMG_FP64
    from swe_workloads import config2
    prob = config2(seed, "sub", n=12800, levels=8)
    (Uo, ito, reso, _), = _oracle_floor([prob])
    Ut, _, _, _ = oracle.Oracle1D(prob).newton_solve()
    for name, prec, bar in (("fp64", NMG_FP64, 1e-10), ("fp32mg", NMG_FP32_MG, 1e-9)):
        s = _solver(prob, precision=prec, tol=1e-13, n_max=5000)
        U = s.state()
        st, _ = s.newton_solve(U)
        err = np.abs(U.cpu().numpy() - Uo).max()
        s10 = _solver(prob, precision=prec)
        U10 = s10.state()
        s10.newton_solve(U10)
        err10 = np.abs(U10.cpu().numpy() - Ut).max()
        print(f"seed {seed} {name}: floor {st.iters} it res {st.res:.2e} (oracle {ito} it {reso:.2e}) "
              f"|dU| {err:.2e}; at res < 1e-10 termination |dU| {err10:.2e}")
        assert st.status == 0 and reso < 1e-13
        assert err <= bar


def test_full_uneven_batch_sampled_against_the_oracle():
    """The uneven batch at its full size and launch configuration (512 instances, N from 256 to
    16384, FP32 multigrid, HIP graph): every instance converges; then the same batch iterated to
    the round-off floor (res < 1e-13) agrees with the FP64 oracle's floor within the FP32-multigrid
    bar (1e-9) on a sample spanning the sizes: the two smallest (256 cells), two of the three
    largest (16384 cells) and two seeded picks in between."""
    import dataclasses
    from paper_2505_10857_amd import NMG_FP32_MG, BatchSolver1D
    from swe_workloads import config4_instance
    probs = [config4_instance(i) for i in range(512)]
    b = BatchSolver1D(probs, device=DEV, precision=NMG_FP32_MG)
    Us = b.states()
    st = b.solve(Us, use_graph=True)
    assert all(s[1] == 0 and s[2] < 1e-10 for s in st)
    by_n = sorted(range(512), key=lambda k: probs[k].n)
    rng = np.random.default_rng(12)
    sample = by_n[:2] + [k for k in by_n if probs[k].n == 16384][:2] + [int(k) for k in rng.choice(by_n[2:-3], 2, replace=False)]
    assert sum(probs[k].n == 16384 for k in sample) == 2
    fprobs = [dataclasses.replace(p, params=dataclasses.replace(p.params, tol=1e-13, n_max=5000)) for p in probs]
    bf = BatchSolver1D(fprobs, device=DEV, precision=NMG_FP32_MG)
    Uf = bf.states()
    stf = bf.solve(Uf, use_graph=True)
    ref = _oracle_floor([probs[k] for k in sample])
    for k, (Uo, ito, reso, _) in zip(sample, ref):
        err = np.abs(Uf[k].cpu().numpy() - Uo).max()
        print(f"instance {k} (N={probs[k].n}): floor |U - U_oracle| = {err:.2e}, steps {stf[k][0]} vs {ito}; "
              f"res {stf[k][2]:.1e} vs {reso:.1e}")
        assert stf[k][1] == 0 and reso < 1e-13
        assert err <= 1e-9
