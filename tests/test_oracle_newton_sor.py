"""Pins of the oracle's Newton-SOR (the reference solver of section 5.1.1, Table 2)."""
import numpy as np

from oracle import Oracle1D
from swe_workloads import e1_problem


def test_newton_sor_reaches_the_nmgm_solution_with_at_least_as_many_steps():
    """E1, 96 cells: Newton-SOR (symmetric lexicographic block SOR, <= 10 steps, l1 change
    1e-7) and NMGM-3 end at the same discrete solution; Table 2 has Newton-SOR needing more
    Newton iterations, and it never needs fewer here."""
    o = Oracle1D(e1_problem(96))
    U3, it3, r3, _ = o.newton_solve(tol=1e-12)
    Us, its, rs, _ = o.newton_solve(tol=1e-12, linear=1, smoother=1, sor_max=10, sor_tol=1e-7)
    assert r3 < 1e-12 and rs < 1e-12
    assert np.abs(U3 - Us).max() < 1e-9
    assert its >= it3


def test_inner_iteration_stops_on_the_change_norm():
    """A tolerance no change can reach leaves exactly one symmetric step per Newton step, the
    same as a step limit of one."""
    o = Oracle1D(e1_problem(96))
    a = o.newton_solve(n_max=6, linear=1, smoother=1, sor_max=10, sor_tol=1e300)
    b = o.newton_solve(n_max=6, linear=1, smoother=1, sor_max=1, sor_tol=0.0)
    assert np.array_equal(a[0], b[0])
    c = o.newton_solve(n_max=6, linear=1, smoother=1, sor_max=10, sor_tol=0.0)
    assert not np.array_equal(a[0], c[0])
