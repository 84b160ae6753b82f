"""Pins of the oracle's cycle option (cycle_gamma = number of visits of the next level per
coarse correction; 2 = W-cycle).  The W-cycle is not in the paper, which uses V-cycles;
the pins tie the recursion to closed forms of the two-level iteration."""
import numpy as np
import pytest

from oracle_util import build, dense_of, small_problem


@pytest.fixture(scope="module")
def prob():
    return small_problem(N=4, D_log10=(0.0, 3.0))


def _two_grid(o, b, coarse):
    """One cycle on level 0 with the coarse correction `coarse(rc)` (l1-Jacobi V(1,1))."""
    lev = o.levels[0]
    A, P = lev.A.csr(), lev.P.csr()
    x = o.smooth(0, b, np.zeros_like(b))
    x = x + P @ coarse(P.T @ (b - A @ x))
    return o.smooth(0, b, x)


def test_three_levels_gamma2_is_the_two_fold_coarse_iteration(prob):
    """gamma = 2: the coarse correction is (2 B_1 - B_1 A_1 B_1) P^T r, B_1 the level-1
    V-cycle (exact coarsest solve below it)."""
    o = build(prob, coarse_max_nodes=8, cycle_gamma=2)
    assert o.nlev == 3
    A1 = o.levels[1].A.csr()
    rng = np.random.default_rng(3)
    b = rng.standard_normal(o.levels[0].A.nrows * 3)

    def two_fold(rc):
        y = o.vcycle(rc, 1)
        return 2 * y - o.vcycle(A1 @ y, 1)

    w = o.vcycle(b)
    ref = _two_grid(o, b, two_fold)
    assert np.linalg.norm(w - ref) <= 1e-12 * np.linalg.norm(ref)


def test_many_visits_approach_the_exact_coarse_solve(prob):
    """As gamma grows the coarse correction converges to A_1^{-1} P^T r (the level-1 cycle
    is a convergent iteration), so the cycle tends to the two-grid cycle with an exact
    level-1 solve, formed here with a dense solve.  The level-1 V-cycle contracts by 0.975
    per visit on this case (contact modes), hence the many visits."""
    o = build(prob, coarse_max_nodes=8, cycle_gamma=1500)
    assert o.nlev == 3
    A1 = o.levels[1].A.todense()
    rng = np.random.default_rng(4)
    b = rng.standard_normal(o.levels[0].A.nrows * 3)
    w = o.vcycle(b)
    ref = _two_grid(o, b, lambda rc: np.linalg.solve(A1, rc))
    assert np.linalg.norm(w - ref) <= 1e-9 * np.linalg.norm(ref)
    o1 = build(prob, coarse_max_nodes=8)
    assert np.linalg.norm(o1.vcycle(b) - ref) > 1e-4 * np.linalg.norm(ref)


def test_gamma_is_idle_above_the_coarsest_level_and_keeps_symmetry(prob):
    o1 = build(prob, coarse_max_nodes=8, max_levels=2)
    o2 = build(prob, coarse_max_nodes=8, max_levels=2, cycle_gamma=2)
    assert o1.nlev == o2.nlev == 2
    rng = np.random.default_rng(5)
    b = rng.standard_normal(o1.levels[0].A.nrows * 3)
    assert np.array_equal(o1.vcycle(b), o2.vcycle(b))
    o = build(prob, coarse_max_nodes=8, cycle_gamma=2)
    n = o.levels[0].A.nrows * 3
    B = dense_of(o.vcycle, n)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_w_cycle_pcg_needs_fewer_iterations(prob):
    from amgf_inputs import make_config
    p = make_config("C1")
    its = {g: build(p, coarse_max_nodes=16, cycle_gamma=g).pcg(p.b).iterations for g in (1, 2)}
    assert its[2] < its[1], its
