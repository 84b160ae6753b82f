"""Pins of the oracle's numeric re-setup for a new barrier diagonal (same K and J)."""
import numpy as np
import pytest

from oracle_util import build, dense_of, small_problem


@pytest.fixture(scope="module")
def pair():
    p = small_problem(N=3, D_log10=(0.0, 3.0))
    rng = np.random.default_rng(99)
    D2 = 10.0 ** rng.uniform(0.0, 3.0, p.m)     # new draw, same range as the base problem
    return p, D2


def test_same_D_reproduces_setup(pair):
    p, _ = pair
    o = build(p)
    ref = build(p)
    o.update_D(p.D.copy())
    r = np.random.default_rng(1).standard_normal(o.n)
    assert np.array_equal(o.vcycle(r), ref.vcycle(r))
    assert np.array_equal(o.apply(r), ref.apply(r))


def test_updated_hierarchy_is_galerkin_and_definition_5_3(pair):
    p, D2 = pair
    o = build(p, coarse_max_nodes=8, max_levels=2)
    o.update_D(D2)
    A = o.S.todense()
    # A is the new Schur complement K + J^T D2 J
    from oracle_util import J_dense, K_dense
    J = J_dense(p)
    assert np.abs(A - (K_dense(p) + J.T @ (D2[:, None] * J))).max() <= 1e-12 * np.abs(A).max()
    lev = o.levels[0]
    P = lev.P.todense()
    Ac = o.levels[1].A.todense()
    Ac_ref = P.T @ A @ P + np.diag(lev.dead.ravel().astype(float))
    assert np.abs(Ac - Ac_ref).max() <= 1e-10 * np.abs(Ac_ref).max()
    # two-grid formula with the kept P and the new operator
    n = o.n
    I = np.eye(n)
    W = np.diag(lev.w)
    E = (I - W @ A) @ (I - P @ np.linalg.solve(Ac, P.T @ A)) @ (I - W @ A)
    B = dense_of(o.vcycle, n)
    Bref = (I - E) @ np.linalg.inv(A)
    assert np.abs(B - Bref).max() <= 1e-8 * np.abs(Bref).max()
    # Definition 5.3 with the new filter matrix
    M = dense_of(o.apply, n)
    Pf = np.zeros((n, o.n_c))
    Pf[o.Ic, np.arange(o.n_c)] = 1.0
    Aw = Pf.T @ A @ Pf
    E5 = (I - B @ A) @ (I - Pf @ np.linalg.solve(Aw, Pf.T @ A)) @ (I - B @ A)
    assert np.abs((I - M @ A) - E5).max() <= 1e-7


def test_pcg_after_update_solves_new_system(pair):
    p, D2 = pair
    o = build(p)
    o.update_D(D2)
    x = o.pcg(p.b)
    xs = np.linalg.solve(o.S.todense(), p.b)
    assert x.converged
    assert np.linalg.norm(x.x - xs) <= 1e-8 * np.linalg.norm(xs)
