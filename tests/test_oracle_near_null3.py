"""Translations-only near-null space (near_null = 3) in the oracle: the tentative prolongator
in closed form (normalised aggregate indicators per displacement component, R = sqrt(k) I
on unconstrained aggregates), the Galerkin chain with 3x3 coarse blocks, Definition 5.3 and
PCG convergence."""
import numpy as np

from amgf_inputs import make_config
from oracle.amgf_oracle import group_members
from oracle_util import build, dense_of, small_problem


def test_tentative_prolongator_closed_form():
    p = make_config("C1")
    o = build(p, near_null=3, coarse_max_nodes=8)
    lev = o.levels[0]
    members, off = group_members(lev.agg, lev.n_agg)
    Pt = lev.Pt.todense()
    dec = lev.decoupled.reshape(-1, 3)
    assert Pt.shape == (p.n, 3 * lev.n_agg)
    for J in range(lev.n_agg):
        nodes = members[off[J]:off[J + 1]]
        for q in range(3):
            live = nodes[~dec[nodes, q]]
            col = np.zeros(p.n)
            col[3 * live + q] = 1.0 / np.sqrt(len(live)) if len(live) else 0.0
            assert np.allclose(Pt[:, 3 * J + q], col, atol=1e-15)
            assert lev.dead[J, q] == (len(live) == 0)
            assert abs(lev.R[J][q, q] - np.sqrt(len(live))) <= 1e-14 * max(1, len(live))
        assert np.allclose(np.triu(lev.R[J], 1), 0.0)
    for l in range(o.nlev - 1):
        assert o.levels[l + 1].A.br == 3
        P = o.levels[l].P.todense()
        dead = o.levels[l].dead.ravel().astype(float)
        Ac = P.T @ o.levels[l].A.todense() @ P + np.diag(dead)
        assert np.abs(o.levels[l + 1].A.todense() - Ac).max() <= 1e-12 * np.abs(Ac).max()


def test_definition_53_and_pcg():
    p = small_problem(N=3, D_log10=(0.0, 3.0))
    o = build(p, near_null=3, coarse_max_nodes=8)
    assert o.nlev >= 2
    n = o.n
    A = o.S.todense()
    I = np.eye(n)
    M = dense_of(o.apply, n)
    B = dense_of(o.vcycle, n)
    Pw = I[:, o.Ic]
    F = I - Pw @ np.linalg.solve(Pw.T @ A @ Pw, Pw.T @ A)
    assert np.abs((I - M @ A) - (I - B @ A) @ F @ (I - B @ A)).max() <= 1e-8
    assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
    r = o.pcg(p.b)
    assert r.converged and np.linalg.norm(A @ r.x - p.b) <= 1e-6 * np.linalg.norm(p.b)
    # the richer rigid-body space needs no more iterations on the same problem
    r6 = build(p, coarse_max_nodes=8).pcg(p.b)
    assert r6.iterations <= r.iterations
