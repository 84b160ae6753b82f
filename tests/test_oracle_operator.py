"""Pins of the oracle's Schur operator A = K + J^T D J (Sec. 3) and strength graph."""
import numpy as np
import pytest

from amgf_inputs import make_config
from oracle import strength_graph
from oracle_util import build, small_problem, J_dense, K_dense


@pytest.fixture(scope="module")
def c1():
    p = make_config("C1")
    return p, build(p)


def test_operator_equals_dense_definition(c1):
    p, o = c1
    S = o.S.todense()
    ref = K_dense(p) + J_dense(p).T @ np.diag(p.D) @ J_dense(p)
    scale = np.abs(ref).max(axis=1, keepdims=True)
    assert np.abs(S - ref).max() <= 0 or (np.abs(S - ref) <= 4e-16 * scale).all()


def test_operator_bitwise_symmetric_and_pattern(c1):
    p, o = c1
    S = o.S.todense()
    assert np.array_equal(S, S.T)
    # J^T D J adds blocks only between interface nodes (<= n_c x n_c, Sec. 4)
    extra = o.S.nnzb - o.K0.nnzb
    assert extra > 0
    nodes = np.unique(p.J_col // 3)
    assert 3 * len(nodes) == o.n_c == 6 * p.m


def test_operator_apply_matches_split_form(c1):
    p, o = c1
    rng = np.random.default_rng(0)
    v = rng.standard_normal(p.n)
    J = J_dense(p)
    split = K_dense(p) @ v + J.T @ (p.D * (J @ v))
    got = o.A_apply(v)
    assert np.abs(got - split).max() <= 1e-14 * np.abs(split).max()


def test_operator_spd_small():
    p = small_problem(N=2)
    o = build(p)
    ev = np.linalg.eigvalsh(o.S.todense())
    assert ev[0] > 0


def test_strength_graph_symmetric_and_matches_norm_test(c1):
    p, o = c1
    A = o.S
    rp, col, w = strength_graph(A, 0.08)
    n = A.nrows
    rows = np.repeat(np.arange(n), np.diff(rp))
    E = set(zip(rows.tolist(), col.tolist()))
    assert all((b, a) in E for a, b in E)
    assert all(a != b for a, b in E)
    # independent evaluation with numpy's Frobenius norm: ||A_ab|| >= theta sqrt(||A_aa|| ||A_bb||)
    fro = np.linalg.norm(A.val.reshape(A.nnzb, -1), axis=1)
    dp = A.diag_pos()
    r = A.row_index()
    ratio = fro / np.sqrt(fro[dp[r]] * fro[dp[A.col]])
    tpos = A.find(A.col, r)
    both = np.minimum(ratio, ratio[tpos])
    clear = np.abs(both - 0.08) > 1e-9
    strong_ref = (both >= 0.08) & (r != A.col)
    got = np.zeros(A.nnzb, bool)
    got[A.find(rows, col)] = True
    assert (got[clear] == strong_ref[clear]).all()
    # Dirichlet-clamped nodes (bottom face) have no strong neighbour
    assert (np.diff(rp)[: (p.N + 1) ** 2] == 0).all()
