"""Bound-constraint barrier terms (Remark 3.1) in the oracle: the operator against the
stacked Jacobian [J; I; -I] written out, the numeric re-setup against the construction,
and the Galerkin property and Definition 5.3 after a change of both barrier terms."""
import numpy as np
import scipy.sparse as sp

from amgf_inputs import make_two_block
from oracle import OracleAMGF, OracleOptions


def _p():
    return make_two_block(3, D_log10=(0.0, 4.0))


def _E(p, seed, lo=-2.0, hi=3.0):
    rng = np.random.default_rng(seed)
    E = 10.0 ** rng.uniform(lo, hi, p.n)
    E[rng.uniform(size=p.n) < 0.3] = 0.0                  # bounds on part of the DOFs only
    return E


def _oracle(p, E=None, **kw):
    return OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                      p.D, p.coords, OracleOptions(**kw), E=E)


def test_operator_is_K_plus_stacked_barrier():
    p = _p()
    E = _E(p, 1)
    rng = np.random.default_rng(2)
    split = rng.uniform(size=p.n)
    E_lo, E_up = split * E, (1 - split) * E                # D~ = diag(D, D_lo, D_up)
    n = p.n
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, n))
    Jt = sp.vstack([J, sp.identity(n), -sp.identity(n)]).tocsr()
    Dt = np.concatenate([p.D, E_lo, E_up])
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(n, n)).toarray()
    ref = K + (Jt.T @ sp.diags(Dt) @ Jt).toarray()
    S = _oracle(p, E).S.todense()
    assert np.abs(S - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.array_equal(S, S.T)


def test_update_with_same_terms_reproduces_setup():
    p = _p()
    E = _E(p, 3)
    a = _oracle(p, E, coarse_max_nodes=8)
    b = _oracle(p, E, coarse_max_nodes=8)
    b.update_barrier(p.D, E)
    assert a.nlev == b.nlev >= 2
    for la, lb in zip(a.levels, b.levels):
        assert np.array_equal(la.A.val, lb.A.val) and np.array_equal(la.K.val, lb.K.val)
    r = np.random.default_rng(4).standard_normal(a.n)
    assert np.array_equal(a.apply(r), b.apply(r))


def test_galerkin_and_definition_after_update():
    p = _p()
    o = _oracle(p, _E(p, 5), coarse_max_nodes=8)
    # moderate barrier ranges keep the dense identity check below at rounding level
    D2 = 10.0 ** np.random.default_rng(6).uniform(0.0, 3.0, p.m)
    E2 = _E(p, 7, -1.0, 3.0)
    o.update_barrier(D2, E2)
    # A_0 is the new operator, and every coarse operator is the Galerkin product
    p2 = make_two_block(3, D=D2)
    fresh = OracleAMGF(p2.n_nodes, p2.K_rowptr, p2.K_col, p2.K_val, p2.J_rowptr, p2.J_col,
                       p2.J_val, D2, p2.coords, OracleOptions(coarse_max_nodes=8), E=E2)
    assert np.array_equal(o.S.todense(), fresh.S.todense())
    for l in range(o.nlev - 1):
        P = o.levels[l].P.todense()
        G = P.T @ o.levels[l].A.todense() @ P
        # dead coarse DOFs (zero prolongator columns) carry a unit diagonal instead of 0
        A1 = o.levels[l + 1].A.todense() - np.diag(o.levels[l].dead.reshape(-1) * 1.0)
        assert np.abs(G - A1).max() <= 1e-10 * np.abs(A1).max(), l
    # Definition 5.3 with the updated operator: I - M A = (I - B A)(I - P A_w^-1 P^T A)(I - B A)
    n = o.n
    A = o.S.todense()
    I = np.eye(n)
    M = np.column_stack([o.apply(e) for e in I])
    B = np.column_stack([o.vcycle(e) for e in I])
    Ic = o.Ic
    Pw = I[:, Ic]
    Aw = Pw.T @ A @ Pw
    F = I - Pw @ np.linalg.solve(Aw, Pw.T @ A)
    lhs = I - M @ A
    rhs = (I - B @ A) @ F @ (I - B @ A)
    assert np.abs(lhs - rhs).max() <= 1e-8
