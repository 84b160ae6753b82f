"""Shared helpers for the oracle pins (dense matrices of small problems)."""
import numpy as np

from amgf_inputs import make_two_block
from oracle import OracleAMGF, OracleOptions


def build(p, **kw):
    return OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col,
                      p.J_val, p.D, p.coords, OracleOptions(**kw))


def dense_of(apply, n):
    E = np.eye(n)
    return np.stack([apply(E[:, j]) for j in range(n)], axis=1)


def small_problem(N=3, D_log10=(0.0, 6.0), seed=7, **kw):
    return make_two_block(N, D_log10=D_log10, D_seed=seed, rhs_seed=seed + 1, **kw)


def J_dense(p):
    J = np.zeros((p.m, p.n))
    for k in range(p.m):
        s, e = p.J_rowptr[k], p.J_rowptr[k + 1]
        J[k, p.J_col[s:e]] = p.J_val[s:e]
    return J


def K_dense(p):
    import scipy.sparse as sp
    return sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(p.n, p.n)).toarray()


def extended_solution(p, E=None, steps=8):
    """Solution of (K + diag(E) + J^T D J) x = b to far below 1e-12, independent of the
    oracle's solver: a sparse LU of the FP64 matrix, then iterative refinement with the
    residual b - (K + diag(E)) x - J^T (D (J x)) evaluated in extended precision (numpy
    longdouble) until the correction no longer changes x."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(p.n, p.n)).tocsr()
    if E is not None:
        K = K + sp.diags(np.asarray(E, np.float64))
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, p.n))
    lu = spla.splu((K + J.T @ sp.diags(p.D) @ J).tocsc())
    LD = np.longdouble
    KL, JL, DL, bL = K.astype(LD), J.astype(LD), p.D.astype(LD), p.b.astype(LD)
    x = lu.solve(p.b).astype(LD)
    for _ in range(steps):
        r = bL - (KL @ x + JL.T @ (DL * (JL @ x)))
        d = lu.solve(r.astype(np.float64))
        x = x + d.astype(LD)
        if np.linalg.norm(d) <= 1e-15 * np.linalg.norm(x.astype(np.float64)):
            break
    return x.astype(np.float64)
