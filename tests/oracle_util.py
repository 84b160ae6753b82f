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
