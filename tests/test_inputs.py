"""Pins of the synthetic two-body problem (generator only, no solver arithmetic)."""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from amgf_inputs import make_two_block, make_config, q1_element_matrices, ip_sequence_D
from amgf_inputs.twoblock import _body_stiffness

GOLD = os.path.join(os.path.dirname(__file__), "golden", "table1_two_block.txt")


def _csr(rp, c, v, nn):
    return sp.bsr_matrix((v, c, rp), shape=(3 * nn, 3 * nn)).tocsr()


def _rbm(X):
    n = len(X)
    R = np.zeros((3 * n, 6))
    for a in range(3):
        R[a::3, a] = 1
    x, y, z = X.T
    R[1::3, 3] = -z; R[2::3, 3] = y
    R[0::3, 4] = z; R[2::3, 4] = -x
    R[0::3, 5] = -y; R[1::3, 5] = x
    return R


@pytest.mark.parametrize("N", [1, 2, 3])
def test_free_body_stiffness_null_space_is_rigid_motions(N):
    nn = (N + 1) ** 3
    rp, c, v = _body_stiffness(N, 2.0, 0.3, np.ones(3 * nn, bool))
    K = _csr(rp, c, v, nn).toarray()
    assert np.array_equal(K, K.T)
    idx = np.arange(N + 1)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], 1) / N
    assert np.abs(K @ _rbm(X)).max() < 1e-13
    ev = np.linalg.eigvalsh(K)
    assert (np.abs(ev) < 1e-10 * ev.max()).sum() == 6
    assert ev.min() > -1e-12


def test_patch_test_linear_field_gives_zero_interior_force():
    N = 3
    nn = (N + 1) ** 3
    rp, c, v = _body_stiffness(N, 1.0, 0.25, np.ones(3 * nn, bool))
    K = _csr(rp, c, v, nn)
    idx = np.arange(N + 1)
    k, j, i = np.meshgrid(idx, idx, idx, indexing="ij")
    X = np.stack([i.ravel(), j.ravel(), k.ravel()], 1) / N
    G = np.array([[0.1, 0.2, 0.3], [0.4, -0.5, 0.6], [0.7, 0.8, -0.9]])
    f = (K @ (X @ G.T).ravel()).reshape(-1, 3)
    interior = ((X > 0) & (X < 1)).all(1)
    assert np.abs(f[interior]).max() < 1e-14


def test_element_matrix_scaling_and_symmetry():
    Kl, Km = q1_element_matrices()
    for M in (Kl, Km):
        assert np.array_equal(M, M.transpose(1, 0, 3, 2))
    # uniaxial strain energy of the unit cube: u = (x, 0, 0) -> lam/2 + mu
    X = np.array([[l & 1, (l >> 1) & 1, (l >> 2) & 1] for l in range(8)], float)
    u = np.zeros((8, 3)); u[:, 0] = X[:, 0]
    e_l = np.einsum("ap,abpq,bq->", u, Kl, u)
    e_m = np.einsum("ap,abpq,bq->", u, Km, u)
    assert abs(e_l - 1.0) < 1e-14 and abs(e_m - 2.0) < 1e-14


def test_two_block_structure_and_dirichlet():
    p = make_two_block(3)
    K = _csr(p.K_rowptr, p.K_col, p.K_val, p.n_nodes)
    Kd = K.toarray()
    assert np.array_equal(Kd, Kd.T)
    cons = np.nonzero(~p.free)[0]
    for i in cons:
        row = Kd[i].copy(); d = row[i]; row[i] = 0
        assert d > 0 and not row.any()
    assert (p.b[cons] == 0).all()
    nb = (p.N + 1) ** 3
    assert not Kd[:3 * nb, 3 * nb:].any()        # block diagonal per body
    # roller: top face z DOFs free, x/y fixed
    top = nb + p.N * (p.N + 1) ** 2 + np.arange((p.N + 1) ** 2)
    assert p.free[3 * top + 2].all() and not p.free[3 * top].any()


def test_gap_jacobian_rows():
    p = make_two_block(4)
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, p.n))
    assert np.allclose(J @ np.ones(p.n), 0)
    tz = np.zeros(p.n); tz[2::3] = 1.0
    assert np.abs(J @ tz).max() == 0.0            # common z-translation opens no gap
    assert np.linalg.matrix_rank(J.toarray()) == p.m
    assert (np.diff(p.J_rowptr) == 5).all()
    for k in range(p.m):
        c = p.J_col[p.J_rowptr[k]:p.J_rowptr[k + 1]]
        assert (np.diff(c) > 0).all() and (c % 3 == 2).all()


def test_sizes_match_configs():
    sizes = {"C1": (4374, 81, 31250), "C2": (215622, 1089, 1825346)}
    for name, (n, m, nnzb) in sizes.items():
        p = make_config(name)
        assert (p.n, p.m, p.nnzb) == (n, m, nnzb)
    # nnzb formula 2 (3N+1)^3 of the 27-point stencil: C3 and C5 values without building
    for N, nnzb in [(64, 14378114), (128, 114133250)]:
        assert 2 * (3 * N + 1) ** 3 == nnzb


def test_contact_rows_follow_table1_refinement():
    """m of the N = 8 * 2^(k-1) meshes equals Table 1's m_max of Mesh k, and n_c / n
    follow the surface-to-volume trend of Sec. 4 (ratios -> 4 and 8)."""
    rows = np.loadtxt(GOLD, comments="#")
    for mesh, n, ncmax, mmax, *_ in rows:
        N = 8 * 2 ** (int(mesh) - 1)
        assert (N + 1) ** 2 == mmax
    nc = [6 * (N + 1) ** 2 for N in (8, 16, 32, 64, 128, 256)]
    n = [6 * (N + 1) ** 3 for N in (8, 16, 32, 64, 128, 256)]
    r_nc = np.diff(np.log(nc)) / np.log(2)
    r_n = np.diff(np.log(n)) / np.log(2)
    assert (np.diff(r_nc) > 0).all() and abs(r_nc[-1] - 2) < 0.02
    assert abs(r_n[-1] - 3) < 0.02
    paper = np.diff(np.log(rows[:, 2])) / np.log(2)
    assert (np.diff(paper) > 0).all() and abs(paper[-1] - 2) < 0.02


def test_ip_sequence():
    D1 = ip_sequence_D(100, 1)
    D20 = ip_sequence_D(100, 20)
    mu = 0.1 * 0.3 ** 19
    assert D1.min() >= 0.1 * (1 - 1e-12) and D1.max() <= 10.0 * (1 + 1e-12)
    assert D20.min() >= mu * (1 - 1e-9) and D20.max() <= 1.0 / mu * (1 + 1e-9)
    # same active set through the sequence: the order of D is preserved
    assert (np.argsort(D1) == np.argsort(D20)).all()


def test_renumbered_problem_is_the_same_operator():
    """renumber_nodes permutes nodes only: P K P^T, J P^T, P b, with valid sorted inputs
    and a bandwidth beyond 16-bit block-column offsets."""
    import scipy.sparse as sp
    from amgf_inputs import make_two_block, renumber_nodes
    p = make_two_block(28, D_log10=(0.0, 6.0), D_seed=3, rhs_seed=4)
    q = renumber_nodes(p, seed=5)
    n = p.n
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(n, n)).tocsr()
    Kq = sp.bsr_matrix((q.K_val, q.K_col, q.K_rowptr), shape=(n, n)).tocsr()
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, n))
    Jq = sp.csr_matrix((q.J_val, q.J_col, q.J_rowptr), shape=(q.m, n))
    perm = q.meta["node_perm"]
    assert np.array_equal(np.sort(perm), np.arange(p.n_nodes))
    node_q_to_p = np.argsort(perm)
    assert np.array_equal(q.coords, p.coords[node_q_to_p])
    dof = (3 * node_q_to_p[:, None] + np.arange(3)[None, :]).ravel()
    assert (Kq - K[dof][:, dof]).count_nonzero() == 0
    assert (Jq - J[:, dof]).count_nonzero() == 0
    assert np.array_equal(q.b, p.b[dof]) and np.array_equal(q.free, p.free[dof])
    for k in range(q.m):
        c = q.J_col[q.J_rowptr[k]:q.J_rowptr[k + 1]]
        assert np.all(np.diff(c) > 0)
    for a in range(0, q.n_nodes, 997):
        c = q.K_col[q.K_rowptr[a]:q.K_rowptr[a + 1]]
        assert np.all(np.diff(c) > 0)
    rows = np.repeat(np.arange(q.n_nodes), np.diff(q.K_rowptr))
    assert np.abs(q.K_col - rows).max() > 32767
