"""The non-matching block-on-block generator: symmetry, rigid-body modes, mortar weights
that reproduce linear fields, and the filter-space size of the paper's meshes."""
import numpy as np
import scipy.sparse as sp

from amgf_inputs import make_block_on_block, make_config, contact_load_and_gap, lumped_masses


def _K(p):
    return sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(p.n, p.n)).tocsr()


def test_stiffness_symmetric_and_rigid_modes():
    """K is bitwise symmetric and annihilates rigid motions of each body on every node row
    whose stencil touches no Dirichlet DOF (the scaled top-body stiffness included)."""
    p = make_block_on_block(6, 5)
    K = _K(p)
    assert abs(K - K.T).max() == 0.0
    free_node = p.free.reshape(-1, 3).all(axis=1)
    Kb = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr))
    inner = np.array([free_node[Kb.indices[Kb.indptr[i]:Kb.indptr[i + 1]]].all()
                      for i in range(p.n_nodes)])
    rows = np.repeat(inner, 3)
    x, y, z = p.coords[:, 0], p.coords[:, 1], p.coords[:, 2]
    modes = []
    for comp in range(3):
        t = np.zeros(p.n)
        t[comp::3] = 1.0
        modes.append(t)
    rot = np.zeros(p.n)
    rot[0::3], rot[1::3] = -y, x                       # rotation about z
    modes.append(rot)
    for v in modes:
        assert np.abs((K @ v)[rows]).max() < 1e-12


def test_mortar_rows_reproduce_linear_gap_fields():
    """J applied to u_z = alpha + beta x + gamma y on both faces is zero (the bilinear
    weights reproduce affine fields), and each row's mortar weights sum to one."""
    p = make_block_on_block(8, 7)
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, p.n))
    u = np.zeros(p.n)
    x, y = p.coords[:, 0], p.coords[:, 1]
    u[2::3] = 0.3 - 0.7 * x + 1.1 * y
    assert np.abs(J @ u).max() < 1e-13
    for k in range(p.m):
        v = p.J_val[p.J_rowptr[k]:p.J_rowptr[k + 1]]
        assert abs(v.sum()) < 1e-14 and v[-1] == 1.0
        assert np.all(np.diff(p.J_col[p.J_rowptr[k]:p.J_rowptr[k + 1]]) > 0)


def test_filter_space_ratio_like_table1():
    """n_c = 3 x (non-mortar nodes + touched mortar nodes); m and n_c of B1/B2 are within
    a few percent of Table 1's Mesh 1/2 (81, 348 and 289, 1092)."""
    for name, m_ref, nc_ref in (("B1", 81, 348), ("B2", 289, 1092)):
        p = make_config(name)
        nodes = np.unique(p.J_col // 3)
        n_c = 3 * len(nodes)
        assert p.m == m_ref
        assert abs(n_c - nc_ref) <= 0.05 * nc_ref, (name, n_c)


def test_load_gap_and_masses():
    p = make_config("B1")
    f, g0 = contact_load_and_gap(p, pressure=0.05)
    Ms, Mu = lumped_masses(p)
    assert abs(f.sum() + 0.05 * 0.25) < 1e-14           # pressure times the top area 0.5^2
    assert abs(Ms.sum() - 0.25) < 1e-14                   # interface area of the top block
    assert abs(Mu[::3].sum() - (1.0 + 0.125)) < 1e-12     # volumes 1 + 0.5^3
    assert g0.min() >= 0.0 and g0.shape == (p.m,)
