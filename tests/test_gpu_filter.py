"""GPU parity of the filtering-space solve w_c = A_w^{-1} r_c (Sec. 5.1): the
nested-dissection multifrontal factor against the oracle's direct solve of the same A_w."""
import numpy as np
import pytest

from gpu_util import gpu, oracle, problem, rel

pytestmark = pytest.mark.gpu


def _check_solve(name, **opts):
    o = oracle(name, **({"Ic": tuple(int(i) for i in opts["Ic"])} if "Ic" in opts else {}))
    h = gpu(name, **opts)
    rng = np.random.default_rng(5)
    Aw = o.S.csr()[o.Ic][:, o.Ic]
    anorm = abs(Aw).sum(axis=1).max()
    for trial in range(2):
        r = rng.standard_normal(o.n_c)
        w = h.filter_solve(r).cpu().numpy()
        w2 = h.filter_solve(r).cpu().numpy()
        wo = o.filter_solve(r)
        # normwise backward error |r - A w| / (|A| |w| + |r|) (infinity norms): a direct
        # Cholesky solve keeps it at a modest multiple of the unit roundoff
        eta = np.abs(r - Aw @ w).max() / (anorm * np.abs(w).max() + np.abs(r).max())
        eta_o = np.abs(r - Aw @ wo).max() / (anorm * np.abs(wo).max() + np.abs(r).max())
        err = rel(w, wo)
        print(f"{name} n_c={o.n_c}: backward error {eta:.2e} (oracle {eta_o:.2e}), "
              f"rel diff {err:.2e}")
        assert np.array_equal(w, w2)          # fixed summation order: reproducible
        assert eta <= 1e-14
        # both solves are backward stable; their difference is bounded by the condition
        # number of A_w (D spans ten decades here) times the backward errors
        assert err <= 1e-4
    h.close()


@pytest.mark.parametrize("name", ["C1", "N12", "C2"])
def test_filter_solve_matches_oracle(name):
    _check_solve(name)


def test_filter_solve_dof_subset():
    """A user filtering space that is not closed over nodes (z components of the contact
    nodes only) takes the scalar-graph path of the ordering."""
    p = problem("C1")
    nodes = np.unique(p.J_col // 3)
    Ic = (3 * nodes + 2).astype(np.int32)
    _check_solve("C1", Ic=Ic)


def test_apply_with_dof_subset_matches_oracle():
    p = problem("C1")
    nodes = np.unique(p.J_col // 3)
    Ic = (3 * nodes + 2).astype(np.int32)
    o = oracle("C1", Ic=tuple(int(i) for i in Ic))
    h = gpu("C1", Ic=Ic)
    rng = np.random.default_rng(8)
    r = rng.standard_normal(o.n)
    e = rel(h.apply(r).cpu().numpy(), o.apply(r))
    print(f"apply with z-only I_c: rel {e:.2e}")
    assert e < 5e-8
    h.close()


def test_filter_solve_c3_tree():
    """C3 (N = 64, 25,350 filter DOFs): a tree deep and wide enough that its leaf depths
    run one row group per wavefront and its shallow depths split each row group's columns
    over the four wavefronts of a workgroup.  I_c and A_w = S[I_c, I_c] are formed here from
    the input arrays (S = K + J^T D J with scipy); backward error and reproducibility."""
    import scipy.sparse as sp
    from amgf_inputs import make_config
    from paper_2505_18576_amd import AMGF
    p = make_config("C3")
    n = 3 * p.n_nodes
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(n, n)).tocsr()
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(len(p.D), n))
    nodes = np.unique(p.J_col // 3)
    Ic = (3 * nodes[:, None] + np.arange(3)).ravel()
    Jc = J[:, Ic]
    Aw = (K[Ic][:, Ic] + Jc.T @ sp.diags(p.D) @ Jc).tocsr()
    anorm = abs(Aw).sum(axis=1).max()
    print(f"[gpu setup] C3 n_c={len(Ic)}", flush=True)
    h = AMGF.from_problem(p, precision=1)
    assert np.array_equal(h.filter_dofs(len(Ic)), Ic)
    rng = np.random.default_rng(6)
    for trial in range(2):
        r = rng.standard_normal(len(Ic))
        w = h.filter_solve(r).cpu().numpy()
        w2 = h.filter_solve(r).cpu().numpy()
        eta = np.abs(r - Aw @ w).max() / (anorm * np.abs(w).max() + np.abs(r).max())
        print(f"C3 n_c={len(Ic)}: backward error {eta:.2e}")
        assert np.array_equal(w, w2)
        assert eta <= 1e-14
    h.close()
