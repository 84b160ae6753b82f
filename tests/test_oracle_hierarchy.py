"""Pins of the oracle's prolongators and Galerkin products."""
import numpy as np
import pytest

from amgf_inputs import make_config
from oracle import gram_schmidt_qr
from oracle.amgf_oracle import rigid_body_modes, group_members
from oracle_util import build, small_problem


def test_gram_schmidt_matches_householder_on_full_rank():
    rng = np.random.default_rng(3)
    B = rng.standard_normal((30, 6))
    Q, R, dead = gram_schmidt_qr(B, 1e-10)
    Qh, Rh = np.linalg.qr(B)
    s = np.sign(np.diag(Rh))
    assert not dead.any()
    assert np.allclose(Q, Qh * s, atol=1e-13) and np.allclose(R, Rh * s[:, None], atol=1e-13)


def test_gram_schmidt_dead_columns():
    rng = np.random.default_rng(4)
    B = rng.standard_normal((12, 6))
    B[:, 2] = 2 * B[:, 0] - B[:, 1]
    B[:, 5] = 0.0
    Q, R, dead = gram_schmidt_qr(B, 1e-10)
    assert list(dead) == [False, False, True, False, False, True]
    assert np.allclose(Q @ R, B, atol=1e-13)
    assert np.allclose(Q.T @ Q, np.diag(~dead), atol=1e-13)
    assert np.allclose(np.tril(R, -1), 0) and (np.diag(R) >= 0).all()
    assert not Q[:, dead].any() and not R[dead].any()


@pytest.fixture(scope="module")
def c1():
    p = make_config("C1")
    return p, build(p, coarse_max_nodes=8)


def test_tentative_prolongator_reproduces_rigid_modes(c1):
    p, o = c1
    lev = o.levels[0]
    members, off = group_members(lev.agg, lev.n_agg)
    Pt = lev.Pt.todense()
    dec = lev.decoupled
    assert (dec == ~p.free).all()                     # decoupled DOFs are the Dirichlet DOFs
    for J in range(lev.n_agg):
        nodes = members[off[J]:off[J + 1]]
        c = p.coords[nodes].mean(axis=0)
        B = rigid_body_modes(p.coords[nodes] - c)
        B[dec.reshape(-1, 3)[nodes]] = 0
        dofs = (3 * nodes[:, None] + np.arange(3)).ravel()
        QJ = Pt[dofs][:, 6 * J:6 * J + 6]
        assert np.allclose(QJ @ lev.R[J], B.reshape(-1, 6), atol=1e-13)
        live = ~lev.dead[J]
        assert np.allclose(QJ.T @ QJ, np.diag(live), atol=1e-12)
    assert np.allclose(Pt.T @ Pt, np.diag(~lev.dead.ravel()), atol=1e-12)


def test_smoothed_prolongator_and_l1_norms(c1):
    p, o = c1
    lev = o.levels[0]
    A = lev.A.todense()
    assert np.allclose(lev.d, np.abs(A).sum(axis=1), rtol=1e-15)
    Pt = lev.Pt.todense()
    # damping: sa_omega over the spectral radius of D_l1^{-1} A on the coupled DOFs
    keep = ~lev.decoupled
    DA = (A / lev.d[:, None])[keep][:, keep]
    rho = np.abs(np.linalg.eigvals(DA)).max()
    assert 0.9 * rho <= lev.rho <= min(1.0, 1.05 * rho)
    ref = Pt - lev.omega * (A / lev.d[:, None]) @ Pt
    rows = np.repeat(lev.agg >= 0, 3)
    ref[~rows] = 0.0
    P = lev.P.todense()
    assert np.abs(P - ref).max() <= 1e-13 * np.abs(ref).max()


def test_galerkin_coarse_operators(c1):
    p, o = c1
    for l in range(o.nlev - 1):
        lev, nxt = o.levels[l], o.levels[l + 1]
        P = lev.P.todense()
        dead = np.zeros(P.shape[1], bool)
        if lev.dead is not None:
            dead = lev.dead.ravel()
        Kc = P.T @ lev.K.todense() @ P + np.diag(dead.astype(float))
        Ac = P.T @ lev.A.todense() @ P + np.diag(dead.astype(float))
        assert np.abs(nxt.K.todense() - Kc).max() <= 1e-12 * np.abs(Kc).max()
        assert np.abs(nxt.A.todense() - Ac).max() <= 1e-12 * np.abs(Ac).max()
        Jd = lev.J.todense() @ P
        assert np.abs(nxt.J.todense() - Jd).max() <= 1e-13 * max(np.abs(Jd).max(), 1)
        # coarse operators stay symmetric positive definite
        Ad = nxt.A.todense()
        assert np.allclose(Ad, Ad.T, rtol=0, atol=1e-12 * np.abs(Ad).max())
    assert np.linalg.eigvalsh(o.levels[-1].A.todense())[0] > 0


def test_hierarchy_shape_c1():
    p = make_config("C1")
    o = build(p)
    assert o.nlev == 2 and o.levels[1].A.br == 6
    assert 1.0 < o.operator_complexity() < 2.0
