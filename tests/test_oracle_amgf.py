"""Pins of the oracle's V-cycle B and AMGF preconditioner M against Sec. 5.

Dense brute force on a small two-body problem (N = 3, 384 DOFs)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import pcg
from oracle_util import build, dense_of, small_problem


@pytest.fixture(scope="module")
def prob():
    p = small_problem(N=3, D_log10=(0.0, 3.0))
    o = build(p, coarse_max_nodes=8, max_levels=2)       # exactly two levels
    A = o.S.todense()
    B = dense_of(o.vcycle, o.n)
    M = dense_of(o.apply, o.n)
    Pf = np.zeros((o.n, o.n_c))
    Pf[o.Ic, np.arange(o.n_c)] = 1.0
    return p, o, A, B, M, Pf


def test_two_level_vcycle_formula(prob):
    """B from the V-cycle equals the two-grid error propagation
    I - BA = (I - WA)(I - P Ac^{-1} P^T A)(I - WA), W = diag(theta/d)."""
    p, o, A, B, M, Pf = prob
    assert o.nlev == 2
    lev = o.levels[0]
    W = np.diag(lev.w)
    P = lev.P.todense()
    Ac = P.T @ A @ P + np.diag(lev.dead.ravel().astype(float))
    I = np.eye(o.n)
    E = (I - W @ A) @ (I - P @ np.linalg.solve(Ac, P.T @ A)) @ (I - W @ A)
    Bref = (I - E) @ np.linalg.inv(A)
    assert np.abs(B - Bref).max() <= 1e-8 * np.abs(Bref).max()


def test_B_symmetric_and_convergent_with_omega_one(prob):
    """l1 smoothers give a convergent B with omega = 1 (Remark 5.6): lambda(BA) in (0,1]."""
    p, o, A, B, M, Pf = prob
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    lam = np.sort(np.linalg.eigvals(B @ A).real)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-9


def test_definition_5_3_error_propagation(prob):
    """I - MA = (I - BA)(I - P A_w^{-1} P^T A)(I - BA)  (Definition 5.3)."""
    p, o, A, B, M, Pf = prob
    I = np.eye(o.n)
    Aw = Pf.T @ A @ Pf
    E = (I - B @ A) @ (I - Pf @ np.linalg.solve(Aw, Pf.T @ A)) @ (I - B @ A)
    lhs = I - M @ A
    assert np.abs(lhs - E).max() <= 1e-7


def test_definition_5_3_block_form(prob):
    """M = [I P] Mbar^{-1} [I; P^T] with the three-factor Mbar of Definition 5.3."""
    p, o, A, B, M, Pf = prob
    n, nc = o.n, o.n_c
    Binv = np.linalg.inv(B)
    Aw = Pf.T @ A @ Pf
    L = np.block([[Binv, np.zeros((n, nc))], [Pf.T @ A, np.eye(nc)]])
    Dm = np.block([[np.linalg.inv(2 * Binv - A), np.zeros((n, nc))],
                   [np.zeros((nc, n)), Aw]])
    U = np.block([[Binv, A @ Pf], [np.zeros((nc, n)), np.eye(nc)]])
    Mbar = L @ Dm @ U
    IP = np.hstack([np.eye(n), Pf])
    Mref = IP @ np.linalg.solve(Mbar, IP.T)
    assert np.abs(M - Mref).max() <= 1e-6 * np.abs(M).max()


def test_lower_bound_and_condition_number_estimate(prob):
    """(Au,u) <= (M^{-1}u,u) (lower-bound lemma) and
    kappa(MA) <= 2 (beta + 2 + omega) / (2 - omega) (Lemma 5.4)."""
    p, o, A, B, M, Pf = prob
    assert np.abs(M - M.T).max() <= 1e-8 * np.abs(M).max()
    lam = np.sort(np.linalg.eigvals(M @ A).real)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-9
    kappa = lam[-1] / lam[0]
    omega = np.linalg.eigvals(B @ A).real.max()
    # V = A-orthogonal complement of range(P): null(P^T A)
    Z = sla.null_space(Pf.T @ A)
    Binv = np.linalg.inv(B)
    G1 = Z.T @ Binv @ Z
    G2 = Z.T @ A @ Z
    ev = sla.eigh(0.5 * (G1 + G1.T), 0.5 * (G2 + G2.T), eigvals_only=True)
    alpha, beta = ev[0], ev[-1]
    assert alpha >= 1 - 1e-8                      # alpha = 1 for l1 smoothers (Remark 5.6)
    bound = 2 * (beta + 2 + omega) / (2 - omega)
    assert kappa <= bound * (1 + 1e-8)
    assert kappa <= 2 * (beta + 3) * (1 + 1e-8)   # Remark 5.6 with omega <= 1


def test_stability_estimate(prob):
    """2||v||_{B^-1}^2 + (2+omega)||Pw||_A^2 <= 2(beta+2+omega)||u||_A^2 (Lemma 5.5)."""
    p, o, A, B, M, Pf = prob
    Binv = np.linalg.inv(B)
    omega = np.linalg.eigvals(B @ A).real.max()
    Z = sla.null_space(Pf.T @ A)
    G1 = Z.T @ Binv @ Z
    beta = sla.eigh(0.5 * (G1 + G1.T), Z.T @ A @ Z, eigvals_only=True)[-1]
    Aw = Pf.T @ A @ Pf
    rng = np.random.default_rng(5)
    for _ in range(10):
        u = rng.standard_normal(o.n)
        w = np.linalg.solve(Aw, Pf.T @ A @ u)
        v = u - Pf @ w
        lhs = 2 * v @ Binv @ v + (2 + omega) * (Pf @ w) @ A @ (Pf @ w)
        assert lhs <= 2 * (beta + 2 + omega) * (u @ A @ u) * (1 + 1e-9)


def test_filter_correction_exact_on_filter_space(prob):
    p, o, A, B, M, Pf = prob
    Aw = Pf.T @ A @ Pf
    Pi = Pf @ np.linalg.solve(Aw, Pf.T @ A)
    rng = np.random.default_rng(6)
    w = rng.standard_normal(o.n_c)
    assert np.abs((np.eye(o.n) - Pi) @ Pf @ w).max() <= 1e-10 * np.abs(w).max()
    assert np.abs(Pi @ Pi - Pi).max() <= 1e-9
    assert np.abs(A @ Pi - (A @ Pi).T).max() <= 1e-9 * np.abs(A).max()
    # the oracle's filter solve is A_w^{-1}
    r = rng.standard_normal(o.n_c)
    assert np.allclose(o.filter_solve(r), np.linalg.solve(Aw, r), rtol=1e-9, atol=0)


def test_special_cases():
    p = small_problem(N=2, D_log10=(0.0, 3.0))
    n = p.n
    # I_c = all DOFs: M = A^{-1}
    o = build(p, coarse_max_nodes=4, Ic=np.arange(n))
    A = o.S.todense()
    M = dense_of(o.apply, n)
    assert np.abs(M @ A - np.eye(n)).max() <= 1e-8
    res = o.pcg(p.b)
    assert res.iterations == 1
    # one dense level: B = A^{-1}, so M = A^{-1}
    o = build(p, coarse_max_nodes=10 ** 6)
    assert o.nlev == 1
    assert np.abs(dense_of(o.apply, n) @ A - np.eye(n)).max() <= 1e-8
    # empty filter space (no contact): M = 2B - BAB
    q = small_problem(N=2, contact=False, top_bc="clamped")
    o = build(q, coarse_max_nodes=4)
    A = o.S.todense()
    B = dense_of(o.vcycle, n)
    M = dense_of(o.apply, n)
    assert o.n_c == 0
    assert np.abs(M - (2 * B - B @ A @ B)).max() <= 1e-10 * np.abs(M).max()
    # filter off: M = B
    o2 = build(q, coarse_max_nodes=4, filter=False)
    assert np.abs(dense_of(o2.apply, n) - B).max() <= 1e-12 * np.abs(B).max()


def test_pcg_identity_preconditioner_matches_direct_solve():
    p = small_problem(N=2, D_log10=(0.0, 2.0))
    o = build(p)
    A = o.S.todense()
    res = pcg(o.A_apply, lambda r: r.copy(), p.b, rtol=1e-13, max_iters=5000)
    x = np.linalg.solve(A, p.b)
    assert res.converged
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


def test_filter_removes_barrier_ill_conditioning():
    """With D spanning 8 decades, kappa(BA) of plain AMG grows with D while
    kappa(MA) stays within the Lemma 5.4 bound (Sec. 4 and Sec. 5)."""
    kap = {}
    for hi in (0.0, 8.0):
        p = small_problem(N=3, D_log10=(0.0, hi) if hi else (0.0, 0.0))
        o = build(p, coarse_max_nodes=8, max_levels=2)
        A = o.S.todense()
        B = dense_of(o.vcycle, o.n)
        M = dense_of(o.apply, o.n)
        lb = np.sort(np.linalg.eigvals(B @ A).real)
        lm = np.sort(np.linalg.eigvals(M @ A).real)
        kap[hi] = (lb[-1] / lb[0], lm[-1] / lm[0])
    assert kap[8.0][0] > 100 * kap[0.0][0]
    assert kap[8.0][1] < 3 * kap[0.0][1] + 10
