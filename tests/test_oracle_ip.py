"""Pins of the oracle's interior-point driver (the contact QP of Sec. 3): a separable problem
with a closed-form minimiser, the condensed Newton step against the full Newton system
built by finite differences of the residual map, and the first-order conditions plus an
independent active-set solve of the two-body QP."""
import numpy as np
import scipy.sparse as sp
import pytest

from amgf_inputs import make_two_block, contact_load_and_gap
from oracle.ip_newton import (IPOptions, ip_solve, kkt_certificate, newton_direction,
                              residuals, direct_solver)


def _two_block(N, pressure=0.05):
    p = make_two_block(N)
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(p.n, p.n)).tocsr()
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, p.n))
    f, g0 = contact_load_and_gap(p, pressure=pressure)
    return p, K, J, f, g0


def test_separable_closed_form():
    """min 1/2 k u^2 - f u subject to u + g0 >= 0, one unknown per constraint: the minimiser
    is max(f/k, -g0) and the contact force k u - f (zero where the bound is inactive)."""
    rng = np.random.default_rng(0)
    n = 40
    k = rng.uniform(0.5, 4.0, n)
    f = rng.uniform(-2.0, 2.0, n)
    g0 = rng.uniform(0.0, 1.0, n)
    K = sp.diags(k).tocsr()
    J = sp.identity(n, format="csr")
    r = ip_solve(K, J, f, g0, IPOptions(tol=1e-9))
    u_star = np.maximum(f / k, -g0)
    z_star = k * u_star - f
    assert r.converged
    assert np.abs(r.u - u_star).max() < 1e-7
    assert np.abs(r.z - z_star).max() < 1e-7
    assert ((z_star > 1e-3) == (np.abs(r.u + g0) < 1e-6)).all()


def test_condensed_step_equals_full_newton_system():
    """The condensation of Sec. 3 (b, and the recovery of s^, lam^, z^) solves the full
    Newton system of the residual map, whose Jacobian is taken here by central differences
    (exact for the affine and bilinear residuals up to rounding)."""
    p, K, J, f, g0 = _two_block(2)
    rng = np.random.default_rng(1)
    n, m = p.n, p.m
    u = rng.standard_normal(n) * 0.01 * p.free
    s = rng.uniform(0.1, 1.0, m)
    z = rng.uniform(0.1, 1.0, m)
    lam = rng.standard_normal(m)
    mu = 0.05

    def F(x):
        return np.concatenate(residuals(K, J, f, g0, x[:n], x[n:n + m], x[n + m:n + 2 * m],
                                        x[n + 2 * m:], mu))
    x0 = np.concatenate([u, s, lam, z])
    Jac = np.zeros((x0.size, x0.size))
    for i in range(x0.size):
        e = np.zeros(x0.size)
        e[i] = 1e-3
        Jac[:, i] = (F(x0 + e) - F(x0 - e)) / 2e-3
    full = np.linalg.solve(Jac, -F(x0))
    res = residuals(K, J, f, g0, u, s, lam, z, mu)
    u_h, s_h, lam_h, z_h, D = newton_direction(K, J, u, s, lam, z, res, direct_solver(K, J))
    cond = np.concatenate([u_h, s_h, lam_h, z_h])
    assert np.allclose(D, z / s)
    assert np.linalg.norm(cond - full) <= 1e-9 * np.linalg.norm(full)


@pytest.mark.parametrize("N", [4, 6])
def test_two_block_qp_minimiser(N):
    """The IP result satisfies the first-order conditions of the convex QP (so it is its
    minimiser), and agrees with the exact solution of the equality-constrained QP on the
    active set it found, whose multipliers are non-negative and whose other gaps are open."""
    p, K, J, f, g0 = _two_block(N)
    # the contact forces are nodal (about pressure / N^2), so the absolute stopping rule is
    # tightened here to resolve the active set
    r = ip_solve(K, J, f, g0, IPOptions(tol=1e-10))
    assert r.converged and 5 <= len(r.steps) <= 40
    stat, infeas, dneg, compl = kkt_certificate(K, J, f, g0, r.u, r.z)
    assert stat <= 1e-11 and infeas == 0.0 and dneg == 0.0 and compl <= 1e-10
    g = J @ r.u + g0
    act = np.nonzero(r.z > g)[0]
    assert 0 < len(act) < p.m
    JA = J[act]
    KKT = sp.bmat([[K, -JA.T], [JA, None]]).tocsc()
    sol = sp.linalg.spsolve(KKT, np.concatenate([f, -g0[act]]))
    u_a, z_a = sol[:p.n], sol[p.n:]
    assert (z_a > 0).all()
    assert (np.delete(J @ u_a + g0, act) > 0).all()
    assert np.linalg.norm(r.u - u_a) <= 1e-6 * np.linalg.norm(u_a)
    # the barrier diagonal spreads over many orders of magnitude by the end (Sec. 4)
    assert r.steps[-1].D_max / r.steps[-1].D_min > 1e6


def test_barrier_sequence():
    p, K, J, f, g0 = _two_block(4)
    o = IPOptions()
    r = ip_solve(K, J, f, g0, o)
    mus = [s.mu for s in r.steps]
    assert mus[0] == o.mu0 and all(b <= a for a, b in zip(mus, mus[1:]))
    assert all(0 < s.alpha_p <= 1 and 0 < s.alpha_d <= 1 for s in r.steps)
    assert (r.s > 0).all() and (r.z > 0).all()
    assert np.allclose(r.lam, -r.z, rtol=1e-5, atol=1e-8)
