"""Pins of the oracle's smoother options (l1-Jacobi sweeps, Chebyshev) against closed forms.

The Chebyshev smoother's error propagation on the D_l1-preconditioned operator is the scaled
Chebyshev polynomial T_m((theta - lambda)/delta) / T_m(theta/delta) of the generalized
eigenvalues A v = lambda D v; the check builds the smoother's matrix column by column and
compares it with that spectral formula (a dropped recurrence term, a wrong coefficient or a
wrong interval all change the polynomial)."""
import numpy as np
import pytest
import scipy.linalg as sla
from numpy.polynomial import chebyshev as C

from oracle import pcg
from oracle_util import build, dense_of, small_problem


@pytest.fixture(scope="module")
def prob():
    p = small_problem(N=3, D_log10=(0.0, 3.0))
    return p


def _smoother_matrix(o, l=0):
    n = o.levels[l].A.nrows * o.levels[l].A.br
    zero = np.zeros(n)
    return dense_of(lambda e: o.smooth(l, zero, e), n)   # b = 0: columns are E e_j


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_chebyshev_error_polynomial(prob, degree):
    o = build(prob, coarse_max_nodes=8, max_levels=2, smoother="chebyshev", cheb_degree=degree)
    lev = o.levels[0]
    A = lev.A.todense()
    D = np.diag(lev.d)
    E = _smoother_matrix(o)
    lam, V = sla.eigh(A, D)                     # V^T D V = I, D^-1 A = V diag(lam) V^T D
    lmax = min(1.0, 1.1 * lev.lam)
    lmin = 0.3 * lmax
    theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
    coef = np.zeros(degree + 1)
    coef[degree] = 1.0
    q = C.chebval((theta - lam) / delta, coef) / C.chebval(theta / delta, coef)
    Eref = V @ np.diag(q) @ V.T @ D
    assert np.abs(E - Eref).max() <= 1e-10 * max(1.0, np.abs(Eref).max())
    # the smoother contracts in the A-norm: |q| < 1 on the whole spectrum (0, 1]
    assert lam.max() <= 1.0 + 1e-12
    assert np.abs(q).max() < 1.0


def test_power_estimate_brackets_spectrum(prob):
    o = build(prob, coarse_max_nodes=8, max_levels=2)
    lev = o.levels[0]
    lam = sla.eigh(lev.A.todense(), np.diag(lev.d), eigvals_only=True)
    # ten power steps from a fixed start reach at least 80 % of the top eigenvalue here and
    # never exceed it (Rayleigh-type estimate of a symmetric-definite pencil)
    assert 0.8 * lam.max() <= lev.lam <= lam.max() * (1 + 1e-12)


@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_jacobi_sweeps_are_powers(prob, sweeps):
    """nu Jacobi sweeps from x: error propagation (I - W A)^nu."""
    o = build(prob, coarse_max_nodes=8, max_levels=2, sweeps=sweeps)
    lev = o.levels[0]
    A = lev.A.todense()
    W = np.diag(lev.w)
    n = o.n
    zero = np.zeros(n)

    def nu_steps(e):
        x = e
        for _ in range(sweeps):
            x = o.smooth(0, zero, x)
        return x
    E = dense_of(nu_steps, n)
    Eref = np.linalg.matrix_power(np.eye(n) - W @ A, sweeps)
    assert np.abs(E - Eref).max() <= 1e-12


@pytest.mark.parametrize("kw", [dict(smoother="chebyshev"), dict(sweeps=2),
                                dict(smoother="chebyshev", cheb_degree=3, sweeps=2)])
def test_vcycle_options_symmetric_and_convergent(prob, kw):
    """Equal pre- and post-smoothers keep B symmetric; an A-contractive smoother keeps
    lambda(BA) in (0, 1] (two-level V-cycle with an exact coarse solve)."""
    o = build(prob, coarse_max_nodes=8, max_levels=2, **kw)
    A = o.S.todense()
    B = dense_of(o.vcycle, o.n)
    assert np.abs(B - B.T).max() <= 1e-10 * np.abs(B).max()
    lam = np.sort(np.linalg.eigvals(B @ A).real)
    assert lam[0] > 0 and lam[-1] <= 1 + 1e-9
    # two-grid formula with the option's smoother matrix S (error I - S A per application)
    lev = o.levels[0]
    n = o.n
    Es = _smoother_matrix(o)
    Es = np.linalg.matrix_power(Es, kw.get("sweeps", 1))
    P = lev.P.todense()
    Ac = P.T @ A @ P + np.diag(lev.dead.ravel().astype(float))
    I = np.eye(n)
    E = Es @ (I - P @ np.linalg.solve(Ac, P.T @ A)) @ Es
    Bref = (I - E) @ np.linalg.inv(A)
    assert np.abs(B - Bref).max() <= 1e-8 * np.abs(Bref).max()


def test_amgf_pcg_with_options_solves(prob):
    p = prob
    ref = np.linalg.solve(build(p).S.todense(), p.b)
    its = {}
    for name, kw in (("jacobi", {}), ("cheb", dict(smoother="chebyshev")),
                     ("jacobi2", dict(sweeps=2))):
        o = build(p, **kw)
        res = o.pcg(p.b)
        assert res.converged
        assert np.linalg.norm(res.x - ref) <= 1e-8 * np.linalg.norm(ref)
        its[name] = res.iterations
    # a stronger smoother never needs more iterations on this problem
    assert its["jacobi2"] <= its["jacobi"] and its["cheb"] <= its["jacobi"]
