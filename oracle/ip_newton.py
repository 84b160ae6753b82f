"""Plain FP64 interior-point Newton driver for the contact QP.  TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this module.

The problem (Sec. 3 with a quadratic energy and a linear gap):
    minimise 1/2 u^T K u - f^T u   subject to   g(u) = J u + g0 >= 0,
with slacks s >= 0, multipliers lam of J u + g0 - s = 0 and duals z = mu / s.  The barrier
term is weighted by the diagonal lumped slack mass M_s, and the optimality errors measure
r_u and r_s in the M_u^{-1} and M_s^{-1} norms (M_u the lumped mass of the displacements).
The residuals of the barrier subproblem for mu > 0 are
    r_u   = K u - f + J^T lam
    r_s   = -lam - M_s z
    r_lam = J u + g0 - s
    r_z   = s z - mu
The Newton system in (u^, s^, lam^, z^) is condensed as in Sec. 3: eliminating z^ gives
the symmetric 3x3 block system with D = diag(M_s z / s), and eliminating s^ and lam^ leaves
A u^ = b with A = K + J^T D J and b = b_u + J^T (D b_lam + b_s), where
    b_u = -r_u,   b_s = -(r_s + M_s r_z / s),   b_lam = -r_lam.
The other components follow from the eliminated rows:
    s^ = J u^ - b_lam,   lam^ = D s^ - b_s,   z^ = -(r_z + z s^) / s.

The outer structure is the simplified algorithm outline of Sec. 3: Newton steps on one
barrier subproblem until its optimality error is below kappa_eps * mu, then a smaller mu,
until the optimality error of the problem itself (mu = 0) is below tol.  Where the paper
defers to its IP reference (Wachter and Biegler 2006), the published defaults of that
method are used: the fraction-to-the-boundary rule with tau = max(tau_min, 1 - mu) in place
of the filter line search (the problem is a convex QP, so full Newton steps cut back at the
boundary converge), the barrier update mu <- max(tol / 10, min(kappa_mu mu, mu^theta_mu)),
and the optimality-error scaling s_d, s_c with s_max = 100.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


@dataclass
class IPOptions:
    tol: float = 1e-6                 # tol_IP (Sec. 4 uses 1e-6)
    mu0: float = 0.1
    kappa_eps: float = 10.0           # subproblem tolerance kappa_eps * mu (Sec. 3)
    kappa_mu: float = 0.2
    theta_mu: float = 1.5
    tau_min: float = 0.99
    s_max: float = 100.0              # optimality-error scaling constant (Sec. 3)
    s_init: float = 1e-2              # lower bound of the initial slacks
    max_steps: int = 200


@dataclass
class IPStep:
    mu: float
    e_opt: float                      # optimality error of the problem (mu = 0)
    e_opt_mu: float                   # ... of the barrier subproblem
    alpha_p: float
    alpha_d: float
    D_min: float
    D_max: float
    pcg_iterations: int = 0


@dataclass
class IPResult:
    u: np.ndarray
    s: np.ndarray
    lam: np.ndarray
    z: np.ndarray
    mu: float
    converged: bool
    steps: list = field(default_factory=list)


def residuals(K, J, f, g0, u, s, lam, z, mu, Ms=1.0):
    """The four optimality residuals of the barrier subproblem (r_u, r_s, r_lam, r_z)."""
    r_u = K @ u - f + J.T @ lam
    r_s = -lam - Ms * z
    r_lam = J @ u + g0 - s
    r_z = s * z - mu
    return r_u, r_s, r_lam, r_z


def optimality_error(r_u, r_s, r_lam, r_z, lam, z, s_max, Ms=1.0, Mu=1.0):
    """max of the scaled residual norms: the M_u^{-1} and M_s^{-1} norms of the dual
    residuals over s_d, the max-norm of the constraint residual, the max-norm of the
    complementarity residual over s_c."""
    m = max(len(z), 1)
    s_d = max(s_max, (np.abs(lam).sum() + np.abs(z).sum()) / (2 * m)) / s_max
    s_c = max(s_max, np.abs(z).sum() / m) / s_max
    inf = lambda v: float(np.abs(v).max()) if len(v) else 0.0
    return max(math.sqrt(float(np.sum(r_u * r_u / Mu))) / s_d,
               math.sqrt(float(np.sum(r_s * r_s / Ms))) / s_d, inf(r_lam), inf(r_z) / s_c)


def newton_direction(K, J, u, s, lam, z, res, solve, Ms=1.0):
    """Condensed Newton step of Sec. 3.  ``solve(D, b)`` returns the solution of
    (K + J^T diag(D) J) x = b."""
    r_u, r_s, r_lam, r_z = res
    D = Ms * z / s
    b_u, b_s, b_lam = -r_u, -(r_s + Ms * r_z / s), -r_lam
    b = b_u + J.T @ (D * b_lam + b_s)
    u_h = solve(D, b)
    s_h = J @ u_h - b_lam
    lam_h = D * s_h - b_s
    z_h = -(r_z + z * s_h) / s
    return u_h, s_h, lam_h, z_h, D


def max_step(v, dv, tau):
    """Largest alpha in (0, 1] with v + alpha dv >= (1 - tau) v (fraction to the boundary)."""
    neg = dv < 0
    if not neg.any():
        return 1.0
    return float(min(1.0, np.min(-tau * v[neg] / dv[neg])))


def direct_solver(K, J):
    """Exact Newton solves by sparse LU of A = K + J^T D J."""
    K = sp.csr_matrix(K)
    J = sp.csr_matrix(J)

    def solve(D, b):
        A = (K + J.T @ sp.diags(D) @ J).tocsc()
        return spla.spsolve(A, b)
    return solve


def ip_solve(K, J, f, g0, opts: IPOptions | None = None, solve=None, u0=None, Ms=None,
             Mu=None):
    """Run the interior-point method from u0 (default 0) and return an IPResult whose
    ``steps`` record mu, the optimality errors, the step lengths and the range of D of
    every Newton step.  Ms (m) and Mu (n): diagonal lumped masses (default ones).
    ``solve(D, b)`` defaults to ``direct_solver``; a callable that also returns an
    iteration count (a tuple) is accepted and the count recorded."""
    o = opts or IPOptions()
    Ms = np.ones(len(g0)) if Ms is None else np.asarray(Ms, np.float64)
    Mu = np.ones(K.shape[0]) if Mu is None else np.asarray(Mu, np.float64)
    K = sp.csr_matrix(K)
    J = sp.csr_matrix(J)
    solve = solve or direct_solver(K, J)
    n = K.shape[0]
    u = np.zeros(n) if u0 is None else np.array(u0, np.float64)
    mu = o.mu0
    s = np.maximum(J @ u + g0, o.s_init)
    z = mu / s
    lam = -Ms * z
    steps = []
    converged = False
    for _ in range(o.max_steps):
        res = residuals(K, J, f, g0, u, s, lam, z, 0.0, Ms)
        if optimality_error(*res, lam, z, o.s_max, Ms, Mu) < o.tol:
            converged = True
            break
        # barrier subproblem converged: decrease mu (possibly several times)
        while True:
            res = residuals(K, J, f, g0, u, s, lam, z, mu, Ms)
            e_mu = optimality_error(*res, lam, z, o.s_max, Ms, Mu)
            if e_mu >= o.kappa_eps * mu or mu <= o.tol / 10:
                break
            mu = max(o.tol / 10, min(o.kappa_mu * mu, mu ** o.theta_mu))
        res = residuals(K, J, f, g0, u, s, lam, z, mu, Ms)
        e_mu = optimality_error(*res, lam, z, o.s_max, Ms, Mu)
        e0 = optimality_error(*residuals(K, J, f, g0, u, s, lam, z, 0.0, Ms), lam, z, o.s_max,
                              Ms, Mu)
        its = 0

        def counted(D, b):
            nonlocal its
            x = solve(D, b)
            if isinstance(x, tuple):
                x, its = x
            return x
        u_h, s_h, lam_h, z_h, D = newton_direction(K, J, u, s, lam, z, res, counted, Ms)
        tau = max(o.tau_min, 1.0 - mu)
        a_p = max_step(s, s_h, tau)
        a_d = max_step(z, z_h, tau)
        steps.append(IPStep(mu=mu, e_opt=e0, e_opt_mu=e_mu, alpha_p=a_p, alpha_d=a_d,
                            D_min=float(D.min()) if len(D) else 0.0,
                            D_max=float(D.max()) if len(D) else 0.0, pcg_iterations=its))
        u = u + a_p * u_h
        s = s + a_p * s_h
        lam = lam + a_p * lam_h
        z = z + a_d * z_h
    return IPResult(u=u, s=s, lam=lam, z=z, mu=mu, converged=converged, steps=steps)


def kkt_certificate(K, J, f, g0, u, z):
    """Residuals of the first-order conditions of the QP itself, which for a convex QP
    certify a global minimiser: stationarity K u - f - J^T z = 0, feasibility
    J u + g0 >= 0, z >= 0 and complementarity z (J u + g0) = 0, for the constraint forces
    z (= -lam of the driver).  Returns the four max-norm violations."""
    K = sp.csr_matrix(K)
    J = sp.csr_matrix(J)
    g = J @ u + g0
    stat = K @ u - f - J.T @ z
    return (float(np.abs(stat).max()), float(max(0.0, -g.min())),
            float(max(0.0, -z.min())), float(np.abs(z * g).max()))
