"""GPU interior-point driver (amgf_ip_solve) on the two-body contact QP: parity with the
oracle's driver (exact Newton solves), the first-order conditions of the QP at the result,
AMG-PCG against AMGF-PCG along the Newton steps (Sec. 4's comparison), and the switch from
AMG to AMGF once the barrier diagonal has spread (Sec. 7)."""
import numpy as np
import pytest
import scipy.sparse as sp

from amgf_inputs import contact_load_and_gap, lumped_masses, make_two_block
from oracle.ip_newton import IPOptions, ip_solve, kkt_certificate

pytestmark = pytest.mark.gpu


def _qp(N):
    p = make_two_block(N)
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(p.n, p.n)).tocsr()
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, p.n))
    f, g0 = contact_load_and_gap(p)
    Ms, Mu = lumped_masses(p)
    return p, K, J, f, g0, Ms, Mu


def _handle(p, **kw):
    from paper_2505_18576_amd import AMGF
    print(f"[gpu setup] two-block N={p.N} {kw}", flush=True)
    return AMGF.from_problem(p, **kw)


@pytest.mark.parametrize("N,tol,masses", [(6, 1e-6, False), (6, 1e-6, True),
                                          (8, 1e-10, True)])
def test_ip_matches_oracle(N, tol, masses):
    p, K, J, f, g0, Ms, Mu = _qp(N)
    if not masses:
        Ms = Mu = None
    ref = ip_solve(K, J, f, g0, IPOptions(tol=tol), Ms=Ms, Mu=Mu)
    h = _handle(p)
    u, s, lam, z, steps, conv = h.ip_solve(f, g0, Ms=Ms, Mu=Mu, tol=tol)
    u, s, lam, z = (v.cpu().numpy() for v in (u, s, lam, z))
    print(f"N={N} tol={tol}: gpu {len(steps)} steps, oracle {len(ref.steps)} steps; "
          f"PCG its {[st['pcg_iterations'] for st in steps]}")
    assert conv and ref.converged
    assert len(steps) == len(ref.steps)
    assert [st["mu"] for st in steps] == [st.mu for st in ref.steps]
    # the first step starts from the same point: everything but the CG tolerance is equal
    a, b = steps[0], ref.steps[0]
    assert abs(a["e_opt"] - b.e_opt) <= 1e-12 * b.e_opt
    assert abs(a["D_max"] - b.D_max) <= 1e-12 * b.D_max
    assert abs(a["alpha_p"] - b.alpha_p) <= 1e-8 and abs(a["alpha_d"] - b.alpha_d) <= 1e-8
    for x, y in ((u, ref.u), (z, ref.z)):
        assert np.linalg.norm(x - y) <= 1e-6 * np.linalg.norm(y)
    # constraint forces -lam (= M_s z at convergence)
    stat, infeas, dneg, compl = kkt_certificate(K, J, f, g0, u, -lam)
    print(f"  KKT: stationarity {stat:.1e}, infeasibility {infeas:.1e}, "
          f"complementarity {compl:.1e}")
    assert stat <= 10 * tol and infeas == 0.0 and dneg == 0.0 and compl <= 10 * tol
    assert np.allclose(-lam, (1.0 if Ms is None else Ms) * z, rtol=1e-4, atol=10 * tol)
    h.close()


def test_amg_degrades_amgf_does_not():
    """Along the Newton steps the barrier diagonal spreads over many orders of magnitude;
    plain AMG-PCG needs more and more iterations while AMGF-PCG stays flat (Sec. 4)."""
    p, K, J, f, g0, Ms, Mu = _qp(16)
    runs = {}
    for filt in (1, 0):
        h = _handle(p, filter=filt, max_iters=3000)
        u, s, lam, z, steps, conv = h.ip_solve(f, g0, Ms=Ms, Mu=Mu, tol=1e-8)
        runs[filt] = (u.cpu().numpy(), steps, conv)
        print(f"filter={filt}: {len(steps)} steps, D_max/D_min "
              f"{steps[-1]['D_max'] / steps[-1]['D_min']:.1e}, PCG its "
              f"{[st['pcg_iterations'] for st in steps]}", flush=True)
        h.close()
    (u1, st1, c1), (u0, st0, c0) = runs[1], runs[0]
    assert c1 and c0
    its1 = [st["pcg_iterations"] for st in st1]
    its0 = [st["pcg_iterations"] for st in st0]
    assert all(st["pcg_converged"] for st in st1)
    assert max(its1) <= 3 * min(its1)
    assert max(its0[-3:]) >= 3 * max(its1)
    assert np.linalg.norm(u1 - u0) <= 1e-5 * np.linalg.norm(u1)


def test_switch_from_amg_to_amgf():
    """AMG-PCG while D_max / D_min < 1e6, AMGF from the first Newton step that reaches it
    on (the switch Sec. 7 suggests): the filter-on pattern is the one the oracle's own
    barrier diagonals give for the same ratio, and the switched run ends at the oracle's
    solution."""
    p, K, J, f, g0, Ms, Mu = _qp(12)
    ratio = 1e6
    ref = ip_solve(K, J, f, g0, IPOptions(tol=1e-8), Ms=Ms, Mu=Mu)
    reached = [st.D_max >= ratio * st.D_min for st in ref.steps]
    k_ref = reached.index(True)
    expect = [0] * k_ref + [1] * (len(ref.steps) - k_ref)
    h = _handle(p)
    u, s, lam, z, steps, conv = h.ip_solve(f, g0, Ms=Ms, Mu=Mu, tol=1e-8, switch_ratio=ratio)
    on = [st["filter_on"] for st in steps]
    print(f"filter per step {on} (oracle's D range gives {expect}), PCG its "
          f"{[st['pcg_iterations'] for st in steps]}")
    assert conv and ref.converged and len(steps) == len(ref.steps)
    assert on == expect
    k = on.index(1)
    assert all(st["D_max"] < ratio * st["D_min"] for st in steps[:k])
    assert steps[k]["D_max"] >= ratio * steps[k]["D_min"]
    u, z = u.cpu().numpy(), z.cpu().numpy()
    assert np.linalg.norm(u - ref.u) <= 1e-6 * np.linalg.norm(ref.u)
    assert np.linalg.norm(z - ref.z) <= 1e-6 * np.linalg.norm(ref.z)
    h2 = _handle(p)
    u2, *_ = h2.ip_solve(f, g0, Ms=Ms, Mu=Mu, tol=1e-8)
    assert np.linalg.norm(u - u2.cpu().numpy()) <= 1e-5 * np.linalg.norm(u)
    h.close()
    h2.close()
