"""Non-matching interface (small stiff block on a large soft block, bilinear node-to-segment
mortar rows): PCG and the interior-point driver against the oracle."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg  # noqa: F401

from gpu_util import gpu, oracle, problem, rel
from oracle_util import extended_solution

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,precision", [("B1", 0), ("B1", 1), ("B2", 0)])
def test_pcg_matches_oracle(name, precision):
    p = problem(name)
    o = oracle(name)
    ref = o.pcg(p.b)
    h = gpu(name, precision=precision)
    x, info = h.pcg(p.b)
    x = x.cpu().numpy()
    # reference: the solution of A x = b from an extended-precision refinement (shares
    # nothing with either solver); the oracle's own iterate is about 2e-11 from it
    xs = extended_solution(p)
    err, err_o = rel(x, xs), rel(ref.x, xs)
    e = x - xs
    err_S = float(np.sqrt(e @ o.A_apply(e)) / np.sqrt(xs @ o.A_apply(xs)))
    print(f"{name} precision {precision}: gpu {info.iterations} it, oracle {ref.iterations} "
          f"it, error vs exact {err:.2e} (oracle {err_o:.2e}), S-norm {err_S:.2e}, "
          f"gpu vs oracle {rel(x, ref.x):.2e}, n_c {info.n_c}")
    assert info.converged and info.n_c == o.n_c
    if precision == 0:
        assert abs(info.iterations - ref.iterations) <= 1
    else:
        assert info.iterations <= ref.iterations + 5
    assert err <= 1e-8 and err_S <= 1e-8 and rel(x, ref.x) <= 1e-8
    h.close()


def test_ip_matches_oracle_nonmatching():
    from amgf_inputs import contact_load_and_gap, lumped_masses
    from oracle.ip_newton import IPOptions, ip_solve, kkt_certificate
    p = problem("B1")
    K = sp.bsr_matrix((p.K_val, p.K_col, p.K_rowptr), shape=(p.n, p.n)).tocsr()
    J = sp.csr_matrix((p.J_val, p.J_col, p.J_rowptr), shape=(p.m, p.n))
    f, g0 = contact_load_and_gap(p)
    Ms, Mu = lumped_masses(p)
    ref = ip_solve(K, J, f, g0, IPOptions(tol=1e-8), Ms=Ms, Mu=Mu)
    h = gpu("B1")
    u, s, lam, z, steps, conv = h.ip_solve(f, g0, Ms=Ms, Mu=Mu, tol=1e-8)
    u, lam = u.cpu().numpy(), lam.cpu().numpy()
    print(f"B1 IP: gpu {len(steps)} steps, oracle {len(ref.steps)}; PCG its "
          f"{[st['pcg_iterations'] for st in steps]}")
    assert conv and ref.converged and len(steps) == len(ref.steps)
    assert rel(u, ref.u) <= 1e-6
    stat, infeas, dneg, compl = kkt_certificate(K, J, f, g0, u, -lam)
    assert stat <= 1e-7 and infeas == 0.0 and dneg == 0.0 and compl <= 1e-7
    h.close()
