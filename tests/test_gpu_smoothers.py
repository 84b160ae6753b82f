"""GPU parity of the smoother options (Chebyshev, several sweeps) against the oracle."""
import numpy as np
import pytest

from oracle_util import extended_solution
from gpu_util import MIXED_TOL, gpu, oracle, problem, rel

pytestmark = pytest.mark.gpu

CASES = [
    ("C1", dict(smoother=1)),
    ("C1", dict(smoother=1, cheb_degree=3)),
    ("C1", dict(sweeps=2)),
    ("N12", dict(smoother=1, sweeps=2)),
]


def _oracle_opts(kw):
    o = {}
    if kw.get("smoother") == 1:
        o["smoother"] = "chebyshev"
    for k in ("sweeps", "cheb_degree"):
        if k in kw:
            o[k] = kw[k]
    return o


@pytest.mark.parametrize("name,kw", CASES)
def test_vcycle_and_apply_match_oracle(name, kw):
    o = oracle(name, **_oracle_opts(kw))
    h = gpu(name, **kw)
    rng = np.random.default_rng(3)
    r = rng.standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    print(f"{name} {kw}: vcycle rel {e_b:.2e}, apply rel {e_m:.2e}")
    assert e_b <= 1e-10
    assert e_m <= 5e-8          # same cancellation bar as the l1-Jacobi apply (large D)
    h.close()


@pytest.mark.parametrize("name,kw", CASES[:3])
def test_pcg_matches_oracle(name, kw):
    p = problem(name)
    o = oracle(name, **_oracle_opts(kw))
    ref = o.pcg(p.b)
    h = gpu(name, **kw)
    x, info = h.pcg(p.b)
    x = x.cpu().numpy()
    # reference: the solution of A x = b from an extended-precision refinement
    xs = extended_solution(p)
    err, err_o = rel(x, xs), rel(ref.x, xs)
    print(f"{name} {kw}: gpu {info.iterations} it, oracle {ref.iterations} it, error vs exact "
          f"{err:.2e} (oracle {err_o:.2e}), gpu vs oracle {rel(x, ref.x):.2e}")
    assert info.converged and abs(info.iterations - ref.iterations) <= 1
    assert err <= 1e-8 and rel(x, ref.x) <= 1e-8
    h.close()


@pytest.mark.parametrize("precision", [1, 2])
def test_mixed_chebyshev_close_to_fp64(precision):
    o = oracle("C1", smoother="chebyshev")
    h = gpu("C1", smoother=1, precision=precision)
    rng = np.random.default_rng(4)
    r = rng.standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    tol = MIXED_TOL if precision == 1 else 2e-2
    print(f"precision {precision} Chebyshev vcycle rel {e_b:.2e}")
    assert e_b <= tol
    x, info = h.pcg(problem("C1").b)
    assert info.converged
    h.close()


def test_option_errors():
    from paper_2505_18576_amd import amgf as b
    p = problem("C1")
    with pytest.raises(b.AMGFError):
        b.AMGF.from_problem(p, sweeps=0)
    with pytest.raises(b.AMGFError):
        b.AMGF.from_problem(p, smoother=1, cheb_degree=0)
    h = gpu("C1", smoother=1)
    W = np.zeros(b.MLP_NTOTAL, np.float32)
    W[1319:1325] = 1.0
    with pytest.raises(b.AMGFError):
        h.set_mlp(W)
    with pytest.raises(b.AMGFError):
        h.loss_grad(W, np.zeros((h.n, 1)), 2)
    h.close()
