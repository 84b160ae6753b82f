"""Bound-constraint barrier terms (Remark 3.1, A = K + diag(E) + J^T D J) on the GPU against
the oracle: setup, V-cycle, AMGF apply and PCG with E, and the numeric re-setup for new D
and E (amgf_update_barrier)."""
import numpy as np
import pytest

from amgf_inputs import bound_barrier
from gpu_util import MIXED_TOL, problem, rel

pytestmark = pytest.mark.gpu

U = np.finfo(np.float64).eps / 2


def _oracle(p, E, **kw):
    from oracle import OracleAMGF, OracleOptions
    return OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                      p.D, p.coords, OracleOptions(**kw), E=E)


def _gpu(p, E, **kw):
    from paper_2505_18576_amd import AMGF
    print(f"[gpu setup] n={p.n} with bound terms {kw}", flush=True)
    return AMGF.from_problem(p, E=E, **kw)


@pytest.mark.parametrize("name", ["C1", "B1"])
def test_setup_and_solve_match_oracle(name):
    p = problem(name)
    E = bound_barrier(p, seed=1)
    o = _oracle(p, E)
    h = _gpu(p, E)
    L = h.level_arrays(0)
    assert np.array_equal(L["A_val"], o.S.val) and np.array_equal(L["A_col"], o.S.col)
    assert h.n_levels == o.nlev
    for l in range(o.nlev - 1):
        assert np.array_equal(h.level_arrays(l)["agg"], o.levels[l].agg), l
    r = np.random.default_rng(2).standard_normal(o.n)
    assert rel(h.operator(r).cpu().numpy(), o.A_apply(r)) < 1e-14
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    ref = o.pcg(p.b)
    x, info = h.pcg(p.b)
    e_x = rel(x.cpu().numpy(), ref.x)
    print(f"{name}: vcycle {e_b:.2e}, apply {e_m:.2e}; pcg gpu {info.iterations} it, oracle "
          f"{ref.iterations} it, rel diff {e_x:.2e}")
    assert e_b <= 1e-10 and e_m <= 5e-8
    assert info.converged and abs(info.iterations - ref.iterations) <= 1 and e_x <= 1e-7
    h.close()


@pytest.mark.parametrize("drop_E", [False, True])
def test_update_barrier_matches_oracle(drop_E):
    p = problem("C1")
    E = bound_barrier(p, seed=3)
    h = _gpu(p, E)
    same = _gpu(p, E)
    same.update_barrier(p.D, E)               # the same terms reproduce the setup bitwise
    r = np.random.default_rng(4).standard_normal(p.n)
    assert np.array_equal(same.apply(r).cpu().numpy(), h.apply(r).cpu().numpy())
    same.close()
    D2 = 10.0 ** np.random.default_rng(5).uniform(0.0, 6.0, p.m)
    E2 = None if drop_E else bound_barrier(p, seed=6, log10_range=(0.0, 6.0))
    o = _oracle(p, E)
    o.update_barrier(D2, E2)
    h.update_barrier(D2, E2)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    big = max(D2.max(), 0.0 if E2 is None else E2.max())
    print(f"drop_E={drop_E}: updated vcycle {e_b:.2e}, apply {e_m:.2e}")
    # coarse contact blocks: Galerkin on the GPU, J-based in the oracle (u * D_max apart)
    assert e_b <= max(1e-10, U * big) and e_m <= 10 * U * big
    ref = o.pcg(p.b)
    x, info = h.pcg(p.b)
    assert info.converged and abs(info.iterations - ref.iterations) <= 1
    assert rel(x.cpu().numpy(), ref.x) <= 1e-7
    h.close()


def test_mixed_precision_and_rejections():
    from paper_2505_18576_amd import amgf as b
    p = problem("C1")
    E = bound_barrier(p, seed=7)
    o = _oracle(p, E)
    h = _gpu(p, E, precision=1)
    r = np.random.default_rng(8).standard_normal(p.n)
    assert rel(h.vcycle(r).cpu().numpy(), o.vcycle(r)) <= MIXED_TOL
    x, info = h.pcg(p.b)
    assert info.converged
    bad = E.copy()
    bad[5] = -1.0
    with pytest.raises(b.AMGFError):
        h.update_barrier(p.D, bad)
    with pytest.raises(b.AMGFError):
        _gpu(p, bad)
    f = np.zeros(p.n)
    with pytest.raises(b.AMGFError):
        h.ip_solve(f, np.ones(p.m))
    h.close()
