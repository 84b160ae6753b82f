"""GPU branches the default workloads never reach: a coarsest level too large for the
explicit inverse (multifrontal coarsest factor), and level-0 stiffness whose stored blocks
lie beyond 16-bit column offsets of their row (int32 column ids in the sliced ELL copy)."""
import functools

import numpy as np
import pytest

from gpu_util import MIXED_TOL, rel

pytestmark = pytest.mark.gpu


@functools.lru_cache(maxsize=None)
def _two_level():
    from amgf_inputs import make_two_block
    return make_two_block(20, D_log10=(0.0, 8.0), D_seed=9, rhs_seed=10)


@functools.lru_cache(maxsize=None)
def _renumbered():
    from amgf_inputs import make_two_block, renumber_nodes
    return renumber_nodes(make_two_block(28, D_log10=(0.0, 8.0), D_seed=9, rhs_seed=10),
                          seed=5)


@functools.lru_cache(maxsize=None)
def _reference(which):
    """Oracle of the case, its rtol-1e-13 iterate and its rtol-1e-10 iteration count."""
    from oracle import OracleAMGF, OracleOptions
    p, kw = (_two_level(), {"max_levels": 2}) if which == "two_level" else (_renumbered(), {})
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords, OracleOptions(**kw))
    ref = o.pcg(p.b, rtol=1e-13)
    its10 = next(k for k, v in enumerate(ref.history) if v <= 1e-10)
    return o, ref, its10


@pytest.mark.parametrize("precision", [0, 1])
def test_multifrontal_coarsest_level(precision):
    """Two levels on N = 20: the coarsest operator has 3150 unknowns, above the 2048 of the
    explicit inverse, so the V-cycle's coarse solve is the multifrontal factor."""
    from paper_2505_18576_amd import AMGF
    p = _two_level()
    o, ref, its10 = _reference("two_level")
    print(f"[gpu setup] N=20 max_levels=2 precision {precision}", flush=True)
    h = AMGF.from_problem(p, max_levels=2, precision=precision)
    assert h.n_levels == 2 and o.level_sizes()[-1] == 3150
    r = np.random.default_rng(8).standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    x, info = h.pcg(p.b)
    err = rel(x.cpu().numpy(), ref.x)
    print(f"precision {precision}: vcycle rel {e_b:.2e}; {info.iterations} it (oracle "
          f"{its10}), solution rel err {err:.2e}")
    assert e_b <= (1e-10 if precision == 0 else MIXED_TOL)
    assert info.converged and err <= 1e-8
    if precision == 0:
        assert abs(info.iterations - its10) <= 1
    else:
        assert info.iterations <= its10 + 5
    h.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_int32_column_ids_sliced_ell(precision):
    """N = 28 with a seeded random node numbering: block columns lie up to 48,777 nodes
    from their row, so the level-0 sliced ELL copies store int32 column ids.  Operator
    bit-exact, V-cycle and PCG against the oracle on the same numbering."""
    from paper_2505_18576_amd import AMGF
    from paper_2505_18576_amd import amgf as b
    p = _renumbered()
    o, ref, its10 = _reference("renumbered")
    print(f"[gpu setup] renumbered N=28 precision {precision}", flush=True)
    h = AMGF.from_problem(p, precision=precision)
    assert int(h.query(0, b.Q_SIZES)[7]) == 4
    L = h.level_arrays(0)
    assert np.array_equal(L["A_col"], o.S.col) and np.array_equal(L["A_val"], o.S.val)
    r = np.random.default_rng(9).standard_normal(o.n)
    assert rel(h.operator(r).cpu().numpy(), o.A_apply(r)) <= 1e-14
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    x, info = h.pcg(p.b)
    err = rel(x.cpu().numpy(), ref.x)
    print(f"precision {precision}: vcycle rel {e_b:.2e}; {info.iterations} it (oracle "
          f"{its10}), solution rel err {err:.2e}")
    assert e_b <= (1e-10, MIXED_TOL, 2e-2)[precision]
    assert info.converged and err <= 1e-8
    if precision == 0:
        assert abs(info.iterations - its10) <= 1
    else:
        assert info.iterations <= its10 + (5 if precision == 1 else 10)
    h.close()
