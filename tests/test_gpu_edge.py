"""Degenerate cases on the GPU against the oracle: no contact (m = 0, an empty filtering
space, so M = 2B - BAB; also with a coarse level that has no contact term), a hierarchy of one dense level (B = A^{-1}, so CG stops after one
step), and the filter switched off (M = B)."""
import numpy as np
import pytest

from amgf_inputs import make_two_block
from gpu_util import MIXED_TOL, rel
from oracle import OracleAMGF, OracleOptions

pytestmark = pytest.mark.gpu


def _pair(p, **opts):
    """GPU handle and oracle built from the same problem and options."""
    from paper_2505_18576_amd import AMGF
    oo = {k: (bool(v) if k == "filter" else v) for k, v in opts.items()
          if k in ("coarse_max_nodes", "filter")}
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords, OracleOptions(**oo))
    print(f"[gpu setup] n_nodes {p.n_nodes} m {len(p.J_rowptr) - 1} opts {opts}", flush=True)
    return AMGF.from_problem(p, **opts), o


def test_no_contact_matches_oracle():
    p = make_two_block(8, contact=False, top_bc="clamped", rhs_seed=31)
    assert len(p.J_rowptr) == 1
    h, o = _pair(p)
    assert o.n_c == 0 and o.nlev > 1
    r = np.random.default_rng(32).standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    x, info = h.pcg(p.b)
    ref = o.pcg(p.b)
    e_x = rel(x.cpu().numpy(), ref.x)
    print(f"no contact: vcycle {e_b:.2e}, apply {e_m:.2e}, its {info.iterations} / "
          f"{ref.iterations}, solution {e_x:.2e}")
    assert e_b <= 1e-10 and e_m <= 1e-10
    assert info.converged and abs(info.iterations - ref.iterations) <= 1
    assert e_x <= 1e-8
    h.close()


def test_no_contact_mixed_precision():
    p = make_two_block(8, contact=False, top_bc="clamped", rhs_seed=33)
    h, o = _pair(p, precision=1)
    r = np.random.default_rng(34).standard_normal(o.n)
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    x, info = h.pcg(p.b)
    e_x = rel(x.cpu().numpy(), o.pcg(p.b).x)
    print(f"no contact, FP32 V-cycle: apply {e_m:.2e}, its {info.iterations}, solution {e_x:.2e}")
    assert e_m <= MIXED_TOL
    assert info.converged and e_x <= 1e-8
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_no_contact_three_levels(precision):
    """No contact with a smoothed coarse level between level 0 and the coarsest one (N = 12,
    three levels): the coarse V-cycle levels have no contact term at all."""
    p = make_two_block(12, contact=False, top_bc="clamped", rhs_seed=37)
    h, o = _pair(p, coarse_max_nodes=32, precision=precision)
    assert o.n_c == 0 and o.nlev == 3 and h.n_levels == 3
    r = np.random.default_rng(38).standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    x, info = h.pcg(p.b)
    ref = o.pcg(p.b)
    e_x = rel(x.cpu().numpy(), ref.x)
    print(f"no contact, three levels, precision {precision}: vcycle {e_b:.2e}, its "
          f"{info.iterations} / {ref.iterations}, solution {e_x:.2e}")
    assert e_b <= (1e-10 if precision == 0 else MIXED_TOL)
    assert info.converged and e_x <= 1e-8
    if precision == 0:
        assert abs(info.iterations - ref.iterations) <= 1
    h.close()


def test_single_level_is_a_direct_solve():
    # 2 x 27 nodes: below the coarsening threshold, so the hierarchy is one dense level
    p = make_two_block(2, D_log10=(0.0, 4.0), rhs_seed=35)
    h, o = _pair(p)
    assert h.n_levels == 1 and o.nlev == 1
    A = o.S.csr().toarray()
    r = np.random.default_rng(36).standard_normal(o.n)
    z = h.vcycle(r).cpu().numpy()
    e_b = rel(z, np.linalg.solve(A, r))
    x, info = h.pcg(p.b)
    e_x = rel(x.cpu().numpy(), np.linalg.solve(A, p.b))
    print(f"one level: B r vs A^-1 r {e_b:.2e}, its {info.iterations}, solution {e_x:.2e}")
    # cond(A) is about 1e6 here: both sides agree to cond(A) times the FP64 unit roundoff
    assert e_b <= 1e-9
    assert info.converged and info.iterations <= 2 and e_x <= 1e-9
    h.close()


def test_filter_off_apply_is_the_vcycle():
    p = make_two_block(8, rhs_seed=37)
    h, o = _pair(p, filter=0)
    r = np.random.default_rng(38).standard_normal(o.n)
    zb = h.vcycle(r).cpu().numpy()
    zm = h.apply(r).cpu().numpy()
    assert np.array_equal(zb.view(np.uint64), zm.view(np.uint64))
    assert rel(zm, o.apply(r)) <= 1e-10
    h.close()
