"""GPU hierarchy setup against the oracle: operator and aggregation bit-exact,
prolongators and Galerkin operators to FP64 rounding."""
import numpy as np
import pytest

from gpu_util import gpu, oracle, problem, rel

pytestmark = pytest.mark.gpu

CASES = [("C1", {}), ("C1", {"coarse_max_nodes": 8}), ("N12", {"coarse_max_nodes": 16}),
         ("B1", {}), ("B2", {})]


def _blocks_equal(o_bm, rp, col, val, exact):
    assert np.array_equal(o_bm.rowptr, rp)
    assert np.array_equal(o_bm.col, col)
    if exact:
        assert np.array_equal(o_bm.val, val)          # == : bitwise up to the sign of zero
    else:
        return rel(val, o_bm.val)


@pytest.mark.parametrize("name,opts", CASES)
def test_level0_operator_is_bit_exact(name, opts):
    o = oracle(name, **opts)
    h = gpu(name, **opts)
    L = h.level_arrays(0)
    _blocks_equal(o.S, L["A_rowptr"], L["A_col"], L["A_val"], exact=True)
    assert np.array_equal(L["l1"], o.levels[0].d) or rel(L["l1"], o.levels[0].d) < 1e-15
    h.close()


@pytest.mark.parametrize("name,opts", CASES)
def test_aggregation_is_bit_exact_on_every_level(name, opts):
    o = oracle(name, **opts)
    h = gpu(name, **opts)
    assert h.n_levels == o.nlev
    for l in range(o.nlev - 1):
        L = h.level_arrays(l)
        ol = o.levels[l]
        rp, cl, _ = ol.G
        assert np.array_equal(L["G_rowptr"], rp), l
        assert np.array_equal(L["G_col"], cl), l
        assert np.array_equal(L["root"].astype(bool), ol.roots), l
        assert np.array_equal(L["agg"], ol.agg), l
        assert L["n_agg"] == ol.n_agg
    h.close()


@pytest.mark.parametrize("name,opts", CASES)
def test_prolongators_and_coarse_operators(name, opts):
    o = oracle(name, **opts)
    h = gpu(name, **opts)
    for l in range(o.nlev - 1):
        L = h.level_arrays(l)
        ol = o.levels[l]
        rho, omega = L["rho_omega"]
        assert abs(rho - ol.rho) <= 1e-12 * ol.rho and abs(omega - ol.omega) <= 1e-12 * ol.omega
        e = _blocks_equal(ol.P, L["P_rowptr"], L["P_col"], L["P_val"], exact=False)
        assert e < 1e-12, (l, e)
        nx = h.level_arrays(l + 1)
        on = o.levels[l + 1]
        assert rel(nx["l1"], on.d) < 1e-12
        e = _blocks_equal(on.K, nx["K_rowptr"], nx["K_col"], nx["K_val"], exact=False)
        assert e < 1e-12, (l, e)
        e = _blocks_equal(on.A, nx["A_rowptr"], nx["A_col"], nx["A_val"], exact=False)
        assert e < 1e-12, (l, e)
    ic = h.filter_dofs(o.n_c)
    assert np.array_equal(ic, o.Ic)
    h.close()


def test_setup_is_deterministic():
    a = gpu("C1", coarse_max_nodes=8)
    b = gpu("C1", coarse_max_nodes=8)
    for l in range(a.n_levels - 1):
        La, Lb = a.level_arrays(l), b.level_arrays(l)
        for k in ("A_val", "P_val", "agg", "l1"):
            assert np.array_equal(La[k].view(np.uint8), Lb[k].view(np.uint8)), (l, k)
    a.close()
    b.close()
