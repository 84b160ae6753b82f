"""GPU V-cycle, AMGF apply and PCG against the oracle (FP64 and mixed precision)."""
import numpy as np
import pytest

from gpu_util import MIXED_TOL, MIXED_TOL_FP32_TRANSFERS, gpu, oracle, problem, rel
from oracle_util import extended_solution

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,opts", [("C1", {}), ("C1", {"coarse_max_nodes": 8}),
                                       ("N12", {"coarse_max_nodes": 16}), ("B1", {}),
                                       ("B2", {})])
def test_operator_vcycle_and_apply_fp64(name, opts):
    import torch
    o = oracle(name, **opts)
    h = gpu(name, **opts)
    rng = np.random.default_rng(1)
    r = rng.standard_normal(o.n)
    assert rel(h.operator(r).cpu().numpy(), o.A_apply(r)) < 1e-14
    assert rel(h.vcycle(r).cpu().numpy(), o.vcycle(r)) < 1e-10
    # r2 = r - A z2 cancels on the contact rows after the exact filter correction:
    # its rounding error is u * D_max * |z2| there (D spans 8 decades in these cases),
    # so the two FP64 evaluations agree to ~1e-8, not to u.
    z, zr = h.apply(r).cpu().numpy(), o.apply(r)
    S = o.S.csr()
    e = z - zr
    e_A = float(np.sqrt(e @ (S @ e)) / np.sqrt(zr @ (S @ zr)))
    print(f"{name}: apply rel {rel(z, zr):.2e}, energy-norm rel {e_A:.2e}")
    assert rel(z, zr) < 5e-8 and e_A < 5e-8
    torch.cuda.synchronize()
    h.close()


def test_apply_fp64_tight_for_moderate_barrier():
    """With D <= 1e2 the residual cancellation is mild and M r agrees to 1e-11."""
    from amgf_inputs import make_two_block
    from oracle import OracleAMGF
    from paper_2505_18576_amd import AMGF
    p = make_two_block(8, D_log10=(0.0, 2.0), D_seed=21, rhs_seed=22)
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords)
    h = AMGF.from_problem(p)
    r = np.random.default_rng(3).standard_normal(o.n)
    e_v = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    print(f"moderate D: vcycle rel {e_v:.2e}, apply rel {e_m:.2e}")
    assert e_v < 1e-12 and e_m < 1e-11
    h.close()


@pytest.mark.parametrize("precision,fp16,tol", [(1, 1, MIXED_TOL), (2, 1, 2e-2),
                                                (1, 0, MIXED_TOL_FP32_TRANSFERS)])
def test_apply_mixed_precision_close_to_fp64(precision, fp16, tol):
    # FP32 values: relative rounding 6e-8 per entry; FP16 transfer values 4.9e-4; BF16
    # stiffness values (precision 2): 3.9e-3
    o = oracle("C1")
    h = gpu("C1", precision=precision, transfer_fp16=fp16)
    rng = np.random.default_rng(2)
    r = rng.standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    print(f"precision {precision}: vcycle rel {e_b:.2e} apply rel {e_m:.2e}")
    assert e_b < tol and e_m < tol
    h.close()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_pcg_matches_oracle(precision):
    p = problem("C1")
    o = oracle("C1")
    ref = o.pcg(p.b)
    h = gpu("C1", precision=precision)
    x, info = h.pcg(p.b)
    x = x.cpu().numpy()
    # reference: the solution of A x = b from an extended-precision refinement (shares
    # nothing with either solver); the oracle's own rtol-1e-10 iterate is about 2e-11 from it
    xs = extended_solution(p)
    err, err_o = rel(x, xs), rel(ref.x, xs)
    e = x - xs
    err_S = float(np.sqrt(e @ o.A_apply(e)) / np.sqrt(xs @ o.A_apply(xs)))
    print(f"precision {precision}: gpu {info.iterations} it, oracle {ref.iterations} it, "
          f"rel err vs exact {err:.2e} (oracle iterate {err_o:.2e}), S-norm {err_S:.2e}, "
          f"gpu vs oracle iterate {rel(x, ref.x):.2e}, true res {info.rel_true_res:.2e}")
    assert info.converged and info.rel_prec_res <= 1e-10
    assert info.ms_setup_amg > 0 and info.ms_setup_filter > 0 and info.ms_solve > 0
    if precision == 0:
        assert abs(info.iterations - ref.iterations) <= 1
    else:
        assert info.iterations <= ref.iterations + (5 if precision == 1 else 10)
    # FP64-equivalent: within 1e-8 of the exact solution and of the oracle's iterate
    assert err <= 1e-8 and err_S <= 1e-8 and rel(x, ref.x) <= 1e-8
    h.close()


def test_pcg_tight_tolerance_reaches_exact_solution():
    """With the stopping rule tightened to 1e-13 the FP64 and mixed-precision GPU solutions
    stay within 1e-8 of the exact solution of C1: the FP32 V-cycle limits only the rate, not
    the attainable accuracy of the FP64 outer iteration."""
    p = problem("C1")
    o = oracle("C1")
    xs = extended_solution(p)
    for precision in (0, 1):
        h = gpu("C1", precision=precision, rtol=1e-13)
        x, info = h.pcg(p.b)
        err = rel(x.cpu().numpy(), xs)
        print(f"precision {precision} rtol 1e-13: {info.iterations} it, converged "
              f"{info.converged}, rel err vs exact {err:.2e}")
        assert err <= 1e-8
        h.close()


def test_error_codes():
    from paper_2505_18576_amd import AMGF, AMGFError
    from paper_2505_18576_amd import amgf as b
    p = problem("C1")
    D = p.D.copy()
    D[3] = -1.0
    with pytest.raises(AMGFError) as ei:
        AMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val.reshape(-1), p.J_rowptr, p.J_col,
             p.J_val, D, p.coords.reshape(-1))
    assert ei.value.status == b.AMGF_EINVAL
    K = p.K_val.copy()
    K[5, 1, 1] = np.nan
    with pytest.raises(AMGFError) as ei:
        AMGF(p.n_nodes, p.K_rowptr, p.K_col, K.reshape(-1), p.J_rowptr, p.J_col, p.J_val,
             p.D, p.coords.reshape(-1))
    assert ei.value.status == b.AMGF_EINVAL
    h = gpu("C1", max_iters=2)
    x, info = h.pcg(p.b)
    assert info.iterations == 2 and not info.converged
    with pytest.raises(AMGFError) as ei:
        h.pcg(p.b, raise_on_noconv=True)
    assert ei.value.status == b.AMGF_ENOCONV
    h.close()


def test_pcg_run_to_run_bitwise():
    p = problem("C1")
    h = gpu("C1")
    x1, i1 = h.pcg(p.b)
    x2, i2 = h.pcg(p.b)
    assert i1.iterations == i2.iterations
    assert np.array_equal(x1.cpu().numpy().view(np.uint64), x2.cpu().numpy().view(np.uint64))
    h.close()


@pytest.mark.parametrize("kw", [dict(), dict(precision=1), dict(smoother=1)])
def test_three_level_vcycle_and_apply_match_oracle(kw):
    """C2 has a smoothed coarse level between level 0 and the coarsest one; its contact
    term goes through J_1 and D (fewer bytes than the assembled block there)."""
    oo = {"smoother": "chebyshev"} if kw.get("smoother") == 1 else {}
    o = oracle("C2", **oo)
    h = gpu("C2", **kw)
    assert h.n_levels >= 3 and o.nlev == h.n_levels
    rng = np.random.default_rng(12)
    r = rng.standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    print(f"C2 {kw}: levels {h.n_levels}, vcycle rel {e_b:.2e}, apply rel {e_m:.2e}")
    tol = MIXED_TOL if kw.get("precision") else 1e-10
    assert e_b <= tol
    # the residual r - A z inside M cancels on contact rows: FP64 error about u * D_max |z|
    u = np.finfo(np.float64).eps / 2
    dmax = float(problem("C2").D.max())
    assert e_m <= max(MIXED_TOL if kw.get("precision") else 0.0, 10 * u * dmax)
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_assembled_coarse_contact_level(precision):
    """N = 16 coarsened to at most 4 nodes: level 2 (31 nodes) meets every constraint, and
    its assembled block C_2 reads fewer bytes than J_2 and D, so level 2 smooths with
    A_2 = K_2 + C_2 itself (packed rows, FP32 in the mixed cycle); level 1 adds its contact
    term through J_1 and D.  V-cycle, M r and PCG against the oracle (which forms J^T D J)."""
    from amgf_inputs import make_two_block
    from oracle import OracleAMGF, OracleOptions
    from paper_2505_18576_amd import AMGF
    p = make_two_block(16, D_log10=(0.0, 8.0), D_seed=9, rhs_seed=10)
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords, OracleOptions(coarse_max_nodes=4))
    print(f"[gpu setup] N=16 coarse_max_nodes=4 precision {precision}", flush=True)
    h = AMGF.from_problem(p, coarse_max_nodes=4, precision=precision)
    assert h.n_levels == o.nlev == 4
    modes = [h.contact_mode(l) for l in range(4)]
    assert [m[0] for m in modes] == [1, 1, 2, 0], modes
    rng = np.random.default_rng(14)
    r = rng.standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    ref = o.pcg(p.b, rtol=1e-13)
    its10 = next(k for k, v in enumerate(ref.history) if v <= 1e-10)
    x, info = h.pcg(p.b)
    err = rel(x.cpu().numpy(), ref.x)
    print(f"precision {precision}: contact modes {modes}, vcycle rel {e_b:.2e}, apply rel "
          f"{e_m:.2e}, {info.iterations} it (oracle {its10}), solution rel err {err:.2e}")
    u = np.finfo(np.float64).eps / 2
    assert e_b <= (1e-10 if precision == 0 else MIXED_TOL)
    assert e_m <= max(MIXED_TOL if precision else 0.0, 10 * u * float(p.D.max()))
    assert info.converged and err <= 1e-8
    if precision == 0:
        assert abs(info.iterations - its10) <= 1
    else:
        assert info.iterations <= its10 + 5
    h.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_phase_breakdown_sums_to_solve_time(precision):
    """info splits the device time of the solve into the V-cycles, the filter correction
    and the rest of CG (the split Sec. 7 reports); the parts cover the whole solve."""
    p = problem("C2")
    h = gpu("C2", precision=precision)
    x, info = h.pcg(p.b)
    parts = (info.ms_amg_apply, info.ms_filter_apply, info.ms_cg_other)
    print(f"C2 precision {precision}: solve {info.ms_solve:.2f} ms = V-cycles {parts[0]:.2f} "
          f"+ filter {parts[1]:.2f} + other CG {parts[2]:.2f} ({info.iterations} it)")
    assert info.converged and all(t > 0 for t in parts)
    assert abs(sum(parts) - info.ms_solve) <= 0.02 * info.ms_solve
    h.close()


@pytest.mark.parametrize("case,precision", [("C2", 0), ("C2", 1), ("N16", 0), ("N16", 1)])
def test_w_cycle_matches_oracle(case, precision):
    """cycle_gamma = 2 (the W-cycle; not in the paper): C2 (three levels: level 1 visited
    twice) and N = 16 coarsened to 4 nodes (four levels, an assembled contact level
    visited four times).  V-cycle operator, M r and PCG against the oracle's W-cycle."""
    from amgf_inputs import make_two_block
    from oracle import OracleAMGF, OracleOptions
    from paper_2505_18576_amd import AMGF
    if case == "C2":
        p, kw = problem("C2"), {}
    else:
        p, kw = make_two_block(16, D_log10=(0.0, 8.0), D_seed=9, rhs_seed=10), \
            {"coarse_max_nodes": 4}
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords, OracleOptions(cycle_gamma=2, **kw))
    print(f"[gpu setup] {case} cycle_gamma=2 precision {precision}", flush=True)
    h = AMGF.from_problem(p, cycle_gamma=2, precision=precision, **kw)
    assert h.n_levels == o.nlev
    rng = np.random.default_rng(15)
    r = rng.standard_normal(o.n)
    e_b = rel(h.vcycle(r).cpu().numpy(), o.vcycle(r))
    e_m = rel(h.apply(r).cpu().numpy(), o.apply(r))
    ref = o.pcg(p.b, rtol=1e-13)
    its10 = next(k for k, v in enumerate(ref.history) if v <= 1e-10)
    x, info = h.pcg(p.b)
    err = rel(x.cpu().numpy(), ref.x)
    print(f"{case} W precision {precision}: levels {o.nlev}, vcycle rel {e_b:.2e}, apply rel "
          f"{e_m:.2e}, {info.iterations} it (oracle {its10}), solution rel err {err:.2e}")
    u = np.finfo(np.float64).eps / 2
    assert e_b <= (1e-10 if precision == 0 else MIXED_TOL)
    assert e_m <= max(MIXED_TOL if precision else 0.0, 10 * u * float(p.D.max()))
    assert info.converged and err <= 1e-8
    if precision == 0:
        assert abs(info.iterations - its10) <= 1
    else:
        assert info.iterations <= its10 + 5
    h.close()
