"""Oracle PCG behaviour: convergence, robustness to D and mesh refinement (Sec. 6)."""
import math

import numpy as np
import pytest

from amgf_inputs import make_config, make_two_block
from oracle_util import build, extended_solution


def test_c1_amgf_pcg_converges_and_solves():
    p = make_config("C1")
    o = build(p)
    res = o.pcg(p.b)
    assert res.converged and res.iterations < 80
    A = o.S.todense()
    x = np.linalg.solve(A, p.b)
    e = res.x - x
    # the relative preconditioned residual controls the energy-norm error
    assert math.sqrt(e @ A @ e) <= 1e-7 * math.sqrt(x @ A @ x)
    assert np.linalg.norm(p.b - A @ res.x) <= 1e-6 * np.linalg.norm(p.b)


def test_amg_without_filter_degrades_with_barrier_range():
    """AMG-PCG iterations blow up as D_max grows, AMGF-PCG stays flat (Sec. 4)."""
    its = {}
    for hi in (0.0, 4.0, 8.0):
        p = make_two_block(4, D_log10=(0.0, hi), D_seed=3, rhs_seed=4)
        amg = build(p, filter=False, max_iters=3000, coarse_max_nodes=16).pcg(p.b)
        amgf = build(p, coarse_max_nodes=16).pcg(p.b)
        assert amgf.converged
        its[hi] = (amg.iterations, amgf.iterations)
    assert its[8.0][0] > 3 * its[0.0][0]
    assert its[8.0][1] <= its[0.0][1] + 10


def test_iteration_bound_and_mesh_independence():
    """AMGF-PCG iterations stay below sqrt(2(beta+3)/beta) x the contact-free AMG-PCG
    count, beta = kappa of contact-free AMG (Sec. 6.1 bound procedure, Remark 5.6)."""
    its = []
    for N in (4, 8, 16):
        cf = make_two_block(N, contact=False, top_bc="clamped", rhs_seed=5)
        rcf = build(cf, filter=False, coarse_max_nodes=16).pcg(cf.b)
        lo, hi = rcf.lanczos_extremes()
        beta = hi / lo
        p = make_two_block(N, D_log10=(0.0, 10.0), D_seed=6, rhs_seed=5)
        r = build(p, coarse_max_nodes=16).pcg(p.b)
        assert r.converged
        bound = math.ceil(math.sqrt(2 * (beta + 3) / beta) * rcf.iterations) + 2
        assert r.iterations <= bound, (N, r.iterations, bound)
        its.append(r.iterations)
    assert its[-1] <= 2.5 * its[0]


def test_pcg_iterates_converge_to_the_solution_of_the_schur_system():
    """C1 (kappa about 6e11, D up to 1e8): the rtol-1e-10 iterate is within 1e-9 of the
    solution of A x = b and the rtol-1e-13 iterate within 1e-12, measured against an
    extended-precision solve that shares nothing with the oracle's operator apply.  A CG
    operator that rounded the assembled entries of J^T D J would be stuck near 1e-8 here."""
    p = make_config("C1")
    o = build(p)
    xs = extended_solution(p)
    r10, r13 = o.pcg(p.b), o.pcg(p.b, rtol=1e-13)
    e10 = np.linalg.norm(r10.x - xs) / np.linalg.norm(xs)
    e13 = np.linalg.norm(r13.x - xs) / np.linalg.norm(xs)
    assert r10.converged and r13.converged
    assert e10 <= 1e-9 and e13 <= 1e-12, (e10, e13)
    # the same solve through the assembled operator S stalls at its entry rounding
    from oracle.amgf_oracle import pcg
    Sc = o.S.csr()
    rS = pcg(lambda v: Sc @ v, o.apply, p.b, rtol=1e-13)
    assert np.linalg.norm(rS.x - xs) / np.linalg.norm(xs) > 100 * e13
