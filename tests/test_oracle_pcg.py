"""Oracle PCG behaviour: convergence, robustness to D and mesh refinement (Sec. 6)."""
import math

import numpy as np
import pytest

from amgf_inputs import make_config, make_two_block
from oracle_util import build


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
