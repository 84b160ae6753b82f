"""Helpers shared by the GPU parity tests (run on the MI355X only)."""
import functools

import numpy as np

from amgf_inputs import make_config, make_two_block
from oracle import OracleAMGF, OracleOptions


@functools.lru_cache(maxsize=None)
def problem(name, **kw):
    if name.startswith("N"):
        return make_two_block(int(name[1:]), D_log10=(0.0, 8.0), D_seed=9, rhs_seed=10)
    return make_config(name, **kw)


@functools.lru_cache(maxsize=None)
def oracle(name, **opts):
    p = problem(name)
    return OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                      p.D, p.coords, OracleOptions(**opts))


def gpu(name, **opts):
    from paper_2505_18576_amd import AMGF
    p = problem(name)
    print(f"[gpu setup] {name} opts={opts}", flush=True)
    return AMGF.from_problem(p, **opts)


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
