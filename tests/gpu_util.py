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


# V-cycle and preconditioner bar of the FP32 modes against the FP64 oracle.  The transfer
# operators are stored in FP16 by default (unit roundoff 2^-11 = 4.9e-4): a V-cycle with
# FP16-rounded prolongators differs from the FP64 one by about 0.4 of that (oracle replay:
# 1.7e-4 on C1, 2.2e-4 on C2), so the bar is two units, 1e-3.  With FP32 transfers
# (transfer_fp16 = 0) the FP32 arithmetic alone keeps it below 1e-4.
MIXED_TOL = 1e-3
MIXED_TOL_FP32_TRANSFERS = 1e-4
