"""Seeded random inputs of the learned-smoother training: probe vectors and the initial
MLP parameter vector (1313 weights and biases followed by 6 means and 6 deviations)."""
import math

import numpy as np

NPARAM = 1313
NTOTAL = 1325


def probes(n, free, count, seed):
    """(n, count) Gaussian probe columns, zero on constrained DOFs."""
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((n, count))
    P[~np.asarray(free, bool)] = 0.0
    return P


def init_params(seed=0, mu=None, sd=None, last_scale=0.0):
    """Uniform Glorot-scaled first two layers; the last layer is zero by default so
    that training starts from theta = 1 (plain l1-Jacobi)."""
    rng = np.random.default_rng(seed)
    W = np.zeros(NTOTAL)
    W[0:192] = rng.uniform(-1, 1, 192) * math.sqrt(6.0 / (6 + 32))
    W[224:1248] = rng.uniform(-1, 1, 1024) * math.sqrt(6.0 / (32 + 32))
    if last_scale:
        W[1280:1312] = rng.uniform(-1, 1, 32) * last_scale
    W[1313:1319] = 0.0 if mu is None else mu
    W[1319:1325] = 1.0 if sd is None else sd
    return W.astype(np.float32)
