"""Load vector and initial gap of the two-body contact problem that the interior-point
driver solves: a uniform downward pressure on the top face of the top body (whose top face
is on rollers, so the body is held up by contact alone) and a curved initial gap between
the bodies, so that part of the interface closes and part stays open.

Data only: the optimisation itself lives in the GPU library and, independently, in the
CPU oracle.
"""
from __future__ import annotations

import numpy as np


def contact_load_and_gap(p, pressure=0.05, gap0=0.0, curvature=0.2):
    """f (n) and g0 (m) for a problem from ``make_two_block``.

    f: nodal forces -pressure * (lattice area of the node) in z on the top face of the
    top body (interior nodes 1/N^2, edge nodes half, corner nodes a quarter).
    g0: initial normal gap of constraint k, the non-mortar node at (x, y) on the
    interface: gap0 + curvature * ((x - 1/2)^2 + (y - 1/2)^2).
    """
    if "nm_xy" in p.meta:          # geometry carried by the problem (block on block)
        f = np.zeros(p.n)
        f[3 * p.meta["load_nodes"] + 2] = -pressure * p.meta["load_area"]
        x, y = p.meta["nm_xy"][:, 0], p.meta["nm_xy"][:, 1]
        cx, cy = p.meta["center"]
        g0v = gap0 + curvature * ((x - cx) ** 2 + (y - cy) ** 2)
        assert g0v.shape == (p.m,)
        return f, g0v
    N = p.N
    n1 = N + 1
    nb = n1 ** 3
    w = np.ones(n1)
    w[0] = w[-1] = 0.5
    area = np.outer(w, w).ravel() / N ** 2              # index i + n1 * j
    top_face = nb + N * n1 * n1 + np.arange(n1 * n1)
    f = np.zeros(p.n)
    f[3 * top_face + 2] = -pressure * area
    r = np.arange(n1 * n1)
    x = (r % n1) / N
    y = (r // n1) / N
    g0v = gap0 + curvature * ((x - 0.5) ** 2 + (y - 0.5) ** 2)
    assert g0v.shape == (p.m,)
    return f, g0v


def lumped_masses(p):
    """Diagonal lumped masses of the lattice: Ms (m) the interface area of each constraint's
    non-mortar node, Mu (n) the volume of each node, repeated for its three DOFs (interior
    weights 1/N^2 and 1/N^3, halved once per boundary the node lies on)."""
    if "nm_area" in p.meta:
        Ms = np.asarray(p.meta["nm_area"], np.float64)
        Mu = np.repeat(np.asarray(p.meta["node_vol"], np.float64), 3)
        assert Ms.shape == (p.m,) and Mu.shape == (p.n,)
        return Ms, Mu
    N = p.N
    n1 = N + 1
    w = np.ones(n1)
    w[0] = w[-1] = 0.5
    Ms = np.outer(w, w).ravel() / N ** 2
    vol = (w[:, None, None] * w[None, :, None] * w[None, None, :]).ravel() / N ** 3
    Mu = np.repeat(np.concatenate([vol, vol]), 3)
    assert Ms.shape == (p.m,) and Mu.shape == (p.n,)
    return Ms, Mu


def bound_barrier(p, seed=0, log10_range=(-2.0, 4.0), fraction=0.7):
    """Barrier diagonal E (n values >= 0) of bound constraints on the displacements
    (Remark 3.1): log-uniform on a random `fraction` of the free DOFs, 0 elsewhere."""
    rng = np.random.default_rng(seed)
    E = 10.0 ** rng.uniform(log10_range[0], log10_range[1], p.n)
    E[(rng.uniform(size=p.n) >= fraction) | ~p.free] = 0.0
    return E
