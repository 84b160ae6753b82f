"""Small block on a large block with non-matching meshes at the contact interface (the
paper's two-block model problem of Sec. 4 has a small cube resting on a larger block, the
cube's bottom face being the non-mortar side; synthetic stand-in).

Geometry: the bottom body is the unit cube [0,1]^3 with Nb^3 Q1 hexahedra; the top body is
a cube of side `width` on [a, a+width]^2 x [1, 1+width] with Nt^3 hexahedra (a centres it),
so the two interface meshes do not match.  Node numbering as in ``make_two_block``: bottom
body first, then the top body.

* K: per-body linear elasticity (Lame parameters from (E, nu) per body); the top body's
  stiffness is its unit-cube stiffness scaled by `width` (a Q1 element matrix scales with
  the element size in 3D).
* BCs: bottom face of the bottom body clamped; top face of the top body on rollers (or
  clamped).
* J: one normal-gap row per node of the top body's bottom face: +1 on its z DOF and minus
  the bilinear interpolation weights of its position in the facing bottom-body face element
  on that element's four corner z DOFs (a node-to-segment mortar; weights that vanish
  because a node sits on a grid line are not stored).  Columns ascending.
* D, b: as in ``make_two_block`` (log-uniform D from a seed, b ~ N(0,1) on free DOFs).
"""
from __future__ import annotations

import numpy as np

from .twoblock import TwoBlockProblem, _body_stiffness


def _lattice_weights(n1):
    w = np.ones(n1)
    w[0] = w[-1] = 0.5
    return w


def make_block_on_block(Nt, Nb, width=0.5, E=(1.0, 1.0), nu=(0.3, 0.3), top_bc="roller",
                        D_log10=(0.0, 8.0), D_seed=1, rhs_seed=11):
    """Build the problem.  E, nu: (bottom, top).  Returns a TwoBlockProblem whose N is Nt
    and whose meta holds the geometry used by the load, gap and mass helpers."""
    Nt, Nb = int(Nt), int(Nb)
    nt1, nb1 = Nt + 1, Nb + 1
    nb = nb1 ** 3
    nt = nt1 ** 3
    n_nodes = nb + nt
    a = 0.5 * (1.0 - width)
    free = np.ones((n_nodes, 3), bool)
    free[np.arange(nb1 * nb1)] = False                        # bottom face, k = 0
    top_face = nb + Nt * nt1 * nt1 + np.arange(nt1 * nt1)     # top body, k = Nt
    if top_bc == "roller":
        free[top_face, 0] = False
        free[top_face, 1] = False
    elif top_bc == "clamped":
        free[top_face] = False
    else:
        raise ValueError(top_bc)

    rp0, c0, v0 = _body_stiffness(Nb, E[0], nu[0], free[:nb])
    rp1, c1, v1 = _body_stiffness(Nt, E[1], nu[1], free[nb:])
    v1 = v1 * width
    K_rowptr = np.concatenate([rp0, rp1[1:] + rp0[-1]]).astype(np.int32)
    K_col = np.concatenate([c0, c1 + nb]).astype(np.int32)
    K_val = np.ascontiguousarray(np.concatenate([v0, v1]))

    # non-mortar nodes: the top body's bottom face (k = 0), row r = i + nt1 * j
    r = np.arange(nt1 * nt1)
    it, jt = r % nt1, r // nt1
    x = a + width * it / Nt
    y = a + width * jt / Nt
    m = nt1 * nt1
    cols, vals, rowptr = [], [], [0]
    mortar_base = Nb * nb1 * nb1                              # bottom body, k = Nb
    for k in range(m):
        fx, fy = x[k] * Nb, y[k] * Nb
        ib = min(int(np.floor(fx)), Nb - 1)
        jb = min(int(np.floor(fy)), Nb - 1)
        xi, eta = fx - ib, fy - jb
        xi = 0.0 if abs(xi) < 1e-12 else (1.0 if abs(xi - 1.0) < 1e-12 else xi)
        eta = 0.0 if abs(eta) < 1e-12 else (1.0 if abs(eta - 1.0) < 1e-12 else eta)
        c00 = mortar_base + ib + nb1 * jb
        corners = [(c00, (1 - xi) * (1 - eta)), (c00 + 1, xi * (1 - eta)),
                   (c00 + nb1, (1 - xi) * eta), (c00 + nb1 + 1, xi * eta)]
        for node, wgt in corners:
            if wgt != 0.0:
                cols.append(3 * node + 2)
                vals.append(-wgt)
        cols.append(3 * (nb + r[k]) + 2)
        vals.append(1.0)
        rowptr.append(len(cols))
    J_rowptr = np.asarray(rowptr, np.int32)
    J_col = np.asarray(cols, np.int32)
    J_val = np.asarray(vals, np.float64)

    rng = np.random.default_rng(D_seed)
    D = 10.0 ** rng.uniform(D_log10[0], D_log10[1], m)
    rng = np.random.default_rng(rhs_seed)
    b = rng.standard_normal(3 * n_nodes)
    freef = free.ravel()
    b[~freef] = 0.0

    ib_ = np.arange(nb1)
    kz, jy, ix = np.meshgrid(ib_, ib_, ib_, indexing="ij")
    base = np.stack([ix.ravel() / Nb, jy.ravel() / Nb, kz.ravel() / Nb], axis=1)
    it_ = np.arange(nt1)
    kz, jy, ix = np.meshgrid(it_, it_, it_, indexing="ij")
    top = np.stack([a + width * ix.ravel() / Nt, a + width * jy.ravel() / Nt,
                    1.0 + width * kz.ravel() / Nt], axis=1)
    coords = np.concatenate([base, top])

    wt = _lattice_weights(nt1)
    wb = _lattice_weights(nb1)
    face_area = np.outer(wt, wt).ravel() * (width / Nt) ** 2
    vol_b = (wb[:, None, None] * wb[None, :, None] * wb[None, None, :]).ravel() / Nb ** 3
    vol_t = ((wt[:, None, None] * wt[None, :, None] * wt[None, None, :]).ravel()
             * (width / Nt) ** 3)
    meta = dict(N=Nt, Nb=Nb, width=width, E=tuple(E), nu=tuple(nu), top_bc=top_bc,
                D_log10=tuple(D_log10), D_seed=D_seed, rhs_seed=rhs_seed,
                load_nodes=top_face, load_area=face_area,
                nm_xy=np.stack([x, y], axis=1), nm_area=face_area,
                node_vol=np.concatenate([vol_b, vol_t]), center=(0.5, 0.5))
    return TwoBlockProblem(N=Nt, n_nodes=n_nodes, K_rowptr=K_rowptr, K_col=K_col,
                           K_val=K_val, J_rowptr=J_rowptr, J_col=J_col, J_val=J_val, D=D,
                           b=b, coords=coords, free=freef, meta=meta)
