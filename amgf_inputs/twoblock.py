"""Two-body contact test problem (paper Sec. 2.2 and Sec. 4, synthetic stand-in).

Geometry: two unit cubes, the *bottom* body on [0,1]^3 and the *top* body on
[0,1]^2 x [1,2], each meshed with N^3 trilinear hexahedra (Q1), 3 displacement DOFs
per node.  Node numbering: bottom body first, id = i + (N+1)*(j + (N+1)*k) with
(i, j, k) the lattice position; the top body follows with an offset of (N+1)^3.

* K: block-diagonal (per body) linear-elasticity stiffness with Lame parameters from
  (E, nu) per body (Sec. 2.2, the energy functional and Hooke's law).  Stored as a
  symmetric BSR matrix with 3x3 node blocks on the full 27-point node stencil.
  A Dirichlet DOF keeps its diagonal entry and loses every other entry of its row
  and column (the block stays stored), so it is decoupled and scale-consistent.
  K is bitwise symmetric: every block is a sum over the shared elements in ascending
  element order of an exactly symmetric element matrix.
* BCs: bottom face of the bottom body clamped; top face of the top body on rollers
  (u_x = u_y = 0, u_z free), so that S = K + J^T D J is SPD through the contact term.
  The paper's model problem (Sec. 4) drives the top face instead; that variant
  (``top_bc="clamped"``) is available too.
* J: one normal-gap row per node of the top body's bottom face (the non-mortar
  side, Sec. 4): +1 on its z DOF and -1/4 on the z DOFs of the four corners of the
  facing bottom-body face element.  Rows sum to zero.  Shape m x n with
  m = (N+1)^2, 5 nonzeros per row, columns ascending.
* D: the log-barrier Hessian diagonal (Sec. 3, D = diag(M_s z / s)).  Either drawn
  log-uniformly from a seed, or from a synthetic interior-point sequence
  (``ip_sequence_D``).
* b: standard normal from a seed, zero on Dirichlet DOFs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

__all__ = ["TwoBlockProblem", "make_two_block", "q1_element_matrices",
           "ip_sequence_D", "CONFIGS", "BLOCK_CONFIGS", "make_config"]


# --------------------------------------------------------------------------------------
# Q1 element matrices
# --------------------------------------------------------------------------------------
def q1_element_matrices():
    """Return (K_lambda, K_mu), each (8, 8, 3, 3), for the unit cube element.

    The element stiffness for Lame parameters (lam, mu) and edge length h is
    h * (lam * K_lambda + mu * K_mu).  Local node l = cx + 2 cy + 4 cz for the corner
    (cx, cy, cz) in {0,1}^3.  2x2x2 Gauss quadrature (exact for this integrand).
    Both matrices are made exactly symmetric.
    """
    g = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
    corners = np.array([[l & 1, (l >> 1) & 1, (l >> 2) & 1] for l in range(8)], dtype=float)
    Kl = np.zeros((8, 8, 3, 3))
    Km = np.zeros((8, 8, 3, 3))
    for qz in g:
        for qy in g:
            for qx in g:
                xi = np.array([qx, qy, qz])
                # dN_l / dxi_d
                grad = np.zeros((8, 3))
                for l in range(8):
                    f = np.where(corners[l] == 1, xi, 1.0 - xi)
                    df = np.where(corners[l] == 1, 1.0, -1.0)
                    grad[l, 0] = df[0] * f[1] * f[2]
                    grad[l, 1] = f[0] * df[1] * f[2]
                    grad[l, 2] = f[0] * f[1] * df[2]
                w = 1.0 / 8.0
                # lambda term: d_p N_a d_q N_b
                Kl += w * np.einsum("ap,bq->abpq", grad, grad)
                # mu term: delta_pq grad N_a . grad N_b + d_q N_a d_p N_b
                dot = grad @ grad.T
                Km += w * (np.einsum("ab,pq->abpq", dot, np.eye(3))
                           + np.einsum("aq,bp->abpq", grad, grad))
    # exact symmetry: K[a,b,p,q] == K[b,a,q,p]
    Kl = 0.5 * (Kl + Kl.transpose(1, 0, 3, 2))
    Km = 0.5 * (Km + Km.transpose(1, 0, 3, 2))
    return Kl, Km


def _lame(E, nu):
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


# per-axis element options: (class, offset) -> list of (corner of a, corner of b) in
# ascending element index.  class 0: i == 0, 1: interior, 2: i == N.
_AXIS_OPTS = {
    (0, 0): [(0, 0)], (1, 0): [(1, 1), (0, 0)], (2, 0): [(1, 1)],
    (0, 1): [(0, 1)], (1, 1): [(0, 1)], (2, 1): [],
    (0, -1): [], (1, -1): [(1, 0)], (2, -1): [(1, 0)],
}


def _block_table(Ke):
    """Table T[cz, cy, cx, slot] (3x3 blocks) of assembled node-pair blocks.

    slot = (oz+1)*9 + (oy+1)*3 + (ox+1).  Each entry is the sum over the elements
    shared by the node pair, in ascending global element order (z outermost), so
    the (a, b) and (b, a) blocks are exact transposes of each other.
    """
    T = np.zeros((3, 3, 3, 27, 3, 3))
    for cz in range(3):
        for cy in range(3):
            for cx in range(3):
                for oz in (-1, 0, 1):
                    for oy in (-1, 0, 1):
                        for ox in (-1, 0, 1):
                            s = (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1)
                            acc = np.zeros((3, 3))
                            for (az, bz) in _AXIS_OPTS[(cz, oz)]:
                                for (ay, by) in _AXIS_OPTS[(cy, oy)]:
                                    for (ax, bx) in _AXIS_OPTS[(cx, ox)]:
                                        la = ax + 2 * ay + 4 * az
                                        lb = bx + 2 * by + 4 * bz
                                        acc = acc + Ke[la, lb]
                            T[cz, cy, cx, s] = acc
    return T


# --------------------------------------------------------------------------------------
# problem container
# --------------------------------------------------------------------------------------
@dataclass
class TwoBlockProblem:
    N: int
    n_nodes: int
    K_rowptr: np.ndarray      # int32 (n_nodes+1)
    K_col: np.ndarray         # int32 (nnzb)
    K_val: np.ndarray         # float64 (nnzb, 3, 3)
    J_rowptr: np.ndarray      # int32 (m+1)
    J_col: np.ndarray         # int32 (nnz)
    J_val: np.ndarray         # float64 (nnz)
    D: np.ndarray             # float64 (m)
    b: np.ndarray             # float64 (n)
    coords: np.ndarray        # float64 (n_nodes, 3)
    free: np.ndarray          # bool (n) : False on Dirichlet DOFs
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return 3 * self.n_nodes

    @property
    def m(self):
        return len(self.D)

    @property
    def nnzb(self):
        return len(self.K_col)


def _body_stiffness(N, E, nu, free_body):
    """BSR arrays of one body's stiffness (local node numbering)."""
    n1 = N + 1
    h = 1.0 / N
    lam, mu = _lame(E, nu)
    Kl, Km = q1_element_matrices()
    Ke = h * (lam * Kl + mu * Km)                       # exactly symmetric
    T = _block_table(Ke).reshape(27, 27, 3, 3)           # [class, slot]

    idx = np.arange(n1)
    cls1 = np.where(idx == 0, 0, np.where(idx == N, 2, 1)).astype(np.int64)
    # per-axis validity of offsets -1, 0, +1
    val1 = np.stack([idx >= 1, np.ones(n1, bool), idx <= N - 1], axis=1)   # (n1, 3)

    # slots in (oz, oy, ox) lexicographic order == ascending neighbour id
    nn = n1 ** 3
    k_, j_, i_ = np.meshgrid(idx, idx, idx, indexing="ij")
    i_ = i_.ravel(); j_ = j_.ravel(); k_ = k_.ravel()
    node_cls = (cls1[k_] * 9 + cls1[j_] * 3 + cls1[i_])
    valid = (val1[k_][:, :, None, None] & val1[j_][:, None, :, None]
             & val1[i_][:, None, None, :]).reshape(nn, 27)
    counts = valid.sum(axis=1)
    rowptr = np.zeros(nn + 1, np.int64)
    np.cumsum(counts, out=rowptr[1:])
    rows, slots = np.nonzero(valid)                       # row-major: sorted by row, slot
    so = np.array([(s // 9 - 1) * n1 * n1 + (s // 3 % 3 - 1) * n1 + (s % 3 - 1)
                   for s in range(27)], dtype=np.int64)
    cols = rows + so[slots]
    vals = T[node_cls[rows], slots]                       # (nnzb, 3, 3)
    del valid

    # Dirichlet: identity rows/columns on constrained DOFs (DOF-wise, blocks kept)
    # the constrained DOF keeps its original diagonal entry (scale-consistent with
    # the rest of the row block), its off-diagonal row and column entries become 0
    fb = free_body.reshape(nn, 3).astype(np.float64)
    cons_node = (fb < 1.0).any(axis=1)
    touch = cons_node[rows] | cons_node[cols]
    tb = np.nonzero(touch)[0]
    diag = tb[rows[tb] == cols[tb]]
    kept = vals[diag][:, [0, 1, 2], [0, 1, 2]]            # (nd, 3) original diagonal
    fr = fb[rows[tb]]
    fc = fb[cols[tb]]
    vals[tb] = vals[tb] * fr[:, :, None] * fc[:, None, :]
    dfix = (1.0 - fb[rows[diag]]) * kept
    vals[diag] = vals[diag] + dfix[:, :, None] * np.eye(3)[None]
    return rowptr, cols, vals


def make_two_block(N, E=(1.0, 1.0), nu=(0.3, 0.3), top_bc="roller",
                   D_log10=(0.0, 8.0), D_seed=1, D=None, rhs_seed=11, contact=True):
    """Build the two-body problem with N^3 Q1 elements per body.

    E, nu: (bottom, top) material constants.  top_bc: "roller" (default), "clamped"
    or "free".  D: explicit barrier diagonal (length (N+1)^2); otherwise
    log10 D ~ U(D_log10) from ``D_seed``.  contact=False gives J with zero rows
    (m = 0), the contact-free operator.
    """
    N = int(N)
    n1 = N + 1
    nb = n1 ** 3
    n_nodes = 2 * nb
    free = np.ones((n_nodes, 3), bool)
    bottom_face = np.arange(n1 * n1)                      # body 0, k = 0
    free[bottom_face] = False
    top_face = nb + N * n1 * n1 + np.arange(n1 * n1)      # body 1, k = N
    if top_bc == "roller":
        free[top_face, 0] = False
        free[top_face, 1] = False
    elif top_bc == "clamped":
        free[top_face] = False
    elif top_bc != "free":
        raise ValueError(top_bc)

    rp0, c0, v0 = _body_stiffness(N, E[0], nu[0], free[:nb])
    rp1, c1, v1 = _body_stiffness(N, E[1], nu[1], free[nb:])
    K_rowptr = np.concatenate([rp0, rp1[1:] + rp0[-1]]).astype(np.int32)
    K_col = np.concatenate([c0, c1 + nb]).astype(np.int32)
    K_val = np.concatenate([v0, v1])
    del v0, v1

    idx = np.arange(n1)
    kk, ii = np.meshgrid(idx, idx, indexing="ij")         # row r = i + n1*j
    jj_, ii_ = kk.ravel(), ii.ravel()
    if contact:
        m = n1 * n1
        ip = np.minimum(ii_, N - 1)
        jp = np.minimum(jj_, N - 1)
        mortar_base = N * n1 * n1
        c00 = mortar_base + ip + n1 * jp
        cols = np.stack([c00, c00 + 1, c00 + n1, c00 + n1 + 1,
                         nb + ii_ + n1 * jj_], axis=1)
        J_col = (3 * cols + 2).astype(np.int32).ravel()
        J_val = np.tile(np.array([-0.25, -0.25, -0.25, -0.25, 1.0]), m)
        J_rowptr = (5 * np.arange(m + 1)).astype(np.int32)
        if D is None:
            rng = np.random.default_rng(D_seed)
            D = 10.0 ** rng.uniform(D_log10[0], D_log10[1], m)
        D = np.ascontiguousarray(D, dtype=np.float64)
        assert D.shape == (m,)
    else:
        m = 0
        J_col = np.zeros(0, np.int32)
        J_val = np.zeros(0)
        J_rowptr = np.zeros(1, np.int32)
        D = np.zeros(0)

    rng = np.random.default_rng(rhs_seed)
    b = rng.standard_normal(3 * n_nodes)
    freef = free.ravel()
    b[~freef] = 0.0

    kz, jy, ix = np.meshgrid(idx, idx, idx, indexing="ij")
    base = np.stack([ix.ravel() / N, jy.ravel() / N, kz.ravel() / N], axis=1)
    top = base.copy()
    top[:, 2] += 1.0
    coords = np.concatenate([base, top])

    meta = dict(N=N, E=tuple(E), nu=tuple(nu), top_bc=top_bc, D_log10=tuple(D_log10),
                D_seed=D_seed, rhs_seed=rhs_seed, contact=contact)
    return TwoBlockProblem(N=N, n_nodes=n_nodes, K_rowptr=K_rowptr, K_col=K_col,
                           K_val=np.ascontiguousarray(K_val), J_rowptr=J_rowptr,
                           J_col=J_col, J_val=J_val, D=D, b=b, coords=coords,
                           free=freef, meta=meta)


def ip_sequence_D(m, t, seed=4, mu0=0.1, factor=0.3):
    """Barrier diagonal of step t (1-based) of a synthetic interior-point sequence.

    mu_t = mu0 * factor^(t-1); one uniform draw u_k per constraint (shared by all
    steps) gives slack s_k = mu_t^{u_k} (log-uniform on [mu_t, 1]) and dual
    z_k = mu_t / s_k; with a unit lumped slack mass, D_k = z_k / s_k (Sec. 3).
    """
    rng = np.random.default_rng(seed)
    u = rng.uniform(0.0, 1.0, m)
    mu = mu0 * factor ** (t - 1)
    s = mu ** u
    z = mu / s
    return z / s


# workload presets: sizes, materials and seeds of the five benchmark configurations
CONFIGS = {
    "C1": dict(N=8, E=(1.0, 1.0), nu=(0.3, 0.3), D_log10=(0.0, 8.0), D_seed=1, rhs_seed=11),
    "C2": dict(N=32, E=(1.0, 1.0), nu=(0.3, 0.3), D_log10=(0.0, 10.0), D_seed=2, rhs_seed=21),
    "C3": dict(N=64, E=(1.0, 100.0), nu=(0.45, 0.45), D_log10=(0.0, 12.0), D_seed=3, rhs_seed=31),
    "C4": dict(N=32, E=(1.0, 1.0), nu=(0.3, 0.3), ip_seed=4),
    "C5": dict(N=128, E=(1.0, 1.0), nu=(0.3, 0.3), D_log10=(0.0, 12.0), D_seed=5, rhs_seed=51),
}


# small block (E = 1000, nu = 0) on a large block (E = 1, nu = 0.45) with non-matching
# interface meshes (Nb = 7/8 Nt over a top block of half the width, so the bottom mesh is
# about 2.3 times coarser at the interface); m = (Nt + 1)^2 equals Table 1's m_max for
# Nt = 8 * 2^(k-1)
BLOCK_CONFIGS = {
    "B1": dict(Nt=8, Nb=7, D_log10=(0.0, 8.0), D_seed=61, rhs_seed=71),
    "B2": dict(Nt=16, Nb=14, D_log10=(0.0, 8.0), D_seed=62, rhs_seed=72),
    "B3": dict(Nt=64, Nb=56, D_log10=(0.0, 12.0), D_seed=63, rhs_seed=73),
    "B5": dict(Nt=128, Nb=112, D_log10=(0.0, 12.0), D_seed=65, rhs_seed=75),
}


def make_config(name, rhs_seed=None, ip_step=None, N=None):
    """Build one of the presets.  C4 needs ``ip_step`` (1..20); its rhs seed is 40+t.
    B1..B5 are the non-matching block-on-block problems."""
    if name in BLOCK_CONFIGS:
        from .block_on_block import make_block_on_block
        c = dict(BLOCK_CONFIGS[name])
        if rhs_seed is not None:
            c["rhs_seed"] = rhs_seed
        return make_block_on_block(c.pop("Nt"), c.pop("Nb"), E=(1.0, 1000.0),
                                   nu=(0.45, 0.0), **c)
    c = dict(CONFIGS[name])
    if N is not None:
        c["N"] = N
    if name == "C4":
        t = int(ip_step)
        n1 = c["N"] + 1
        D = ip_sequence_D(n1 * n1, t, seed=c.pop("ip_seed"))
        rs = 40 + t if rhs_seed is None else rhs_seed
        return make_two_block(c["N"], c["E"], c["nu"], D=D, rhs_seed=rs)
    if rhs_seed is not None:
        c["rhs_seed"] = rhs_seed
    return make_two_block(**c)


def renumber_nodes(p, seed):
    """The same problem with the nodes numbered by a seeded random permutation: node a of
    ``p`` becomes node perm[a] (its three DOFs move together; meta["node_perm"] = perm).  K keeps ascending block
    columns per row and J ascending columns per row, so the result is a valid input in
    which stored blocks lie far from the diagonal (the matrix bandwidth becomes about the
    node count)."""
    rng = np.random.default_rng(seed)
    nn = p.n_nodes
    perm = rng.permutation(nn)                 # old node -> new node
    inv = np.argsort(perm)                     # new node -> old node
    rows_old = np.repeat(np.arange(nn), np.diff(p.K_rowptr))
    rows_new = perm[rows_old]
    cols_new = perm[p.K_col]
    order = np.lexsort((cols_new, rows_new))
    K_rowptr = np.zeros(nn + 1, np.int64)
    np.cumsum(np.bincount(rows_new, minlength=nn), out=K_rowptr[1:])
    K_col = cols_new[order].astype(np.int32)
    K_val = np.ascontiguousarray(p.K_val[order])
    jcol = 3 * perm[p.J_col // 3] + p.J_col % 3
    J_col = np.empty_like(p.J_col)
    J_val = np.empty_like(p.J_val)
    for k in range(p.m):
        s, e = p.J_rowptr[k], p.J_rowptr[k + 1]
        o = np.argsort(jcol[s:e], kind="stable")
        J_col[s:e] = jcol[s:e][o]
        J_val[s:e] = p.J_val[s:e][o]
    dof_old = (3 * inv[:, None] + np.arange(3)[None, :]).ravel()   # new DOF -> old DOF
    meta = dict(p.meta, renumber_seed=seed, node_perm=perm)
    return TwoBlockProblem(N=p.N, n_nodes=nn, K_rowptr=K_rowptr.astype(np.int32),
                           K_col=K_col, K_val=K_val, J_rowptr=p.J_rowptr.copy(),
                           J_col=J_col.astype(np.int32), J_val=J_val, D=p.D.copy(),
                           b=p.b[dof_old], coords=p.coords[inv], free=p.free[dof_old],
                           meta=meta)
