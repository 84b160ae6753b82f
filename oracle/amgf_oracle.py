"""Plain FP64 CPU oracle of AMGF-preconditioned CG.  TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg may use this module.
It is slow and direct: every step is written from its definition, with numpy/scipy
primitives (sparse products, dense Cholesky, sparse LU) as the only library steps.

What it computes (paper references are to arXiv 2505.18576):

* the IP-Newton Schur complement A = K + J^T D J  (Sec. 3, the condensed system);
* an AMG V-cycle B on A with the convergent l1-Jacobi smoother (Remark 5.6 uses
  l1 smoothers so that B is convergent with omega = 1).  The paper's AMG is
  BoomerAMG, whose internals it does not give; here B is smoothed aggregation:
  level-0 strength of connection (coarse levels: aggregate adjacency),
  distance-2 maximal independent set aggregation,
  rigid-body-mode tentative prolongator, one damped-Jacobi prolongator smoothing
  step (damping sa_omega, default 1.5, over a power-iteration estimate of rho(D_l1^{-1} A)),
  Galerkin coarse operators, V(1,1), dense Cholesky on the coarsest level;
* the filtering space (Sec. 5.1): I_c = every DOF of a node touched by J, the
  embedding P and A_w = P^T A P, solved exactly by a Cholesky/LU factorisation;
* the multiplicative AMGF preconditioner M of Definition 5.3:
  I - M A = (I - B A)(I - P A_w^{-1} P^T A)(I - B A);
* preconditioned CG stopped on the relative preconditioned residual
  sqrt(r.Mr / r0.Mr0) < rtol with a cap on the iterations (Sec. 4, Sec. 6.1).

Readings where the paper is silent (SA internals, priorities, tie-breaks, rounding
order of the level-0 operator, dead near-null columns) are fixed here and stated
at the function that implements each of them.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np
import scipy.sparse as sp
import scipy.linalg as sla
import scipy.sparse.linalg as spla

__all__ = ["BlockMatrix", "OracleOptions", "OracleAMGF", "schur_operator",
           "strength_graph", "coarse_graph", "fmix32", "mis2_sequential", "aggregate",
           "gram_schmidt_qr", "pcg", "scalar_J_to_blocks"]


# ======================================================================================
# block sparse matrices
# ======================================================================================
class BlockMatrix:
    """Block-row sparse matrix with (br x bc) blocks and ascending columns per row."""

    def __init__(self, rowptr, col, val, ncols):
        self.rowptr = np.asarray(rowptr, np.int64)
        self.col = np.asarray(col, np.int64)
        self.val = np.asarray(val, np.float64)
        self.ncols = int(ncols)
        assert self.val.ndim == 3 and len(self.val) == len(self.col)
        self._csr = None

    @property
    def nrows(self):
        return len(self.rowptr) - 1

    @property
    def br(self):
        return self.val.shape[1]

    @property
    def bc(self):
        return self.val.shape[2]

    @property
    def nnzb(self):
        return len(self.col)

    @property
    def shape(self):
        return (self.nrows * self.br, self.ncols * self.bc)

    def row_index(self):
        return np.repeat(np.arange(self.nrows), np.diff(self.rowptr))

    def keys(self):
        return self.row_index() * self.ncols + self.col

    def csr(self):
        """Scalar CSR copy (all stored entries kept)."""
        if self._csr is None:
            br, bc = self.br, self.bc
            rows = (self.row_index()[:, None, None] * br
                    + np.arange(br)[None, :, None]) + 0 * np.arange(bc)[None, None, :]
            cols = (self.col[:, None, None] * bc + np.arange(bc)[None, None, :]) \
                + 0 * np.arange(br)[None, :, None]
            m = sp.coo_matrix((self.val.ravel(), (rows.ravel(), cols.ravel())),
                              shape=self.shape).tocsr()
            m.sort_indices()
            self._csr = m
        return self._csr

    def pattern(self):
        return sp.csr_matrix((np.ones(self.nnzb, np.int64), self.col, self.rowptr),
                             shape=(self.nrows, self.ncols))

    def transpose(self):
        rows = self.row_index()
        order = np.lexsort((rows, self.col))
        counts = np.bincount(self.col, minlength=self.ncols)
        rp = np.zeros(self.ncols + 1, np.int64)
        np.cumsum(counts, out=rp[1:])
        return BlockMatrix(rp, rows[order], self.val[order].transpose(0, 2, 1), self.nrows)

    def todense(self):
        return self.csr().toarray()

    def find(self, rows, cols):
        """Positions of blocks (rows[i], cols[i]); -1 where not stored."""
        k = self.keys()
        q = np.asarray(rows, np.int64) * self.ncols + np.asarray(cols, np.int64)
        pos = np.searchsorted(k, q)
        pos = np.minimum(pos, max(len(k) - 1, 0))
        ok = (len(k) > 0) & (k[pos] == q) if len(k) else np.zeros(len(q), bool)
        return np.where(ok, pos, -1)

    def diag_pos(self):
        return self.find(np.arange(self.nrows), np.arange(self.nrows))


def _from_pattern(pat, br, bc):
    pat = pat.tocsr()
    pat.sort_indices()
    return BlockMatrix(pat.indptr, pat.indices, np.zeros((pat.nnz, br, bc)), pat.shape[1])


def block_spgemm(A, B, keep_rows=None):
    """C = A B with the *structural* block pattern (no cancellation drops a block).

    The pattern is the product of the 0/1 block patterns; values come from the scalar
    sparse product (a library step) scattered into it.  ``keep_rows`` (bool per
    block row) restricts C to those rows.
    """
    pat = (A.pattern() @ B.pattern()).tocsr()
    if keep_rows is not None:
        pat = sp.diags(np.asarray(keep_rows, np.int64)) @ pat
        pat.eliminate_zeros()
    C = _from_pattern(pat, A.br, B.bc)
    X = (A.csr() @ B.csr()).tocoo()
    a = X.row // A.br
    Jc = X.col // B.bc
    if keep_rows is not None:
        sel = np.asarray(keep_rows, bool)[a]
        X = sp.coo_matrix((X.data[sel], (X.row[sel], X.col[sel])), shape=X.shape)
        a = a[sel]
        Jc = Jc[sel]
    pos = C.find(a, Jc)
    assert (pos >= 0).all()
    C.val[pos, X.row % A.br, X.col % B.bc] = X.data
    return C


def block_add(A, B):
    """A + B on the union pattern.  Blocks present in only one operand are copied
    exactly; shared blocks are added once (A + B)."""
    pat = (A.pattern() + B.pattern()).tocsr()
    C = _from_pattern(pat, A.br, A.bc)
    pa = C.find(A.row_index(), A.col)
    C.val[pa] = A.val
    pb = C.find(B.row_index(), B.col)
    C.val[pb] = C.val[pb] + B.val
    return C


def scalar_J_to_blocks(J_rowptr, J_col, J_val, n_nodes, bs=3):
    """m x n scalar CSR -> m x n_nodes block rows with 1 x bs blocks (node groups)."""
    m = len(J_rowptr) - 1
    rows = np.repeat(np.arange(m), np.diff(J_rowptr))
    node = np.asarray(J_col, np.int64) // bs
    comp = np.asarray(J_col, np.int64) % bs
    pat = sp.csr_matrix((np.ones(len(node), np.int64), (rows, node)), shape=(m, n_nodes))
    pat.sum_duplicates()
    Jb = _from_pattern(pat, 1, bs)
    pos = Jb.find(rows, node)
    Jb.val[pos, 0, comp] = J_val
    return Jb


# ======================================================================================
# O2: the Schur operator A = K + J^T D J  (Sec. 3)
# ======================================================================================
def contact_exact(Jb, D):
    """C = Jb^T diag(D) Jb, block form, with a fixed rounding order.

    Reading: C_ab(p,q) = sum over constraint rows k in ascending order of
    fl(D_k * fl(J_{k,a,p} * J_{k,b,q})), each product and sum rounded separately
    (no fused multiply-add), starting from 0.  The product J*J is formed first so
    that C is bitwise symmetric.
    """
    acc = {}
    for k in range(Jb.nrows):
        s, e = Jb.rowptr[k], Jb.rowptr[k + 1]
        nodes = Jb.col[s:e]
        v = Jb.val[s:e, 0, :]
        Dk = D[k]
        for ia in range(e - s):
            for ib in range(e - s):
                term = Dk * np.multiply.outer(v[ia], v[ib])
                key = (int(nodes[ia]), int(nodes[ib]))
                acc[key] = (acc[key] + term) if key in acc else (0.0 + term)
    bs = Jb.bc
    n = Jb.ncols
    if not acc:
        return BlockMatrix(np.zeros(n + 1, np.int64), np.zeros(0, np.int64),
                           np.zeros((0, bs, bs)), n)
    keys = sorted(acc)
    rows = np.array([k[0] for k in keys], np.int64)
    cols = np.array([k[1] for k in keys], np.int64)
    counts = np.bincount(rows, minlength=n)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    return BlockMatrix(rp, cols, np.stack([acc[k] for k in keys]), n)


def contact_product(Jb, D):
    """C = Jb^T diag(D) Jb on the structural pattern (coarse levels, library product)."""
    JT = Jb.transpose()
    Dm = BlockMatrix(np.arange(Jb.nrows + 1), np.arange(Jb.nrows),
                     np.asarray(D, float).reshape(-1, 1, 1), Jb.nrows)
    return block_spgemm(JT, block_spgemm(Dm, Jb))


def with_bound_diagonal(K, E):
    """K + diag(E) for the barrier terms of bound constraints (Remark 3.1: J~ = [J; I; -I]
    adds diag(D_lower + D_upper) = diag(E)); one add per diagonal entry.  E None: K."""
    if E is None:
        return K
    E = np.asarray(E, np.float64).reshape(-1, 3)
    Kt = BlockMatrix(K.rowptr, K.col, K.val.copy(), K.ncols)
    dp = Kt.diag_pos()
    for q in range(3):
        Kt.val[dp, q, q] = Kt.val[dp, q, q] + E[:, q]
    return Kt


def schur_operator(K, Jb, D):
    """Level-0 operator S = K + C with C from ``contact_exact`` and one final add."""
    return block_add(K, contact_exact(Jb, D))


# ======================================================================================
# O3: strength of connection (level 0)
# ======================================================================================
def block_sq_frobenius(A):
    """nu = sum of squared entries of each block, row-major, left to right, no FMA."""
    v = A.val.reshape(A.nnzb, -1)
    acc = np.zeros(A.nnzb)
    for e in range(v.shape[1]):
        acc = acc + v[:, e] * v[:, e]
    return acc


def strength_graph(A, theta):
    """Level-0 symmetric strength graph G (no self loops) with edge weights nu_ab.

    Reading (SA strength on node blocks, squared Frobenius norms nu):
    a ~ b iff fl(nu_ab^2) >= fl(theta4 * fl(nu_aa * nu_bb)) AND the same with (b, a),
    theta4 = fl(fl(theta^2)^2).
    """
    rows = A.row_index()
    off = rows != A.col
    nu = block_sq_frobenius(A)
    nd = nu[A.diag_pos()]
    t2 = theta * theta
    t4 = t2 * t2
    lhs = nu * nu
    rhs = t4 * (nd[rows] * nd[A.col])
    ok = lhs >= rhs
    tpos = A.find(A.col, rows)
    assert (tpos >= 0).all(), "operator pattern must be symmetric"
    lhs_t = nu[tpos] * nu[tpos]
    rhs_t = t4 * (nd[A.col] * nd[rows])
    keep = off & ok & (lhs_t >= rhs_t)
    counts = np.bincount(rows[keep], minlength=A.nrows)
    rp = np.zeros(A.nrows + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    return rp, A.col[keep], nu[keep]


def coarse_graph(rowptr, col, agg, n_agg):
    """Graph of the next level: aggregates I ~ J (I != J) iff some node of I has a
    graph edge to a node of J (the pattern of Q^T (G + I) Q, Q the 0/1 aggregate
    map).  Integer-only, so both implementations build it identically."""
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    a, b = agg[rows], agg[col]
    keep = (a >= 0) & (b >= 0) & (a != b)
    pat = sp.csr_matrix((np.ones(keep.sum(), np.int64), (a[keep], b[keep])),
                        shape=(n_agg, n_agg))
    pat.sum_duplicates()
    pat.sort_indices()
    return (pat.indptr.astype(np.int64), pat.indices.astype(np.int64),
            np.ones(pat.nnz))


# ======================================================================================
# O4/O5: MIS-2 aggregation
# ======================================================================================
def fmix32(a):
    """MurmurHash3 32-bit finalizer (a bijection of uint32), used as node priority."""
    h = np.asarray(a).astype(np.uint32)
    with np.errstate(over="ignore"):                 # arithmetic is mod 2^32
        h = h ^ (h >> np.uint32(16))
        h = h * np.uint32(0x85EBCA6B)
        h = h ^ (h >> np.uint32(13))
        h = h * np.uint32(0xC2B2AE35)
        h = h ^ (h >> np.uint32(16))
    return h


def priority_keys(n):
    ids = np.arange(n, dtype=np.uint64)
    return (fmix32(ids).astype(np.uint64) << np.uint64(32)) | ids


def mis2_sequential(rowptr, col, active):
    """Greedy distance-2 maximal independent set of G restricted to ``active`` nodes.

    Nodes are visited by descending priority key (fmix32(a), a); a node becomes a
    root when no root lies within graph distance 2.  (The GPU computes the same set
    by parallel rounds; this is the sequential definition.)
    """
    n = len(rowptr) - 1
    order = np.argsort(priority_keys(n), kind="stable")[::-1]
    blocked = np.zeros(n, bool)
    root = np.zeros(n, bool)
    for a in order:
        if not active[a] or blocked[a]:
            continue
        root[a] = True
        nb = col[rowptr[a]:rowptr[a + 1]]
        blocked[a] = True
        blocked[nb] = True
        for u in nb:
            blocked[col[rowptr[u]:rowptr[u + 1]]] = True
    return root


def aggregate(rowptr, col, weight, root, active, level):
    """Aggregates from the MIS-2 roots.

    Ids: roots numbered in ascending node order.  Phase 1: each root and its graph
    neighbours (a node touches at most one root since roots are >= 3 apart).
    Phase 2 (reads phase-1 state only): every other active node joins an adjacent
    phase-1 aggregate -- level 0: the one holding the neighbour with the largest
    edge weight nu_ab; levels >= 1: the one it has most edges into; ties go to the
    smallest aggregate id.  Inactive (isolated) nodes get -1.
    """
    n = len(rowptr) - 1
    rows = np.repeat(np.arange(n), np.diff(rowptr))
    agg_of_root = np.full(n, -1, np.int64)
    rid = np.nonzero(root)[0]
    agg_of_root[rid] = np.arange(len(rid))
    p1 = agg_of_root.copy()
    m = root[col] & ~root[rows]
    assert len(np.unique(rows[m])) == m.sum(), "node adjacent to two roots"
    p1[rows[m]] = agg_of_root[col[m]]
    agg = p1.copy()
    left = np.nonzero(active & (p1 < 0))[0]
    for v in left:
        nb = col[rowptr[v]:rowptr[v + 1]]
        wv = weight[rowptr[v]:rowptr[v + 1]]
        ids = p1[nb]
        ok = ids >= 0
        assert ok.any(), "MIS-2 maximality violated"
        ids = ids[ok]
        wv = wv[ok]
        if level == 0:
            best = None
            for J, w in zip(ids, wv):
                if best is None or w > best[0] or (w == best[0] and J < best[1]):
                    best = (w, J)
            agg[v] = best[1]
        else:
            u, c = np.unique(ids, return_counts=True)       # u ascending
            agg[v] = u[np.argmax(c)]                          # first max = smallest id
    return agg, len(rid)


# ======================================================================================
# O6: tentative prolongator from the near-null space
# ======================================================================================
def gram_schmidt_qr(B, tol):
    """QR of B by Gram-Schmidt with dead columns.

    Column j: v = component of b_j orthogonal to the live q_i (i < j), projected
    twice; if ||v|| <= tol * ||b_j|| (or b_j = 0) the column is dead: q_j = 0 and
    row j of R is 0.  Otherwise q_j = v / ||v||, R_jj = ||v|| > 0.
    """
    nr, k = B.shape
    Q = np.zeros((nr, k))
    R = np.zeros((k, k))
    dead = np.zeros(k, bool)
    for j in range(k):
        v = B[:, j].copy()
        nb = math.sqrt(float(v @ v))
        for _ in range(2):
            c = Q[:, :j].T @ v
            v = v - Q[:, :j] @ c
            R[:j, j] += c
        nv = math.sqrt(float(v @ v))
        if nb == 0.0 or nv <= tol * nb:
            dead[j] = True
            R[:j, j] = R[:j, j]
        else:
            Q[:, j] = v / nv
            R[j, j] = nv
    return Q, R, dead


def rigid_body_modes(coords_rel):
    """(k, 3, 6) rigid-body modes of nodes at positions coords_rel (about the origin):
    three translations, then rotations about x, y, z (omega x v)."""
    k = len(coords_rel)
    x, y, z = coords_rel[:, 0], coords_rel[:, 1], coords_rel[:, 2]
    B = np.zeros((k, 3, 6))
    B[:, 0, 0] = 1.0
    B[:, 1, 1] = 1.0
    B[:, 2, 2] = 1.0
    B[:, 1, 3] = -z
    B[:, 2, 3] = y
    B[:, 0, 4] = z
    B[:, 2, 4] = -x
    B[:, 0, 5] = -y
    B[:, 1, 5] = x
    return B


def group_members(agg, n_agg):
    order = np.argsort(agg, kind="stable")
    counts = np.bincount(agg[agg >= 0], minlength=n_agg)
    start = np.searchsorted(agg[order], 0)
    off = np.zeros(n_agg + 1, np.int64)
    np.cumsum(counts, out=off[1:])
    return order[start:], off


def tentative_prolongator(agg, n_agg, near_fn, br, tol, nc=6):
    """P_t (one block per aggregated row, column = its aggregate) and the coarse
    near-null blocks R_J (n_agg, nc, nc) plus the dead-column flags (n_agg, nc), for nc
    near-null vectors (6 rigid-body modes, or 3 translations)."""
    n = len(agg)
    members, off = group_members(agg, n_agg)
    Pval = np.zeros((n, br, nc))
    Rall = np.zeros((n_agg, nc, nc))
    dead = np.zeros((n_agg, nc), bool)
    for J in range(n_agg):
        nodes = members[off[J]:off[J + 1]]
        Bj = near_fn(J, nodes)                            # (k, br, nc)
        Q, R, dd = gram_schmidt_qr(Bj.reshape(-1, nc), tol)
        Pval[nodes] = Q.reshape(len(nodes), br, nc)
        Rall[J] = R
        dead[J] = dd
    keep = agg >= 0
    counts = keep.astype(np.int64)
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(counts, out=rp[1:])
    Pt = BlockMatrix(rp, agg[keep], Pval[keep], n_agg)
    return Pt, Rall, dead


def power_start(n):
    """Deterministic start vector x_i = fmix32(i) * 2^-32 - 1/2 (exact in FP64)."""
    return fmix32(np.arange(n)).astype(np.float64) * 2.0 ** -32 - 0.5


def power_estimate(Acsr, d, decoupled, iters, clip=True):
    """Spectral radius estimate of D_l1^{-1} A on the coupled DOFs.

    x_0 from ``power_start``; each step y = (A x) / d with decoupled entries zeroed,
    lam = ||y||_2, x = y / lam.  Returns min(1, lam) after ``iters`` steps (the l1
    diagonal already bounds the radius by 1), or lam itself with clip=False."""
    x = power_start(Acsr.shape[0])
    x[decoupled] = 0.0
    x = x / math.sqrt(float(x @ x))
    lam = 1.0
    for _ in range(iters):
        y = (Acsr @ x) / d
        y[decoupled] = 0.0
        lam = math.sqrt(float(y @ y))
        x = y / lam
    return min(1.0, lam) if clip else lam


# ======================================================================================
# options, levels, setup
# ======================================================================================
@dataclass
class OracleOptions:
    filter: bool = True
    max_levels: int = 10
    coarse_max_nodes: int = 1024
    strength_theta: float = 0.04
    sa_omega: float = 1.5                  # numerator; divided by the estimate below
    sa_power_iters: int = 10
    qr_tol: float = 1e-10
    max_coarse_ratio: float = 0.9
    rtol: float = 1e-10
    max_iters: int = 5000
    Ic: np.ndarray | None = None          # optional DOF list of the filter space
    theta: list | None = None             # per-level smoother damping (default 1)
    dense_filter_max: int = 8000
    near_null: int = 6                    # 6 rigid-body modes or 3 translations
    smoother: str = "jacobi"              # "jacobi" (l1-Jacobi) or "chebyshev"
    sweeps: int = 1                       # smoother applications before and after
    cheb_degree: int = 2                  # Chebyshev polynomial degree
    cycle_gamma: int = 1                  # coarse visits per level: 1 V-cycle, 2 W-cycle


@dataclass
class Level:
    A: BlockMatrix                        # assembled operator of this level
    K: BlockMatrix                        # stiffness part
    J: BlockMatrix                        # contact Jacobian part (m x nodes, 1 x b)
    d: np.ndarray = None                  # l1 row norms
    w: np.ndarray = None                  # smoother weights theta / d
    agg: np.ndarray = None
    n_agg: int = 0
    roots: np.ndarray = None
    G: tuple = None
    Pt: BlockMatrix = None
    P: BlockMatrix = None
    R: np.ndarray = None
    dead: np.ndarray = None
    decoupled: np.ndarray = None
    rho: float = 1.0
    lam: float = 1.0                      # unclipped power estimate of rho(D_l1^{-1} A)
    omega: float = 4.0 / 3.0


class OracleAMGF:
    """Setup + apply of the AMGF preconditioner and its PCG driver (FP64)."""

    def __init__(self, n_nodes, K_rowptr, K_col, K_val, J_rowptr, J_col, J_val, D,
                 coords, opts: OracleOptions | None = None, E=None):
        self.opts = opts or OracleOptions()
        o = self.opts
        self.n_nodes = int(n_nodes)
        self.D = np.asarray(D, np.float64)
        self.K_in = BlockMatrix(K_rowptr, K_col, np.asarray(K_val).reshape(-1, 3, 3), n_nodes)
        K0 = with_bound_diagonal(self.K_in, E)
        J0 = scalar_J_to_blocks(J_rowptr, J_col, J_val, n_nodes, 3)
        self.K0, self.J0 = K0, J0
        self.coords = None if coords is None else np.asarray(coords, np.float64).reshape(-1, 3)
        S = schur_operator(K0, J0, self.D)
        self.S = S
        self.levels = []
        A, K, J = S, K0, J0
        R_prev = None
        for l in range(o.max_levels):
            lev = Level(A=A, K=K, J=J)
            self.levels.append(lev)
            Acsr = A.csr()
            lev.d = np.asarray(abs(Acsr).sum(axis=1)).ravel()
            th = 1.0 if o.theta is None else np.asarray(o.theta[l], float)
            lev.w = th / lev.d
            if A.nrows <= o.coarse_max_nodes or l == o.max_levels - 1:
                break
            if l == 0:
                rp, cl, wt = strength_graph(A, o.strength_theta)
            else:
                rp, cl, wt = G_next
            active = np.diff(rp) > 0
            root = mis2_sequential(rp, cl, active)
            agg, n_agg = aggregate(rp, cl, wt, root, active, l)
            if n_agg == 0 or n_agg > o.max_coarse_ratio * A.nrows:
                break
            lev.G = (rp, cl, wt)
            lev.roots, lev.agg, lev.n_agg = root, agg, n_agg
            br = A.br
            if l == 0:
                lev.decoupled = self._decoupled_dofs(Acsr)
                near0 = self._level0_near(lev.decoupled)
                near_fn = near0
            else:
                Rp = R_prev
                near_fn = (lambda J_, nodes, Rp=Rp: Rp[nodes])
            Pt, R, dead = tentative_prolongator(agg, n_agg, near_fn, br, o.qr_tol,
                                                o.near_null)
            lev.Pt, lev.R, lev.dead = Pt, R, dead
            # O7: prolongator smoothing  P = P_t - omega D_l1^{-1} A P_t
            dec = lev.decoupled if l == 0 else np.zeros(A.nrows * br, bool)
            lev.lam = power_estimate(Acsr, lev.d, dec, o.sa_power_iters, clip=False)
            lev.rho = min(1.0, lev.lam)
            lev.omega = o.sa_omega / lev.rho
            APt = block_spgemm(A, Pt, keep_rows=agg >= 0)
            P = BlockMatrix(APt.rowptr, APt.col, APt.val.copy(), n_agg)
            dinv = (lev.omega / lev.d).reshape(A.nrows, br)
            P.val = -(APt.val * dinv[APt.row_index()][:, :, None])
            pos = P.find(np.nonzero(agg >= 0)[0], agg[agg >= 0])
            P.val[pos] = Pt.val + P.val[pos]
            lev.P = P
            # O8: Galerkin coarse operators
            PT = P.transpose()
            Kc = block_spgemm(PT, block_spgemm(K, P))
            dd = dead.reshape(-1)
            if dd.any():
                dp = Kc.diag_pos()
                for J_ in np.nonzero(dead.any(axis=1))[0]:
                    for j in np.nonzero(dead[J_])[0]:
                        Kc.val[dp[J_], j, j] = 1.0
            Jc = block_spgemm(J, P)
            Ac = block_add(Kc, contact_product(Jc, self.D))
            A, K, J = Ac, Kc, Jc
            R_prev = R
            G_next = coarse_graph(rp, cl, agg, n_agg)
        last = self.levels[-1]
        self.coarse_dense = last.A.todense()
        self.coarse_chol = sla.cho_factor(self.coarse_dense, lower=True)
        self._setup_filter()

    # ---------------------------------------------------------------- new barrier diagonal
    def update_barrier(self, D, E=None):
        """Numeric re-setup for new barrier terms of both kinds: D of the contact rows and
        the diagonal E of bound constraints (Remark 3.1, A = K + J^T D J + E).  The
        aggregates and prolongators are kept; the level-0 stiffness K + diag(E), the
        coarse stiffness chain K_{l+1} = P_l^T K_l P_l (dead coarse DOFs again with a unit
        diagonal) and everything ``update_D`` rebuilds are recomputed."""
        self.K0 = with_bound_diagonal(self.K_in, E)
        self.levels[0].K = self.K0
        for l in range(self.nlev - 1):
            lev, nxt = self.levels[l], self.levels[l + 1]
            Kc = block_spgemm(lev.P.transpose(), block_spgemm(lev.K, lev.P))
            if lev.dead.any():
                dp = Kc.diag_pos()
                for J_ in np.nonzero(lev.dead.any(axis=1))[0]:
                    for j in np.nonzero(lev.dead[J_])[0]:
                        Kc.val[dp[J_], j, j] = 1.0
            nxt.K = Kc
        self.update_D(D)

    def update_D(self, D):
        """Numeric re-setup for a new interior-point step (same K and J, new D).

        The aggregates, prolongators P_l, coarse stiffness K_{l+1} = P_l^T K_l P_l and coarse
        Jacobians J_{l+1} = J_l P_l are kept; the operators A_l = K_l + J_l^T D J_l, their l1
        norms, the smoother weights, the spectral estimates, the coarsest factor and the
        filter factor are recomputed for the new D.  A_{l+1} = P_l^T A_l P_l still holds, so
        B stays a Galerkin V-cycle and M the AMGF operator of Definition 5.3 for the new
        Schur complement."""
        o = self.opts
        self.D = np.asarray(D, np.float64)
        for l, lev in enumerate(self.levels):
            if l == 0:
                lev.A = schur_operator(self.K0, self.J0, self.D)
                self.S = lev.A
            else:
                lev.A = block_add(lev.K, contact_product(lev.J, self.D))
            Acsr = lev.A.csr()
            lev.d = np.asarray(abs(Acsr).sum(axis=1)).ravel()
            th = 1.0 if o.theta is None else np.asarray(o.theta[l], float)
            lev.w = th / lev.d
            if l + 1 < self.nlev:
                dec = lev.decoupled if l == 0 else np.zeros(lev.A.nrows * lev.A.br, bool)
                lev.lam = power_estimate(Acsr, lev.d, dec, o.sa_power_iters, clip=False)
        last = self.levels[-1]
        self.coarse_dense = last.A.todense()
        self.coarse_chol = sla.cho_factor(self.coarse_dense, lower=True)
        self._setup_filter()

    # ---------------------------------------------------------------- level-0 helpers
    def _decoupled_dofs(self, Acsr):
        """DOFs whose row has no nonzero off-diagonal entry (e.g. Dirichlet DOFs)."""
        coo = Acsr.tocoo()
        off = (coo.row != coo.col) & (coo.data != 0.0)
        cnt = np.bincount(coo.row[off], minlength=Acsr.shape[0])
        return cnt == 0

    def _level0_near(self, decoupled):
        X = self.coords
        dec = decoupled.reshape(-1, 3)
        if self.opts.near_null == 3:
            # the three translations: unit displacement in x, y, z at every node
            def translations(J, nodes):
                B = np.zeros((len(nodes), 3, 3))
                B[:, [0, 1, 2], [0, 1, 2]] = 1.0
                B[dec[nodes]] = 0.0
                return B
            return translations

        def near(J, nodes):
            c = np.zeros(3)
            for a in nodes:                     # centroid, ascending node order
                c = c + X[a]
            c = c / len(nodes)
            B = rigid_body_modes(X[nodes] - c)
            B[dec[nodes]] = 0.0
            return B
        return near

    # ---------------------------------------------------------------- filter (Sec. 5.1)
    def _setup_filter(self):
        o = self.opts
        if o.Ic is not None:
            Ic = np.unique(np.asarray(o.Ic, np.int64))
        else:
            nodes = np.unique(self.J0.col)
            Ic = (3 * nodes[:, None] + np.arange(3)[None, :]).ravel()
        self.Ic = Ic
        self.n_c = len(Ic)
        if self.n_c == 0:
            self.Aw = None
            return
        Aw = self.S.csr()[Ic][:, Ic]
        if self.n_c <= o.dense_filter_max:
            self.Aw = Aw.toarray()
            self._aw_chol = sla.cho_factor(self.Aw, lower=True)
            self._aw_solve = lambda r: sla.cho_solve(self._aw_chol, r)
        else:
            self.Aw = Aw.tocsc()
            lu = spla.splu(self.Aw)
            self._aw_solve = lu.solve

    # ---------------------------------------------------------------- apply
    @property
    def n(self):
        return 3 * self.n_nodes

    @property
    def nlev(self):
        return len(self.levels)

    def A_apply(self, x):
        """y = A x for A = K + J^T D J (Sec. 3, the condensed system), evaluated as the
        product the formula writes: K x, plus J^T applied to D times the gaps J x.

        Reading: this is the operator of the CG iteration and of the two residuals inside
        Definition 5.3.  The assembled S (``schur_operator``) rounds every entry
        D_k J_ki J_kj on its own, a perturbation of size u D_max in the contact rows that
        is not confined to the range of J^T; with D up to 1e10 it moves the solution of
        S x = b by about 6e-6 from that of A x = b.  Here each rounding error of the contact
        term stays in the range of J^T (where A is as stiff as D) and the converged CG
        iterate agrees with an extended-precision solve of A x = b to about rtol.  S keeps
        serving what needs the matrix entries: strength, aggregation, l1 norms,
        smoothing, coarse operators and A_w."""
        J = self.J0.csr()
        return self.K0.csr() @ x + J.T @ (self.D * (J @ x))

    def smooth(self, l, b, x):
        """One smoother application on level l for A x = b (O10).

        l1-Jacobi: x + w (b - A x).  Chebyshev: the degree-m Chebyshev iteration on the
        D_l1-preconditioned system over [0.3 lam, lam], lam = min(1, 1.1 * power
        estimate); its error propagation is T_m((theta - D^-1 A)/delta) / T_m(theta/delta)
        with theta, delta the centre and half-width of that interval."""
        lev = self.levels[l]
        A = lev.A.csr()
        if self.opts.smoother == "jacobi":
            return x + lev.w * (b - A @ x)
        lmax = min(1.0, 1.1 * lev.lam)
        lmin = 0.3 * lmax
        theta, delta = 0.5 * (lmax + lmin), 0.5 * (lmax - lmin)
        sigma = theta / delta
        dinv = 1.0 / lev.d
        r = dinv * (b - A @ x)
        rho = 1.0 / sigma
        dk = r / theta
        for k in range(self.opts.cheb_degree):
            x = x + dk
            if k + 1 == self.opts.cheb_degree:
                break
            r = r - dinv * (A @ dk)
            rho_new = 1.0 / (2.0 * sigma - rho)
            dk = rho_new * rho * dk + (2.0 * rho_new / delta) * r
            rho = rho_new
        return x

    def vcycle(self, b, l=0):
        """B b: symmetric V(nu, nu) from a zero initial guess (O11): nu smoother
        applications, coarse correction, nu smoother applications.  With cycle_gamma = g
        the coarse correction visits level l+1 g times, each later visit on the residual
        the earlier ones left (g = 2: the W-cycle); the coarsest solve is exact and is
        visited once."""
        if l == self.nlev - 1:
            return sla.cho_solve(self.coarse_chol, b)
        lev = self.levels[l]
        A = lev.A.csr()
        x = np.zeros_like(b)
        for _ in range(self.opts.sweeps):
            x = self.smooth(l, b, x)
        r = b - A @ x
        rc = lev.P.csr().T @ r
        xc = self.vcycle(rc, l + 1)
        if l + 1 < self.nlev - 1:
            Ac = self.levels[l + 1].A.csr()
            for _ in range(self.opts.cycle_gamma - 1):
                xc = xc + self.vcycle(rc - Ac @ xc, l + 1)
        x = x + lev.P.csr() @ xc
        for _ in range(self.opts.sweeps):
            x = self.smooth(l, b, x)
        return x

    def filter_solve(self, r_c):
        return self._aw_solve(r_c)

    def apply(self, r):
        """z = M r, Definition 5.3 (multiplicative AMGF), or z = B r without filter."""
        z1 = self.vcycle(r)
        if not self.opts.filter:
            return z1
        z2 = z1.copy()
        if self.n_c > 0:
            ra = r - self.A_apply(z1)
            z2[self.Ic] += self.filter_solve(ra[self.Ic])
        r2 = r - self.A_apply(z2)
        return z2 + self.vcycle(r2)

    def pcg(self, b, x0=None, rtol=None, max_iters=None):
        o = self.opts
        return pcg(self.A_apply, self.apply, b, x0,
                   o.rtol if rtol is None else rtol,
                   o.max_iters if max_iters is None else max_iters)

    # ---------------------------------------------------------------- stats
    def level_sizes(self):
        return [lev.A.nrows * lev.A.br for lev in self.levels]

    def operator_complexity(self):
        nz = [lev.A.nnzb * lev.A.br * lev.A.bc for lev in self.levels]
        return sum(nz) / nz[0]


# ======================================================================================
# O14: preconditioned CG (Sec. 4 / Sec. 6.1 stopping rule)
# ======================================================================================
@dataclass
class PCGResult:
    x: np.ndarray
    iterations: int
    converged: bool
    rel_prec_res: float
    history: list = field(default_factory=list)
    status: str = "ok"
    alphas: list = field(default_factory=list)
    betas: list = field(default_factory=list)

    def lanczos_extremes(self):
        """Extreme eigenvalue estimates of M A from the CG coefficients (Lanczos
        tridiagonal: T_kk = 1/a_k + b_{k-1}/a_{k-1}, T_k,k+1 = sqrt(b_k)/a_k)."""
        a = np.asarray(self.alphas)
        bt = np.asarray(self.betas)
        k = len(a)
        T = np.zeros((k, k))
        for i in range(k):
            T[i, i] = 1.0 / a[i] + (bt[i - 1] / a[i - 1] if i > 0 else 0.0)
            if i + 1 < k:
                T[i, i + 1] = T[i + 1, i] = math.sqrt(bt[i]) / a[i]
        ev = np.linalg.eigvalsh(T)
        return ev[0], ev[-1]


def pcg(A_apply, M_apply, b, x0=None, rtol=1e-10, max_iters=5000):
    """CG preconditioned by M; stops when sqrt(r.z / r0.z0) <= rtol.

    beta is the Polak-Ribiere form r_{k+1}.(z_{k+1} - z_k) / (r_k.z_k), equal to the
    classical one in exact arithmetic.  Returns the last iterate on failure.
    """
    b = np.asarray(b, np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, np.float64)
    r = b - A_apply(x) if x0 is not None else b.copy()
    z = M_apply(r)
    rz = float(r @ z)
    rz0 = rz
    hist = [1.0]
    if rz0 == 0.0:
        return PCGResult(x, 0, True, 0.0, hist)
    p = z.copy()
    res = PCGResult(x, 0, False, 1.0, hist)
    for it in range(1, max_iters + 1):
        q = A_apply(p)
        pq = float(p @ q)
        if not pq > 0.0:
            res.x, res.iterations, res.status = x, it - 1, "not_spd"
            return res
        alpha = rz / pq
        res.alphas.append(alpha)
        x = x + alpha * p
        r = r - alpha * q
        z_old = z
        z = M_apply(r)
        rz_new = float(r @ z)
        rel = math.sqrt(abs(rz_new) / rz0)
        hist.append(rel)
        res.betas.append(rz_new / rz)
        if rel <= rtol:
            res.x, res.iterations, res.converged, res.rel_prec_res = x, it, True, rel
            return res
        beta = (rz_new - float(r @ z_old)) / rz
        p = z + beta * p
        rz = rz_new
    res.x, res.iterations, res.rel_prec_res, res.status = x, max_iters, hist[-1], "no_conv"
    return res
