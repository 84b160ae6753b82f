"""FP64 oracle of the learned smoother damping.  TEST INFRASTRUCTURE ONLY.

Not part of the paper: the l1-Jacobi weights of every smoothed level become theta_i / d_i
with theta_i = 1 + 0.98 tanh(MLP(f_i)), a 6 -> 32 (tanh) -> 32 (tanh) -> 1 network on
six standardised row features.  Any theta in (0, 2) keeps the smoother convergent
(2 D_l1 / theta - A is SPD because D_l1 - A is diagonally dominant), so the V-cycle B
stays SPD and convergent (Assumption 1 holds with omega < 2).

Training objective (per system and probe e0): (1/k) log(||E^k e0||_S / ||e0||_S) with
E = I - M S, M the AMGF preconditioner of Definition 5.3 built with the learned B.
The gradient here is reverse mode written out step by step; the pins compare it with
central finite differences of ``loss``.
"""
from __future__ import annotations

import math
import numpy as np

from .amgf_oracle import OracleAMGF

NPARAM = 1313
NTOTAL = 1325


def unpack(W):
    W = np.asarray(W, np.float64)
    return dict(W1=W[0:192].reshape(32, 6), b1=W[192:224], W2=W[224:1248].reshape(32, 32),
                b2=W[1248:1280], W3=W[1280:1312], b3=W[1312], mu=W[1313:1319],
                sd=W[1319:1325])


def level_features(o: OracleAMGF):
    """Per smoothed level, the (6, n_l) features of its scalar rows:
    log10 a_ii, log10 d_i, a_ii/d_i, log10(1 + sum_k D_k J_ki^2), contact flag (node has
    a contact term), level/(levels - 1)."""
    L = o.nlev
    out = []
    for l in range(L - 1):
        lev = o.levels[l]
        A = lev.A
        b = A.br
        diag = A.val[A.diag_pos()]                      # (nn, b, b)
        aii = np.einsum("npp->np", diag).reshape(-1)
        Jc = lev.J.csr()
        beta = np.asarray(Jc.multiply(Jc).T @ o.D).ravel()
        node_contact = np.zeros(A.nrows)
        node_contact[np.unique(lev.J.col)] = 1.0
        frac = l / (L - 1) if L > 1 else 0.0
        F = np.stack([np.log10(aii), np.log10(lev.d), aii / lev.d, np.log10(1.0 + beta),
                      np.repeat(node_contact, b), np.full(A.nrows * b, frac)])
        out.append(F)
    return out


def mlp_forward(W, F):
    """theta and the intermediates of the 6-32-32-1 MLP for feature matrix F (6, n)."""
    p = unpack(W)
    fh = (F - p["mu"][:, None]) / p["sd"][:, None]
    h1 = np.tanh(p["W1"] @ fh + p["b1"][:, None])
    h2 = np.tanh(p["W2"] @ h1 + p["b2"][:, None])
    y = p["W3"] @ h2 + p["b3"]
    theta = 1.0 + 0.98 * np.tanh(y)
    return theta, (fh, h1, h2, y)


def mlp_backward(W, F, thbar):
    """d loss / d (W1 b1 W2 b2 W3 b3) given d loss / d theta."""
    p = unpack(W)
    fh, h1, h2, y = mlp_forward(W, F)[1]
    ybar = thbar * 0.98 * (1.0 - np.tanh(y) ** 2)
    g = np.zeros(NPARAM)
    g[1280:1312] = h2 @ ybar
    g[1312] = ybar.sum()
    a2 = (p["W3"][:, None] * ybar[None, :]) * (1.0 - h2 ** 2)
    g[224:1248] = (a2 @ h1.T).ravel()
    g[1248:1280] = a2.sum(axis=1)
    a1 = (p["W2"].T @ a2) * (1.0 - h1 ** 2)
    g[0:192] = (a1 @ fh.T).ravel()
    g[192:224] = a1.sum(axis=1)
    return g


def set_damping(o: OracleAMGF, W, feats=None):
    """Install theta/d as the smoother weights of every smoothed level."""
    feats = level_features(o) if feats is None else feats
    for l, F in enumerate(feats):
        theta, _ = mlp_forward(W, F)
        o.levels[l].w = theta / o.levels[l].d
    return feats


def reset_damping(o: OracleAMGF):
    for l in range(o.nlev - 1):
        o.levels[l].w = 1.0 / o.levels[l].d


# ----------------------------------------------------------------- taped forward / adjoint
def _vcycle_tape(o, b, l, tape):
    tape.setdefault(l, {})["b"] = b.copy()
    if l == o.nlev - 1:
        import scipy.linalg as sla
        return sla.cho_solve(o.coarse_chol, b)
    lev = o.levels[l]
    A = lev.A.csr()
    P = lev.P.csr()
    x = lev.w * b
    r = b - A @ x
    xc = _vcycle_tape(o, P.T @ r, l + 1, tape)
    x = x + P @ xc
    s2 = b - A @ x
    tape[l]["s2"] = s2
    return x + lev.w * s2


def _vcycle_adj(o, ybar, l, tape, wbar):
    if l == o.nlev - 1:
        import scipy.linalg as sla
        return sla.cho_solve(o.coarse_chol, ybar)
    lev = o.levels[l]
    A = lev.A.csr()
    P = lev.P.csr()
    s2bar = lev.w * ybar
    wbar[l] += ybar * tape[l]["s2"]
    xpbar = ybar - A @ s2bar
    bcbar = _vcycle_adj(o, P.T @ xpbar, l + 1, tape, wbar)
    rbar = P @ bcbar
    xbar = xpbar - A @ rbar
    wbar[l] += xbar * tape[l]["b"]
    return s2bar + rbar + lev.w * xbar


def _apply_tape(o, v):
    t1, t2 = {}, {}
    z1 = _vcycle_tape(o, v, 0, t1)
    z2 = z1.copy()
    if o.n_c > 0:
        ra = v - o.A_apply(z1)
        z2[o.Ic] += o.filter_solve(ra[o.Ic])
    r2 = v - o.A_apply(z2)
    return z2 + _vcycle_tape(o, r2, 0, t2), (t1, t2)


def _apply_adj(o, zbar, tapes, wbar):
    t1, t2 = tapes
    r2bar = _vcycle_adj(o, zbar, 0, t2, wbar)
    vbar = r2bar.copy()
    z2bar = zbar - o.A_apply(r2bar)
    z1bar = z2bar.copy()
    if o.n_c > 0:
        u = np.zeros(o.n)
        u[o.Ic] = o.filter_solve(z2bar[o.Ic])
        vbar += u
        z1bar = z2bar - o.A_apply(u)
    return vbar + _vcycle_adj(o, z1bar, 0, t1, wbar)


def loss(o: OracleAMGF, W, probes, k=2, feats=None):
    """Mean over the probe columns of (1/k) log(||E^k e0||_S / ||e0||_S)."""
    set_damping(o, W, feats)
    tot = 0.0
    for q in range(probes.shape[1]):
        e = probes[:, q].copy()
        s0 = e @ o.A_apply(e)
        for _ in range(k):
            e = e - o.apply(o.A_apply(e))
        tot += (math.log(e @ o.A_apply(e)) - math.log(s0)) / (2 * k)
    return tot / probes.shape[1]


def loss_grad(o: OracleAMGF, W, probes, k=2, feats=None):
    """(loss, d loss / d W[:1313]) by reverse mode through M (both V-cycles, filter)."""
    feats = set_damping(o, W, feats)
    wbar = {l: np.zeros(o.levels[l].A.nrows * o.levels[l].A.br) for l in range(o.nlev - 1)}
    tot = 0.0
    npb = probes.shape[1]
    for q in range(npb):
        e = probes[:, q].copy()
        s0 = e @ o.A_apply(e)
        tapes = []
        for _ in range(k):
            z, tp = _apply_tape(o, o.A_apply(e))
            tapes.append(tp)
            e = e - z
        Se = o.A_apply(e)
        sk = e @ Se
        tot += (math.log(sk) - math.log(s0)) / (2 * k)
        ebar = Se / (k * sk)
        for j in range(k - 1, -1, -1):
            vbar = _apply_adj(o, -ebar, tapes[j], wbar)
            ebar = ebar + o.A_apply(vbar)
    g = np.zeros(NPARAM)
    for l, F in enumerate(feats):
        thbar = wbar[l] / o.levels[l].d / npb
        g += mlp_backward(W, F, thbar)
    return tot / npb, g


# the MLP damping is kept unless theta = 1 leaves a one-step error smaller by more than this
JUDGE_MARGIN = 1.25


def judge_keeps_mlp(ratio_mlp, ratio_plain):
    return ratio_mlp <= JUDGE_MARGIN * ratio_plain


def judge(o: OracleAMGF, W, feats=None):
    """The judge of the learned damping: energy-norm error after one AMGF step
    e1 = (I - M A) e0 from the power-iteration start e0 (zero on the decoupled level-0
    DOFs), with the MLP damping and with theta = 1.  Returns (ratio_mlp, ratio_plain),
    each ||e1||_A / ||e0||_A; ``judge_keeps_mlp`` decides.  Leaves the oracle with
    theta = 1."""
    from .amgf_oracle import power_start
    e0 = power_start(o.n)
    dec = getattr(o.levels[0], "decoupled", None)
    if dec is not None:
        e0[dec] = 0.0
    n0 = float(e0 @ o.A_apply(e0))

    def ratio():
        e1 = e0 - o.apply(o.A_apply(e0))
        return math.sqrt(abs(float(e1 @ o.A_apply(e1))) / n0)

    set_damping(o, W, feats)
    r_mlp = ratio()
    reset_damping(o)
    return r_mlp, ratio()
