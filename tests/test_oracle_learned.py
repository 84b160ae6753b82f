"""Pins of the oracle's learned-smoother loss and gradient."""
import numpy as np
import pytest

from amgf_inputs import learning
from oracle import learned
from oracle_util import build, dense_of, small_problem


@pytest.fixture(scope="module")
def setup():
    p = small_problem(N=3, D_log10=(0.0, 3.0))
    o = build(p, coarse_max_nodes=8, max_levels=3)
    feats = learned.level_features(o)
    mu = np.concatenate(feats, axis=1).mean(axis=1)
    sd = np.concatenate(feats, axis=1).std(axis=1) + 1e-3
    W = learning.init_params(seed=3, mu=mu, sd=sd, last_scale=0.3)
    P = learning.probes(o.n, p.free, 2, seed=5)
    return p, o, feats, W, P


def test_zero_last_layer_is_plain_l1_jacobi(setup):
    p, o, feats, W, P = setup
    W0 = W.copy()
    W0[1280:1313] = 0.0
    learned.set_damping(o, W0, feats)
    r = np.random.default_rng(0).standard_normal(o.n)
    z_l = o.apply(r)
    learned.reset_damping(o)
    assert np.array_equal(z_l, o.apply(r))


def test_theta_range_keeps_B_spd_and_convergent(setup):
    p, o, feats, W, P = setup
    Wb = W.copy()
    Wb[1280:1312] *= 40.0                  # drive theta towards its bounds
    learned.set_damping(o, Wb, feats)
    th = np.concatenate([learned.mlp_forward(Wb, F)[0] for F in feats])
    assert th.min() > 0.02 and th.max() < 1.98 and (th.max() - th.min()) > 1.0
    A = o.S.todense()
    B = dense_of(o.vcycle, o.n)
    lam = np.linalg.eigvals(B @ A).real
    assert np.abs(B - B.T).max() <= 1e-9 * np.abs(B).max()
    assert lam.min() > 0 and lam.max() < 2.0
    learned.reset_damping(o)


def test_gradient_matches_central_differences(setup):
    p, o, feats, W, P = setup
    L0, g = learned.loss_grad(o, W, P, k=2, feats=feats)
    assert abs(L0 - learned.loss(o, W, P, k=2, feats=feats)) <= 1e-12 * abs(L0)
    rng = np.random.default_rng(7)
    idx = np.concatenate([rng.choice(192, 6, replace=False), 192 + rng.choice(32, 3),
                          224 + rng.choice(1024, 8, replace=False), 1248 + rng.choice(32, 3),
                          1280 + rng.choice(32, 5, replace=False), [1312]])
    h = 1e-3
    for i in idx:
        Wp = W.astype(np.float64).copy()
        Wm = Wp.copy()
        Wp[i] += h
        Wm[i] -= h
        fd = (learned.loss(o, Wp, P, 2, feats) - learned.loss(o, Wm, P, 2, feats)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1e-4, abs(g).max()) + 1e-5 * abs(g[i]), (i, fd, g[i])
    # a random direction through all parameters
    v = rng.standard_normal(1313)
    h = 1e-5
    Wp = W.astype(np.float64).copy()
    Wm = Wp.copy()
    Wp[:1313] += h * v
    Wm[:1313] -= h * v
    fd = (learned.loss(o, Wp, P, 2, feats) - learned.loss(o, Wm, P, 2, feats)) / (2 * h)
    assert abs(fd - g @ v) <= 1e-5 * abs(fd)
    learned.reset_damping(o)


def test_loss_is_error_reduction(setup):
    """theta = 1: the loss equals the measured log energy-norm reduction of E = I - MS."""
    p, o, feats, W, P = setup
    W0 = W.copy()
    W0[1280:1313] = 0.0
    L = learned.loss(o, W0, P, k=2, feats=feats)
    A = o.S.todense()
    M = dense_of(o.apply, o.n)
    E = np.eye(o.n) - M @ A
    vals = []
    for q in range(P.shape[1]):
        e = P[:, q]
        ek = E @ (E @ e)
        vals.append(np.log((ek @ A @ ek) / (e @ A @ e)) / (2 * 2))   # (1/k) log of the norm ratio
    assert abs(L - np.mean(vals)) <= 1e-10 * abs(L)
    assert L < 0
    learned.reset_damping(o)


def test_features_match_explicit_loops_over_dense_operators():
    """Each of the six features, recomputed with plain loops over the dense level operator
    A_l, the dense coarse Jacobian J_l and D (a Sigma D J instead of Sigma D J^2, a swapped
    feature or a wrong level fraction fails here)."""
    import math
    p = small_problem(N=2, D_log10=(0.0, 4.0), seed=17)
    o = build(p, coarse_max_nodes=2, max_levels=3)
    L = o.nlev
    assert L == 3
    feats = learned.level_features(o)
    assert len(feats) == L - 1
    Ic = set(int(i) for i in o.Ic)
    for l, F in enumerate(feats):
        lev = o.levels[l]
        A = lev.A.todense()
        J = lev.J.todense()
        b = lev.A.br
        n_l = A.shape[0]
        assert F.shape == (6, n_l) and J.shape == (p.m, n_l)
        for i in range(n_l):
            aii = A[i, i]
            d = 0.0
            for j in range(n_l):
                d += abs(A[i, j])
            beta = 0.0
            for k in range(p.m):
                beta += p.D[k] * J[k, i] * J[k, i]
            node = i // b
            touched = any(J[k, node * b + c] != 0.0 for k in range(p.m) for c in range(b))
            want = [math.log10(aii), math.log10(d), aii / d, math.log10(1.0 + beta),
                    1.0 if touched else 0.0, l / (L - 1)]
            for f in range(6):
                assert abs(F[f, i] - want[f]) <= 1e-12 * max(1.0, abs(want[f])), (l, i, f)
            if l == 0:
                # at level 0 the contact flag is exactly membership of the filter space
                assert F[4, i] == (1.0 if i in Ic else 0.0)
        assert F[4].sum() > 0 and (l > 0 or F[4].sum() < n_l)


def test_mlp_forward_matches_rowwise_evaluation_of_the_header_layout():
    """theta row by row from the flat parameter layout W1[32][6] b1[32] W2[32][32] b2[32]
    W3[32] b3 mu[6] sigma[6] (a transposed W1 or W2 or a swapped bias block fails)."""
    import math
    rng = np.random.default_rng(23)
    W = rng.uniform(-0.8, 0.8, 1325)
    W[1313:1319] = rng.uniform(-1, 1, 6)
    W[1319:1325] = rng.uniform(0.5, 2.0, 6)
    F = rng.standard_normal((6, 9)) * 2.0
    theta, _ = learned.mlp_forward(W, F)
    for i in range(F.shape[1]):
        fh = [(F[j, i] - W[1313 + j]) / W[1319 + j] for j in range(6)]
        h1 = []
        for a in range(32):
            s = W[192 + a]
            for j in range(6):
                s += W[a * 6 + j] * fh[j]
            h1.append(math.tanh(s))
        h2 = []
        for c in range(32):
            s = W[1248 + c]
            for a in range(32):
                s += W[224 + c * 32 + a] * h1[a]
            h2.append(math.tanh(s))
        y = W[1312]
        for c in range(32):
            y += W[1280 + c] * h2[c]
        want = 1.0 + 0.98 * math.tanh(y)
        assert abs(theta[i] - want) <= 1e-13, (i, theta[i], want)
    assert np.all((theta > 0.02) & (theta < 1.98))


def test_judge_is_the_one_step_energy_norm_reduction(setup):
    """learned.judge against the dense error propagation I - M A (A = K + J^T D J written
    out densely), for the MLP damping and for theta = 1."""
    from oracle.amgf_oracle import power_start
    from oracle_util import J_dense, K_dense
    p, o, feats, W, P = setup
    Jd = J_dense(p)
    A = K_dense(p) + Jd.T @ (p.D[:, None] * Jd)
    e0 = power_start(o.n)
    e0[o.levels[0].decoupled] = 0.0
    want = []
    for Wx in (W, None):
        if Wx is None:
            learned.reset_damping(o)
        else:
            learned.set_damping(o, Wx, feats)
        M = dense_of(o.apply, o.n)
        e1 = e0 - M @ (A @ e0)
        want.append(np.sqrt((e1 @ A @ e1) / (e0 @ A @ e0)))
    got = learned.judge(o, W, feats)
    assert abs(got[0] - want[0]) <= 1e-9 * want[0] and abs(got[1] - want[1]) <= 1e-9 * want[1]
    assert np.all(o.levels[0].w == 1.0 / o.levels[0].d)      # left at theta = 1


def test_judge_choice_agrees_with_cg_on_c1():
    """The trained network against theta = 1 on C1 with and without the barrier terms of
    bound constraints: the judge prefers whichever damping CG converges faster with."""
    import os
    from amgf_inputs import bound_barrier, make_config
    from oracle import OracleAMGF
    from paper_2505_18576_amd.train_smoother import load_weights
    W = load_weights(os.path.join(os.path.dirname(os.path.dirname(__file__)),
                                  "paper_2505_18576_amd", "weights", "smoother_ip.bin"))
    W = W.astype(np.float64)
    for bounds in (False, True):
        p = make_config("C1")
        E = bound_barrier(p, seed=9) if bounds else None
        o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col,
                       p.J_val, p.D, p.coords, E=E)
        r_mlp, r_plain = learned.judge(o, W)
        its_plain = o.pcg(p.b).iterations
        learned.set_damping(o, W)
        its_mlp = o.pcg(p.b).iterations
        assert learned.judge_keeps_mlp(r_mlp, r_plain) == (its_mlp < its_plain), \
            (bounds, r_mlp, r_plain)
