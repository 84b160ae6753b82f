"""GPU learned-smoother kernels against the oracle: features, damping, loss, gradient."""
import numpy as np
import pytest

from amgf_inputs import learning, make_two_block
from gpu_util import rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    from oracle import OracleAMGF, OracleOptions, learned
    p = make_two_block(4, D_log10=(0.0, 3.0), D_seed=31, rhs_seed=32)
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords, OracleOptions(coarse_max_nodes=16))
    feats = learned.level_features(o)
    allf = np.concatenate(feats, axis=1)
    W = learning.init_params(seed=11, mu=allf.mean(axis=1), sd=allf.std(axis=1) + 1e-3,
                             last_scale=0.3)
    P = learning.probes(o.n, p.free, 3, seed=12)
    return p, o, feats, W, P


def test_features_match_oracle(case):
    from paper_2505_18576_amd import AMGF
    p, o, feats, W, P = case
    h = AMGF.from_problem(p, coarse_max_nodes=16)
    assert h.n_levels == o.nlev
    for l, F in enumerate(feats):
        G = h.features(l)
        assert rel(G, F) < 1e-13, l
    h.close()


def test_loss_and_gradient_match_oracle(case):
    from oracle import learned
    from paper_2505_18576_amd import AMGF
    p, o, feats, W, P = case
    L_o, g_o = learned.loss_grad(o, W, P, k=2, feats=feats)
    learned.reset_damping(o)
    h = AMGF.from_problem(p, coarse_max_nodes=16)
    L_g, g_g = h.loss_grad(W, P, k=2)
    g_g = g_g.cpu().numpy()
    print(f"loss gpu {L_g:.12f} oracle {L_o:.12f}; grad rel {rel(g_g, g_o):.2e}")
    assert abs(L_g - L_o) <= 1e-10 * abs(L_o)
    assert rel(g_g, g_o) < 1e-9
    # the handle keeps theta = 1 after the gradient call
    assert np.all(h.theta(0) == 1.0)
    h.close()


def test_learned_damping_applies_the_mlp(case):
    from oracle import learned
    from paper_2505_18576_amd import AMGF
    p, o, feats, W, P = case
    h = AMGF.from_problem(p, coarse_max_nodes=16, mlp_weights=W, learned_judge=0)
    learned.set_damping(o, W, feats)
    for l, F in enumerate(feats):
        assert rel(h.theta(l), learned.mlp_forward(W, F)[0]) < 1e-13
    r = np.random.default_rng(4).standard_normal(o.n)
    assert rel(h.apply(r).cpu().numpy(), o.apply(r)) < 1e-11
    x, info = h.pcg(p.b)
    ref = o.pcg(p.b)
    learned.reset_damping(o)
    assert info.converged and abs(info.iterations - ref.iterations) <= 1
    assert info.used_fallback == 0
    h.close()


def test_zero_last_layer_is_bitwise_plain(case):
    from paper_2505_18576_amd import AMGF
    p, o, feats, W, P = case
    W0 = W.copy()
    W0[1280:1313] = 0.0
    a = AMGF.from_problem(p, coarse_max_nodes=16, mlp_weights=W0)
    b = AMGF.from_problem(p, coarse_max_nodes=16)
    xa, ia = a.pcg(p.b)
    xb, ib = b.pcg(p.b)
    assert ia.iterations == ib.iterations
    assert np.array_equal(xa.cpu().numpy().view(np.uint64), xb.cpu().numpy().view(np.uint64))
    a.close()
    b.close()


def test_fallback_when_learned_damping_fails(case):
    """NaN weights make the learned V-cycle non-finite.  Without the judge, CG breaks down,
    the solve reruns with theta = 1 from the same initial guess and reports fallback 1; with
    the judge (default) the non-finite error reduction loses against theta = 1 at setup and
    the solve runs plain from the start (fallback 2).  Both equal the plain solve bitwise."""
    from paper_2505_18576_amd import AMGF
    p, o, feats, W, P = case
    Wbad = W.copy()
    Wbad[1312] = np.nan
    ref = AMGF.from_problem(p, coarse_max_nodes=16)
    xr, iref = ref.pcg(p.b)
    for judge, code in ((0, 1), (1, 2)):
        h = AMGF.from_problem(p, coarse_max_nodes=16, mlp_weights=Wbad, learned_judge=judge)
        x, info = h.pcg(p.b)
        assert info.used_fallback == code and info.converged
        assert info.iterations == iref.iterations
        assert np.array_equal(x.cpu().numpy(), xr.cpu().numpy())
        h.close()
    ref.close()


@pytest.mark.parametrize("bounds", [False, True])
def test_judge_matches_oracle_and_keeps_the_better_damping(bounds):
    """The judge's one-step error reductions against the oracle's; on C1 the trained damping
    wins, with the bound-constraint barrier terms (which the network never saw) theta = 1
    wins and the solve is bitwise the plain one.  In both cases the choice agrees with the
    CG iteration counts."""
    import os
    from amgf_inputs import bound_barrier, make_config
    from oracle import OracleAMGF, learned
    from paper_2505_18576_amd import AMGF
    from paper_2505_18576_amd.train_smoother import load_weights
    W = load_weights(os.path.join(os.path.dirname(os.path.dirname(__file__)),
                                  "paper_2505_18576_amd", "weights", "smoother_ip.bin"))
    p = make_config("C1")
    E = bound_barrier(p, seed=9) if bounds else None
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords, E=E)
    r_mlp, r_plain = learned.judge(o, W.astype(np.float64))
    plain = AMGF.from_problem(p, E=E)
    h = AMGF.from_problem(p, E=E, mlp_weights=W)
    xp, ip = plain.pcg(p.b)
    x, info = h.pcg(p.b)
    hf = AMGF.from_problem(p, E=E, mlp_weights=W, learned_judge=0)
    _, il = hf.pcg(p.b)
    print(f"bounds {bounds}: judge gpu {info.judge_learned:.6e} / {info.judge_plain:.6e}, "
          f"oracle {r_mlp:.6e} / {r_plain:.6e}; its plain {ip.iterations}, learned "
          f"{il.iterations}, judged {info.iterations} (fallback {info.used_fallback})")
    assert abs(info.judge_learned - r_mlp) <= 1e-6 * r_mlp
    assert abs(info.judge_plain - r_plain) <= 1e-6 * r_plain
    if bounds:
        assert not learned.judge_keeps_mlp(r_mlp, r_plain) and info.used_fallback == 2
        assert il.iterations > ip.iterations and info.iterations == ip.iterations
        assert np.array_equal(x.cpu().numpy(), xp.cpu().numpy())
    else:
        assert learned.judge_keeps_mlp(r_mlp, r_plain) and info.used_fallback == 0
        assert il.iterations < ip.iterations and info.iterations == il.iterations
    for a in (plain, h, hf):
        a.close()


def test_adam_step_matches_reference():
    import torch
    from paper_2505_18576_amd.amgf import adam_step
    rng = np.random.default_rng(0)
    W = rng.standard_normal(1325).astype(np.float32)
    g = rng.standard_normal(1313)
    Wd = torch.from_numpy(W.copy()).cuda()
    gd = torch.from_numpy(g).cuda()
    m1 = torch.zeros(1313, dtype=torch.float32, device="cuda")
    m2 = torch.zeros_like(m1)
    adam_step(Wd, gd, m1, m2, 1, 1e-3)
    torch.cuda.synchronize()
    # t = 1: m_hat = g, v_hat = g^2, step = lr * g / (|g| + eps)
    ref = W.copy()
    ref[:1313] -= (1e-3 * g / (np.abs(g) + 1e-8)).astype(np.float32)
    assert np.allclose(Wd.cpu().numpy(), ref, rtol=1e-5, atol=1e-6)


def test_trained_network_reduces_iterations_on_held_out_systems():
    """The committed parameters (trained on interior-point steps 1-10) against plain
    l1-Jacobi AMGF on held-out steps 13 and 19: fewer CG iterations, same solution."""
    import os
    from amgf_inputs import make_config
    from paper_2505_18576_amd import AMGF
    from paper_2505_18576_amd.train_smoother import load_weights
    W = load_weights(os.path.join(os.path.dirname(os.path.dirname(__file__)),
                                  "paper_2505_18576_amd", "weights", "smoother_ip.bin"))
    for t in (13, 19):
        p = make_config("C4", ip_step=t)
        a = AMGF.from_problem(p)
        b = AMGF.from_problem(p, mlp_weights=W)
        xa, ia = a.pcg(p.b)
        xb, ib = b.pcg(p.b)
        print(f"t={t}: plain {ia.iterations}, learned {ib.iterations}")
        assert ia.converged and ib.converged and ib.used_fallback == 0
        assert ib.iterations <= 0.9 * ia.iterations
        assert rel(xb.cpu().numpy(), xa.cpu().numpy()) < 1e-7
        a.close()
        b.close()


@pytest.mark.parametrize("t", [1, 10])
def test_gradient_matches_oracle_at_training_size(t):
    """Loss and gradient on the training systems themselves (interior-point steps t of the
    N = 32 two-block problem, 215,622 DOFs, three levels; D up to 1e1 at t = 1 and 5e5 at
    t = 10), at the committed parameters, against the oracle's reverse mode.  Training runs
    on FP64 handles only: a mixed-precision handle refuses the call."""
    import os
    from amgf_inputs import make_config
    from oracle import OracleAMGF, learned
    from paper_2505_18576_amd import AMGF
    from paper_2505_18576_amd.amgf import AMGFError
    from paper_2505_18576_amd.train_smoother import load_weights
    W = load_weights(os.path.join(os.path.dirname(os.path.dirname(__file__)),
                                  "paper_2505_18576_amd", "weights", "smoother_ip.bin"))
    p = make_config("C4", ip_step=t, N=32)
    print(f"[oracle] C4 t={t} N=32 setup", flush=True)
    o = OracleAMGF(p.n_nodes, p.K_rowptr, p.K_col, p.K_val, p.J_rowptr, p.J_col, p.J_val,
                   p.D, p.coords)
    P = learning.probes(o.n, p.free, 2, seed=1000 + t)
    L_o, g_o = learned.loss_grad(o, W, P, k=2)
    print(f"[gpu setup] C4 t={t} N=32", flush=True)
    h = AMGF.from_problem(p)
    assert h.n_levels == o.nlev
    L_g, g_g = h.loss_grad(W, P, k=2)
    g_g = g_g.cpu().numpy()
    print(f"t={t}: levels {o.nlev}, loss gpu {L_g:.12f} oracle {L_o:.12f}, "
          f"grad rel {rel(g_g, g_o):.2e}")
    assert abs(L_g - L_o) <= 1e-10 * abs(L_o)
    assert rel(g_g, g_o) < 1e-9
    h.close()
    hm = AMGF.from_problem(p, precision=1)
    with pytest.raises(AMGFError):
        hm.loss_grad(W, P, k=2)
    hm.close()
