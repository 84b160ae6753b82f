"""Train the learned smoother damping on the GPU.

Training systems: steps 1..10 of the synthetic interior-point sequence on the 32^3-per-
block two-body mesh (barrier mu = 0.1 * 0.3^(t-1), D = z/s); evaluation: steps 11..20,
PCG iterations with the learned damping against plain l1-Jacobi AMGF.  The loss and its
gradient come from the library's own forward/adjoint kernels (amgf_mlp_loss_grad), the
update from amgf_adam_step.  Writes the parameters (and a JSON log next to them).

    python -m paper_2505_18576_amd.train_smoother --out weights/smoother_ip.bin
"""
import argparse
import json
import os
import struct
import sys
import time

import numpy as np

MAGIC = b"AMGFMLP1"


def save_weights(path, W, meta=None):
    W = np.ascontiguousarray(W, dtype="<f4")
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<ii", 1, W.size))
        f.write(W.tobytes())
    if meta is not None:
        with open(os.path.splitext(path)[0] + ".json", "w") as f:
            json.dump(meta, f, indent=1)


def load_weights(path):
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not an AMGF MLP parameter file")
        ver, n = struct.unpack("<ii", f.read(8))
        if ver != 1 or n != 1325:
            raise ValueError(f"{path}: unsupported version {ver} / size {n}")
        return np.frombuffer(f.read(4 * n), dtype="<f4").copy()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", default="1-10")
    ap.add_argument("--eval", default="11-20")
    ap.add_argument("--N", type=int, default=32)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--probes", type=int, default=4)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(__file__), "weights",
                                                  "smoother_ip.bin"))
    a = ap.parse_args(argv)
    import torch
    ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, ROOT)
    from amgf_inputs import learning, make_config
    from paper_2505_18576_amd import AMGF
    from paper_2505_18576_amd.amgf import adam_step

    def rng_of(s):
        lo, hi = (int(v) for v in s.split("-"))
        return list(range(lo, hi + 1))

    t0 = time.perf_counter()
    train = []
    for t in rng_of(a.train):
        p = make_config("C4", ip_step=t, N=a.N)
        h = AMGF.from_problem(p)
        P = learning.probes(p.n, p.free, a.probes, seed=1000 + t)
        train.append((t, p, h, torch.from_numpy(P.T.copy()).cuda().T))
        print(f"[train] system t={t}: n={p.n}, levels {h.n_levels}", flush=True)
    feats = np.concatenate([h.features(l) for _, _, h, _ in train
                            for l in range(h.n_levels - 1)], axis=1)
    mu, sd = feats.mean(axis=1), feats.std(axis=1) + 1e-3
    W = torch.from_numpy(learning.init_params(a.seed, mu, sd)).cuda()
    m1 = torch.zeros(1313, dtype=torch.float32, device="cuda")
    m2 = torch.zeros_like(m1)
    hist = []
    for step in range(1, a.steps + 1):
        tot, g = 0.0, torch.zeros(1313, dtype=torch.float64, device="cuda")
        for t, p, h, P in train:
            l, gi = h.loss_grad(W, P, k=a.k)
            tot += l
            g += gi
        g /= len(train)
        tot /= len(train)
        hist.append(tot)
        adam_step(W, g, m1, m2, step, a.lr)
        if step == 1 or step % 10 == 0:
            print(f"[train] step {step}: loss {tot:.6f} |g| {float(g.norm()):.3e} "
                  f"({time.perf_counter() - t0:.1f}s)", flush=True)
    torch.cuda.synchronize()
    Wn = W.cpu().numpy()
    for _, _, h, _ in train:
        h.close()
    evals = []
    for t in rng_of(a.eval):
        p = make_config("C4", ip_step=t, N=a.N)
        row = {"t": t}
        for name, kw in (("plain", {}), ("learned", {"mlp_weights": Wn})):
            for prec in (0, 1):
                h = AMGF.from_problem(p, precision=prec, **kw)
                x, info = h.pcg(p.b)
                row[f"{name}_{'fp64' if prec == 0 else 'mixed'}"] = dict(
                    iterations=int(info.iterations), converged=bool(info.converged),
                    fallback=int(info.used_fallback), ms_solve=float(info.ms_solve))
                h.close()
        evals.append(row)
        print(f"[eval] t={t}: plain {row['plain_fp64']['iterations']} / "
              f"learned {row['learned_fp64']['iterations']} iterations (fp64), "
              f"mixed {row['plain_mixed']['iterations']} / {row['learned_mixed']['iterations']}",
              flush=True)
    meta = dict(train=a.train, eval=a.eval, N=a.N, steps=a.steps, lr=a.lr, probes=a.probes,
                k=a.k, seed=a.seed, loss_history=hist, feature_mean=mu.tolist(),
                feature_std=sd.tolist(), evaluation=evals,
                seconds=time.perf_counter() - t0)
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    save_weights(a.out, Wn, meta)
    print(f"[train] wrote {a.out}", flush=True)


if __name__ == "__main__":
    main()
