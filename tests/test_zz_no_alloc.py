"""amgf_pcg_noalloc (the CG entry point that allocates nothing) against amgf_pcg: two
calls in a row on one GPU, the second on a smaller problem, each bitwise equal to the
allocating entry point on the same handle, with no device allocation made."""
import numpy as np
import pytest

from gpu_util import problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", [0, 1])
def test_pcg_noalloc_matches_pcg(precision):
    import torch
    from paper_2505_18576_amd import AMGF
    from paper_2505_18576_amd import amgf as b
    handles = []
    for name in ("C2", "C1"):                       # the second call is the smaller input
        p = problem(name)
        print(f"[gpu setup] {name} precision {precision}", flush=True)
        h = AMGF.from_problem(p, precision=precision, allocator="torch")
        handles.append(h)
        bd = torch.from_numpy(p.b).cuda()
        x_ref, info_ref = h.pcg(bd)
        x = torch.zeros_like(bd)
        torch.cuda.synchronize()
        n_alloc, live = h.allocator.n_alloc, h.allocator.live
        print(f"[gpu pcg_noalloc] {name}", flush=True)
        st, info = h.pcg_noalloc(bd, x)
        torch.cuda.synchronize()
        print(f"{name} precision {precision}: pcg {info_ref.iterations} it, noalloc "
              f"{info.iterations} it, rel prec res {info.rel_prec_res:.3e} / "
              f"{info_ref.rel_prec_res:.3e}, ms {info.ms_solve:.2f} / {info_ref.ms_solve:.2f}")
        assert st == b.AMGF_OK and info.converged
        assert h.allocator.n_alloc == n_alloc and h.allocator.live == live
        assert info.iterations == info_ref.iterations
        assert info.rel_prec_res == info_ref.rel_prec_res
        assert info.rel_true_res == info_ref.rel_true_res
        assert np.array_equal(x.cpu().numpy().view(np.uint64),
                              x_ref.cpu().numpy().view(np.uint64))
        assert info.ms_amg_apply == 0.0 and info.ms_filter_apply == 0.0
    for h in handles:
        h.close()
