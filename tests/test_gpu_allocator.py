"""Caller-supplied device memory (amgf_options.allocator) through PyTorch's caching
allocator: the same results as hipMalloc'd handles, every block returned, and an allocator
failure reported as ENOMEM with the partial hierarchy released."""
import numpy as np
import pytest

from gpu_util import gpu, problem

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kw", [{}, dict(precision=1), dict(smoother=1, sweeps=2)])
def test_torch_allocator_matches_hipmalloc(kw):
    import torch
    from paper_2505_18576_amd import amgf as b
    p = problem("C1")
    ref = gpu("C1", **kw)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    A = b.TorchAllocator()
    h = b.AMGF.from_problem(p, allocator=A, **kw)
    held = torch.cuda.memory_allocated() - base
    print(f"{kw}: {A.live} blocks, {held / 2**20:.1f} MiB held by the handle", flush=True)
    assert A.live > 0 and held > 0
    r = np.random.default_rng(5).standard_normal(h.n)
    for f in ("vcycle", "apply"):
        assert np.array_equal(getattr(h, f)(r).cpu().numpy(), getattr(ref, f)(r).cpu().numpy())
    x, info = h.pcg(p.b)
    xr, infor = ref.pcg(p.b)
    assert info.converged and info.iterations == infor.iterations
    assert np.array_equal(x.cpu().numpy(), xr.cpu().numpy())
    D2 = 10.0 ** np.random.default_rng(6).uniform(0.0, 6.0, p.m)
    h.update_D(D2)
    ref.update_D(D2)
    assert np.array_equal(h.apply(r).cpu().numpy(), ref.apply(r).cpu().numpy())
    h.close()
    ref.close()
    torch.cuda.synchronize()
    assert A.live == 0
    assert torch.cuda.memory_allocated() - base < held


@pytest.mark.parametrize("fail_after", [0, 7, 60])
def test_allocator_failure_is_enomem_and_releases(fail_after):
    import torch
    from paper_2505_18576_amd import amgf as b
    p = problem("C1")
    A = b.TorchAllocator()
    A.fail_after = fail_after
    print(f"allocator failing after {fail_after} blocks", flush=True)
    with pytest.raises(b.AMGFError) as e:
        b.AMGF.from_problem(p, allocator=A)
    torch.cuda.synchronize()
    assert e.value.status == b.AMGF_ENOMEM
    assert A.n_alloc == fail_after and A.live == 0
