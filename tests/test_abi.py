"""The C ABI library builds, loads without a GPU, and exports what include/amgf.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "amgf.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(amgf_[A-Za-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_2505_18576_amd import amgf as b
    if not os.path.exists(b.LIB_PATH):
        from paper_2505_18576_amd.build import build
        build()
    return b.load_library()


def test_header_declares_the_boundary():
    names = _declared_functions()
    for f in ("amgf_setup", "amgf_apply", "amgf_pcg", "amgf_destroy", "amgf_vcycle",
              "amgf_operator_apply", "amgf_status_string"):
        assert f in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2505_18576_amd import amgf as b
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(b.ABI_FUNCTIONS) == set(_declared_functions())


def test_host_only_entry_points(lib):
    from paper_2505_18576_amd import amgf as b
    o = b.default_options()
    assert o.struct_size == __import__("ctypes").sizeof(b.Options)
    assert (o.rtol, o.max_iters, o.filter, o.coarse_max_nodes) == (1e-10, 5000, 1, 1024)
    assert (o.strength_theta, o.sa_omega, o.near_null) == (0.04, 1.5, 6)
    assert lib.amgf_status_string(b.AMGF_ENOCONV) == b"AMGF_ENOCONV"
    # argument checks happen before any device work
    import ctypes
    h = ctypes.c_void_p()
    st = lib.amgf_setup(ctypes.byref(o), 0, None, None, None, 0, None, None, None, None, None,
                        None, 0, None, ctypes.byref(h))
    assert st == b.AMGF_EINVAL and not h.value
    assert lib.amgf_apply(None, None, None, None) == b.AMGF_EINVAL
    assert lib.amgf_pcg(None, None, None, None, None) == b.AMGF_EINVAL
    lib.amgf_destroy(None)


def test_binding_refuses_to_run_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    from amgf_inputs import make_config
    from paper_2505_18576_amd import AMGF
    with pytest.raises(RuntimeError, match="GPU"):
        AMGF.from_problem(make_config("C1"))


def test_allocator_needs_both_callbacks(lib):
    """An amgf_allocator with alloc but no free is refused before any device work."""
    import ctypes
    from paper_2505_18576_amd import amgf as b
    o = b.default_options()
    keep = b.ALLOC_FN(lambda nbytes, stream, ctx: None)
    o.allocator.alloc = keep
    fake = ctypes.c_void_p(256)
    h = ctypes.c_void_p()
    st = lib.amgf_setup(ctypes.byref(o), 8, fake, fake, fake, 0, None, None, None, None, fake,
                        None, 0, None, ctypes.byref(h))
    assert st == b.AMGF_EINVAL and not h.value
    assert b"alloc and free" in lib.amgf_last_error()


def test_ip_options_defaults(lib):
    import ctypes
    from paper_2505_18576_amd import amgf as b
    o = b.ip_default_options()
    assert o.struct_size == ctypes.sizeof(b.IPOptions)
    assert (o.max_steps, o.tol, o.mu0, o.kappa_eps, o.s_max) == (200, 1e-6, 0.1, 10.0, 100.0)
    assert ctypes.sizeof(b.IPStep) == 7 * 8 + 4 * 4 + 2 * 4
    n, c = ctypes.c_int32(), ctypes.c_int32()
    assert lib.amgf_ip_solve(None, None, None, None, None, None, None, None, None, None, None, 0,
                             ctypes.byref(n), ctypes.byref(c), None) == b.AMGF_EINVAL
