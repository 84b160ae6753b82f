"""ctypes binding of ``libamgf.so`` (the C ABI in include/amgf.h).

Argument marshalling only: every step of setup, V-cycle, filter and CG runs in the
library's HIP kernels.  PyTorch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamgf.so")

AMGF_OK, AMGF_EINVAL, AMGF_ENOTSPD, AMGF_ENOCONV, AMGF_ENOMEM, AMGF_EDEVICE = range(6)
FP64, MIXED_FP32, MIXED_BF16K = 0, 1, 2
L1JACOBI, CHEBYSHEV, LEARNED = 0, 1, 2
(Q_SIZES, Q_A_ROWPTR, Q_A_COL, Q_A_VAL, Q_AGG, Q_ROOT, Q_G_ROWPTR, Q_G_COL, Q_P_ROWPTR,
 Q_P_COL, Q_P_VAL, Q_L1, Q_K_ROWPTR, Q_K_COL, Q_K_VAL, Q_OMEGA, Q_IC, Q_FEATURES,
 Q_THETA, Q_CG_COEF, Q_CONTACT) = range(21)
MLP_NPARAM, MLP_NTOTAL = 1313, 1325

ABI_FUNCTIONS = ["amgf_default_options", "amgf_setup", "amgf_apply", "amgf_vcycle",
                 "amgf_operator_apply", "amgf_pcg", "amgf_destroy", "amgf_status_string",
                 "amgf_last_error", "amgf_num_levels", "amgf_query", "amgf_time_kernel",
                 "amgf_set_mlp", "amgf_mlp_loss_grad", "amgf_adam_step",
                 "amgf_profile_start", "amgf_profile_read", "amgf_filter_solve",
                 "amgf_update_D", "amgf_ip_default_options", "amgf_ip_solve",
                 "amgf_update_barrier", "amgf_pcg_noalloc"]
K_PRESMOOTH, K_POSTSMOOTH, K_VCYCLE, K_OPERATOR = range(4)


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


class TorchAllocator:
    """amgf_allocator backed by PyTorch's caching allocator on the current device.

    Blocks are taken on the stream the library passes and returned with
    ``caching_allocator_delete``; ``live`` counts the blocks the library holds."""

    def __init__(self):
        torch = _torch()
        self._torch = torch
        self.device = torch.cuda.current_device()
        self.live, self.n_alloc, self.fail_after = 0, 0, None
        self._a, self._f = ALLOC_FN(self._alloc), FREE_FN(self._free)
        self.struct = Allocator(self._a, self._f, None)

    def _alloc(self, nbytes, stream, ctx):
        if self.fail_after is not None and self.n_alloc >= self.fail_after:
            return None
        try:
            ptr = self._torch.cuda.caching_allocator_alloc(int(nbytes), self.device, stream or 0)
        except Exception:
            return None
        self.live += 1
        self.n_alloc += 1
        return ptr

    def _free(self, ptr, stream, ctx):
        self._torch.cuda.caching_allocator_delete(ptr)
        self.live -= 1


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("smoother", ctypes.c_int32), ("filter", ctypes.c_int32),
                ("max_levels", ctypes.c_int32), ("coarse_max_nodes", ctypes.c_int32),
                ("max_iters", ctypes.c_int32), ("sa_power_iters", ctypes.c_int32),
                ("strength_theta", ctypes.c_double), ("rtol", ctypes.c_double),
                ("sa_omega", ctypes.c_double), ("qr_tol", ctypes.c_double),
                ("max_coarse_ratio", ctypes.c_double),
                ("mlp_weights", ctypes.POINTER(ctypes.c_float)),
                ("sweeps", ctypes.c_int32), ("cheb_degree", ctypes.c_int32),
                ("allocator", Allocator), ("bound_diag", ctypes.c_void_p),
                ("near_null", ctypes.c_int32), ("learned_judge", ctypes.c_int32),
                ("transfer_fp16", ctypes.c_int32), ("cycle_gamma", ctypes.c_int32)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("n_c", ctypes.c_int32),
                ("rel_prec_res", ctypes.c_double), ("rel_true_res", ctypes.c_double),
                ("op_complexity", ctypes.c_double), ("ms_solve", ctypes.c_float),
                ("used_fallback", ctypes.c_int32), ("ms_setup_amg", ctypes.c_float),
                ("ms_setup_filter", ctypes.c_float), ("ms_amg_apply", ctypes.c_float),
                ("ms_filter_apply", ctypes.c_float), ("ms_cg_other", ctypes.c_float),
                ("pad_", ctypes.c_int32), ("judge_learned", ctypes.c_double),
                ("judge_plain", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class IPOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("tol", ctypes.c_double), ("mu0", ctypes.c_double),
                ("kappa_eps", ctypes.c_double), ("kappa_mu", ctypes.c_double),
                ("theta_mu", ctypes.c_double), ("tau_min", ctypes.c_double),
                ("s_max", ctypes.c_double), ("s_init", ctypes.c_double),
                ("switch_ratio", ctypes.c_double)]


class IPStep(ctypes.Structure):
    _fields_ = [("mu", ctypes.c_double), ("e_opt", ctypes.c_double),
                ("e_opt_mu", ctypes.c_double), ("alpha_p", ctypes.c_double),
                ("alpha_d", ctypes.c_double), ("D_min", ctypes.c_double),
                ("D_max", ctypes.c_double), ("pcg_iterations", ctypes.c_int32),
                ("pcg_converged", ctypes.c_int32), ("filter_on", ctypes.c_int32),
                ("pad", ctypes.c_int32), ("ms_update", ctypes.c_float),
                ("ms_solve", ctypes.c_float)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}


_lib = None


def load_library(path=LIB_PATH):
    """Load libamgf.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           "`python -m paper_2505_18576_amd.build` (there is no CPU path)")
    L = ctypes.CDLL(path)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    L.amgf_default_options.argtypes = [ctypes.POINTER(Options)]
    L.amgf_default_options.restype = None
    L.amgf_setup.argtypes = [ctypes.POINTER(Options), i32, vp, vp, vp, i32, vp, vp, vp, vp, vp,
                             vp, i32, vp, ctypes.POINTER(vp)]
    L.amgf_setup.restype = ctypes.c_int
    for f in ("amgf_apply", "amgf_vcycle", "amgf_operator_apply", "amgf_filter_solve"):
        getattr(L, f).argtypes = [vp, vp, vp, vp]
        getattr(L, f).restype = ctypes.c_int
    L.amgf_pcg.argtypes = [vp, vp, vp, ctypes.POINTER(SolveInfo), vp]
    L.amgf_pcg.restype = ctypes.c_int
    L.amgf_pcg_noalloc.argtypes = [vp, vp, vp, ctypes.POINTER(SolveInfo), vp]
    L.amgf_pcg_noalloc.restype = ctypes.c_int
    L.amgf_destroy.argtypes = [vp]
    L.amgf_destroy.restype = None
    L.amgf_status_string.argtypes = [ctypes.c_int]
    L.amgf_status_string.restype = ctypes.c_char_p
    L.amgf_last_error.argtypes = []
    L.amgf_last_error.restype = ctypes.c_char_p
    L.amgf_num_levels.argtypes = [vp]
    L.amgf_num_levels.restype = i32
    L.amgf_query.argtypes = [vp, i32, i32, vp, ctypes.c_size_t]
    L.amgf_query.restype = ctypes.c_int
    L.amgf_time_kernel.argtypes = [vp, i32, i32, vp, ctypes.POINTER(ctypes.c_double)]
    L.amgf_time_kernel.restype = ctypes.c_int
    L.amgf_set_mlp.argtypes = [vp, vp, vp]
    L.amgf_set_mlp.restype = ctypes.c_int
    L.amgf_mlp_loss_grad.argtypes = [vp, vp, i32, i32, vp, ctypes.POINTER(dbl), vp, vp]
    L.amgf_mlp_loss_grad.restype = ctypes.c_int
    L.amgf_adam_step.argtypes = [vp, vp, vp, vp, i32, ctypes.c_float, vp]
    L.amgf_adam_step.restype = ctypes.c_int
    L.amgf_update_D.argtypes = [vp, vp, vp]
    L.amgf_update_D.restype = ctypes.c_int
    L.amgf_update_barrier.argtypes = [vp, vp, vp, vp]
    L.amgf_update_barrier.restype = ctypes.c_int
    L.amgf_profile_start.argtypes = [vp, i32, i32]
    L.amgf_profile_start.restype = ctypes.c_int
    L.amgf_profile_read.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    L.amgf_profile_read.restype = ctypes.c_int
    L.amgf_ip_default_options.argtypes = [ctypes.POINTER(IPOptions)]
    L.amgf_ip_default_options.restype = None
    L.amgf_ip_solve.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, ctypes.POINTER(IPOptions),
                                ctypes.POINTER(IPStep), i32, ctypes.POINTER(i32),
                                ctypes.POINTER(i32), vp]
    L.amgf_ip_solve.restype = ctypes.c_int
    _lib = L
    return L


class AMGFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


def _check(status, what):
    if status != AMGF_OK:
        L = load_library()
        raise AMGFError(status, f"{what}: {L.amgf_status_string(status).decode()}: "
                                f"{L.amgf_last_error().decode()}")


def default_options(**kw):
    L = load_library()
    o = Options()
    L.amgf_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def ip_default_options(**kw):
    L = load_library()
    o = IPOptions()
    L.amgf_ip_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the AMGF library needs a ROCm GPU (torch.cuda is unavailable)")
    return torch


def _dev(x, dtype):
    torch = _torch()
    if isinstance(x, torch.Tensor):
        t = x.to(device="cuda", dtype=dtype)
    else:
        t = torch.from_numpy(np.ascontiguousarray(x)).to(device="cuda", dtype=dtype)
    return t.contiguous()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _stream():
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class AMGF:
    """Handle of an AMGF hierarchy on the current GPU.

    Inputs may be numpy arrays or torch tensors; they are placed on the GPU with the
    dtypes of the C ABI (int32 indices, float64 values).
    """

    def __init__(self, n_nodes, K_rowptr, K_col, K_val, J_rowptr, J_col, J_val, D, coords,
                 Ic=None, options=None, mlp_weights=None, allocator=None, E=None, **kw):
        torch = _torch()
        self.L = load_library()
        self.options = options if options is not None else default_options(**kw)
        # allocator: None (hipMalloc), "torch", or a TorchAllocator; kept alive with the handle
        self.allocator = TorchAllocator() if allocator == "torch" else allocator
        if self.allocator is not None:
            self.options.allocator = self.allocator.struct
        self._w = None
        if mlp_weights is not None:
            self._w = np.ascontiguousarray(mlp_weights, dtype=np.float32)
            if self._w.size != MLP_NTOTAL:
                raise ValueError(f"mlp_weights needs {MLP_NTOTAL} values")
            self.options.smoother = LEARNED
            self.options.mlp_weights = self._w.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        i32, f64 = torch.int32, torch.float64
        self._keep = [_dev(K_rowptr, i32), _dev(K_col, i32), _dev(K_val, f64),
                      _dev(J_rowptr, i32), _dev(J_col, i32), _dev(J_val, f64), _dev(D, f64),
                      _dev(coords, f64)]
        self.m = int(len(self._keep[3]) - 1)
        self.n_nodes = int(n_nodes)
        self.n = 3 * self.n_nodes
        ic = _dev(Ic, i32) if Ic is not None else None
        # E: barrier diagonal of bound constraints (n values >= 0), read during setup
        Ed = None
        if E is not None:
            Ed = _dev(E, f64).reshape(-1)
            if Ed.numel() != self.n:
                raise ValueError(f"E needs {self.n} values")
            self.options.bound_diag = Ed.data_ptr()
        h = ctypes.c_void_p()
        st = self.L.amgf_setup(ctypes.byref(self.options), self.n_nodes,
                               *[_ptr(t) for t in self._keep[:3]], self.m,
                               *[_ptr(t) for t in self._keep[3:]],
                               _ptr(ic), 0 if ic is None else int(ic.numel()), _stream(),
                               ctypes.byref(h))
        _check(st, "amgf_setup")
        self.h = h
        torch.cuda.synchronize()
        self._keep = None
        self.options.bound_diag = None

    @classmethod
    def from_problem(cls, p, **kw):
        return cls(p.n_nodes, p.K_rowptr, p.K_col, p.K_val.reshape(-1), p.J_rowptr, p.J_col,
                   p.J_val, p.D, p.coords.reshape(-1), **kw)

    def _vec_op(self, fn, x, name):
        torch = _torch()
        xd = _dev(x, torch.float64)
        y = torch.empty_like(xd)
        _check(fn(self.h, _ptr(xd), _ptr(y), _stream()), name)
        return y

    def apply(self, r):
        return self._vec_op(self.L.amgf_apply, r, "amgf_apply")

    def update_D(self, D):
        """New interior-point step: same K and J, new barrier diagonal D (m values > 0)."""
        torch = _torch()
        Dd = _dev(D, torch.float64)
        _check(self.L.amgf_update_D(self.h, _ptr(Dd), _stream()), "amgf_update_D")
        torch.cuda.synchronize()

    def update_barrier(self, D, E=None):
        """New barrier terms: contact diagonal D (m > 0) and bound diagonal E (n >= 0, or
        None to drop it); the stiffness chain is rebuilt with the kept prolongators."""
        torch = _torch()
        Dd = _dev(D, torch.float64)
        Ed = None if E is None else _dev(E, torch.float64).reshape(-1)
        if Ed is not None and Ed.numel() != self.n:
            raise ValueError(f"E needs {self.n} values")
        _check(self.L.amgf_update_barrier(self.h, _ptr(Dd), _ptr(Ed), _stream()),
               "amgf_update_barrier")
        torch.cuda.synchronize()

    def filter_solve(self, rc):
        """w_c = A_w^{-1} r_c on the filtering space (vectors in the order of I_c)."""
        return self._vec_op(self.L.amgf_filter_solve, rc, "amgf_filter_solve")

    def vcycle(self, r):
        return self._vec_op(self.L.amgf_vcycle, r, "amgf_vcycle")

    def operator(self, x):
        return self._vec_op(self.L.amgf_operator_apply, x, "amgf_operator_apply")

    def pcg(self, b, x0=None, raise_on_noconv=False):
        torch = _torch()
        bd = _dev(b, torch.float64)
        x = torch.zeros_like(bd) if x0 is None else _dev(x0, torch.float64).clone()
        info = SolveInfo()
        st = self.L.amgf_pcg(self.h, _ptr(bd), _ptr(x), ctypes.byref(info), _stream())
        if st == AMGF_ENOCONV and not raise_on_noconv:
            return x, info
        _check(st, "amgf_pcg")
        return x, info

    def pcg_noalloc(self, b, x):
        """amgf_pcg_noalloc on caller-owned device tensors b and x (x: initial guess in,
        solution out); returns (status, info).  Allocates nothing on the device."""
        info = SolveInfo()
        st = self.L.amgf_pcg_noalloc(self.h, _ptr(b), _ptr(x), ctypes.byref(info), _stream())
        if st not in (AMGF_OK, AMGF_ENOCONV):
            _check(st, "amgf_pcg_noalloc")
        return st, info

    def ip_solve(self, f, g0, u0=None, Ms=None, Mu=None, **opts):
        """Interior-point solve of min 1/2 u^T K u - f^T u s.t. J u + g0 >= 0 with this
        handle's K and J (amgf_ip_solve); Ms (m) and Mu (n) are the lumped slack and
        displacement masses (default ones).  Returns (u, s, lam, z, steps, converged), the
        vectors as device tensors and ``steps`` a list of per-Newton-step dicts."""
        torch = _torch()
        o = ip_default_options(**opts)
        fd = _dev(f, torch.float64).reshape(-1)
        gd = _dev(g0, torch.float64).reshape(-1)
        if fd.numel() != self.n or gd.numel() != self.m:
            raise ValueError(f"f needs {self.n} values and g0 {self.m}")
        u = torch.zeros_like(fd) if u0 is None else _dev(u0, torch.float64).clone()
        if u.numel() != self.n:
            raise ValueError(f"u0 needs {self.n} values")
        msd = None if Ms is None else _dev(Ms, torch.float64).reshape(-1)
        mud = None if Mu is None else _dev(Mu, torch.float64).reshape(-1)
        if (msd is not None and msd.numel() != self.m) or (mud is not None and
                                                           mud.numel() != self.n):
            raise ValueError(f"Ms needs {self.m} values and Mu {self.n}")
        s, lam, z = (torch.empty(self.m, dtype=torch.float64, device="cuda") for _ in range(3))
        rec = (IPStep * max(o.max_steps, 1))()
        ns, conv = ctypes.c_int32(), ctypes.c_int32()
        _check(self.L.amgf_ip_solve(self.h, _ptr(fd), _ptr(gd), _ptr(msd), _ptr(mud), _ptr(u),
                                    _ptr(s), _ptr(lam),
                                    _ptr(z), ctypes.byref(o), rec, len(rec), ctypes.byref(ns),
                                    ctypes.byref(conv), _stream()), "amgf_ip_solve")
        torch.cuda.synchronize()
        steps = [rec[i].as_dict() for i in range(min(ns.value, len(rec)))]
        return u, s, lam, z, steps, bool(conv.value)

    @property
    def n_levels(self):
        return int(self.L.amgf_num_levels(self.h))

    def query(self, level, which, dtype=None, count=None):
        """Copy one hierarchy array of ``level`` to a numpy array."""
        if which == Q_SIZES:
            out = np.zeros(8, np.int32)
        elif which == Q_OMEGA:
            out = np.zeros(2, np.float64)
        else:
            out = np.zeros(count, dtype)
        st = self.L.amgf_query(self.h, level, which, out.ctypes.data_as(ctypes.c_void_p),
                               out.nbytes)
        _check(st, "amgf_query")
        return out

    def level_arrays(self, level):
        """Dict of the level's operator, aggregation and prolongator arrays."""
        s = self.query(level, Q_SIZES)
        nn, b, nnzA, n_agg, nnzP, nnzG, nnzK = [int(v) for v in s[:7]]
        q = self.query
        d = dict(n_nodes=nn, b=b, n_agg=n_agg,
                 A_rowptr=q(level, Q_A_ROWPTR, np.int32, nn + 1),
                 A_col=q(level, Q_A_COL, np.int32, nnzA),
                 A_val=q(level, Q_A_VAL, np.float64, nnzA * b * b).reshape(-1, b, b),
                 K_rowptr=q(level, Q_K_ROWPTR, np.int32, nn + 1),
                 K_col=q(level, Q_K_COL, np.int32, nnzK),
                 K_val=q(level, Q_K_VAL, np.float64, nnzK * b * b).reshape(-1, b, b),
                 l1=q(level, Q_L1, np.float64, nn * b))
        if n_agg:
            d.update(agg=q(level, Q_AGG, np.int32, nn), root=q(level, Q_ROOT, np.int32, nn),
                     G_rowptr=q(level, Q_G_ROWPTR, np.int32, nn + 1),
                     G_col=q(level, Q_G_COL, np.int32, nnzG),
                     P_rowptr=q(level, Q_P_ROWPTR, np.int32, nn + 1),
                     P_col=q(level, Q_P_COL, np.int32, nnzP),
                     P_val=q(level, Q_P_VAL, np.float64,
                             nnzP * b * self.options.near_null).reshape(
                                 -1, b, self.options.near_null),
                     rho_omega=q(level, Q_OMEGA))
        return d

    def time_kernel(self, which, reps=20):
        """Mean milliseconds per launch of a hot-path kernel (hipEvents, library stream)."""
        ms = ctypes.c_double()
        _check(self.L.amgf_time_kernel(self.h, which, reps, _stream(), ctypes.byref(ms)),
               "amgf_time_kernel")
        return ms.value

    def profile_start(self, which, max_launches=100000):
        """Time every later launch of a level-0 smoother kernel inside solves (hipEvents on
        the solve stream); which < 0 switches it off."""
        _check(self.L.amgf_profile_start(self.h, which, max_launches), "amgf_profile_start")

    def profile_read(self):
        """(number of timed launches, mean milliseconds per launch); clears the record."""
        cnt, ms = ctypes.c_int32(), ctypes.c_double()
        _check(self.L.amgf_profile_read(self.h, ctypes.byref(cnt), ctypes.byref(ms)),
               "amgf_profile_read")
        return cnt.value, ms.value

    def set_mlp(self, W):
        """Damping from the MLP with parameters W (1325 values), or theta = 1 for None."""
        torch = _torch()
        if W is None:
            _check(self.L.amgf_set_mlp(self.h, None, _stream()), "amgf_set_mlp")
            return
        Wd = _dev(W, torch.float32)
        _check(self.L.amgf_set_mlp(self.h, _ptr(Wd), _stream()), "amgf_set_mlp")
        torch.cuda.synchronize()

    def loss_grad(self, W, probes, k=2):
        """(loss, grad) of the learned-damping objective; probes is (n, count)."""
        torch = _torch()
        Wd = _dev(W, torch.float32)
        P = _dev(np.asarray(probes).T if not isinstance(probes, torch.Tensor) else probes.T,
                 torch.float64)                       # column q contiguous
        g = torch.zeros(MLP_NPARAM, dtype=torch.float64, device="cuda")
        loss = ctypes.c_double()
        _check(self.L.amgf_mlp_loss_grad(self.h, _ptr(Wd), k, int(P.shape[0]), _ptr(P),
                                         ctypes.byref(loss), _ptr(g), _stream()),
               "amgf_mlp_loss_grad")
        return loss.value, g

    def features(self, level):
        n = int(self.query(level, Q_SIZES)[0]) * int(self.query(level, Q_SIZES)[1])
        return self.query(level, Q_FEATURES, np.float64, 6 * n).reshape(6, n)

    def theta(self, level):
        n = int(self.query(level, Q_SIZES)[0]) * int(self.query(level, Q_SIZES)[1])
        return self.query(level, Q_THETA, np.float64, n)

    def contact_mode(self, level):
        """(mode, rows) of the level's contact term in the V-cycle: 0 none, 1 through J
        and D, 2 assembled into the smoothing matrix A_l = K_l + C_l; rows = node rows it
        touches."""
        m = self.query(level, Q_CONTACT, np.int32, 2)
        return int(m[0]), int(m[1])

    def filter_dofs(self, n_c):
        return self.query(0, Q_IC, np.int32, n_c)

    def cg_coefficients(self, iterations):
        """(alpha, beta) of the last pcg call with `iterations` iterations: alpha_k =
        r.z / p.Ap, beta_k = r'.z' / r.z, the Lanczos coefficients of M A."""
        c = self.query(0, Q_CG_COEF, np.float64, 2 * int(iterations))
        return c[:iterations], c[iterations:]

    def close(self):
        if getattr(self, "h", None):
            self.L.amgf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adam_step(W, grad, m1, m2, t, lr):
    """In-place Adam step on device tensors (W, m1, m2 float32; grad float64)."""
    L = load_library()
    _check(L.amgf_adam_step(_ptr(W), _ptr(grad), _ptr(m1), _ptr(m2), int(t), float(lr),
                            _stream()), "amgf_adam_step")
