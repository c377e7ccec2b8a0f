"""Thin ctypes binding of the tmx C ABI (``include/tmx.h``).

Every ``tmx_*`` function here has the name and argument order of the C entry
point and only marshals arguments: device memory comes from torch tensors
(``data_ptr()``), the HIP stream is torch's current stream, and every step of
the computation runs in the HIP library.  Importing this module loads
``libtmx.so`` and raises if it is missing -- there is no fallback.

:class:`Context` bundles the calls for convenience (it still only marshals).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmx.so")

TMX_OK, TMX_ENOCONV, TMX_EINVAL, TMX_ENOTLOADED, TMX_ENOMEM, TMX_EHIP = 0, 1, -1, -2, -3, -4
TMX_F64, TMX_F32, TMX_F16 = 0, 1, 2
TMX_OP_PLUS, TMX_OP_MINUS, TMX_OP_ND, TMX_OP_WPLUS, TMX_OP_WMINUS = 1, -1, 2, 3, -3
TMX_FIELD_ODD, TMX_FIELD_ODD_ND, TMX_FIELD_FULL, TMX_FIELD_FULL_ND = 0, 1, 2, 3
TMX_SOLVER_CG, TMX_SOLVER_MPCG_F32, TMX_SOLVER_MPCG_F16, TMX_SOLVER_FGCR_NN, TMX_SOLVER_PCG_NN = 0, 1, 2, 3, 4
TMX_SOLVER_PCG_NN_SYM = 5
TMX_SOLVER_PCG_NN_SYM1 = 6
TMX_LOSS_RESIDUAL, TMX_LOSS_SOLUTION, TMX_LOSS_SYM, TMX_LOSS_SYM1 = 0, 1, 2, 3

PREC = {"f64": TMX_F64, "f32": TMX_F32, "f16": TMX_F16}


class TmxError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tmx error {code}: {msg}")
        self.code = code


class tmx_params(ctypes.Structure):
    _fields_ = [("kappa", ctypes.c_double), ("csw", ctypes.c_double), ("mu", ctypes.c_double),
                ("mubar", ctypes.c_double), ("epsbar", ctypes.c_double), ("t_bc", ctypes.c_int),
                ("rho", ctypes.c_double)]


class tmx_solver_cfg(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("op", ctypes.c_int), ("tol", ctypes.c_double), ("maxiter", ctypes.c_int),
                ("delta", ctypes.c_double), ("restart", ctypes.c_int), ("use_initial_guess", ctypes.c_int),
                ("inner_tol", ctypes.c_double), ("inner_prec", ctypes.c_int)]


class tmx_info(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("reliable_updates", ctypes.c_int), ("restarts", ctypes.c_int),
                ("fallback", ctypes.c_int), ("true_residual", ctypes.c_double), ("seconds", ctypes.c_double),
                ("gbytes", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class tmx_train_cfg(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("seed", ctypes.c_int), ("loss_kind", ctypes.c_int), ("op", ctypes.c_int)]


# the device allocator hooks of tmx_set_allocator
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
NO_ALLOC, NO_RELEASE = ALLOC_FN(0), RELEASE_FN(0)  # NULL hooks: back to hipMalloc / hipFree


def _load():
    # torch first: its bundled HIP runtime then satisfies libtmx.so's
    # dependency, so device pointers and streams are shared by both.
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_06635_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, Z = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "tmx_create": ([ctypes.POINTER(ctypes.c_int), P, ctypes.POINTER(P)], I),
        "tmx_destroy": ([P], I),
        "tmx_last_error": ([P], ctypes.c_char_p),
        "tmx_set_stream": ([P, P], I),
        "tmx_set_params": ([P, ctypes.POINTER(tmx_params)], I),
        "tmx_set_allocator": ([P, ALLOC_FN, RELEASE_FN, P], I),
        "tmx_free_workspaces": ([P], I),
        "tmx_load_gauge": ([P, P, D], I),
        "tmx_gauge_uploads": ([P], I),
        "tmx_load_clover": ([P, P], I),
        "tmx_get_clover": ([P, P], I),
        "tmx_field_bytes": ([P, I, I, ctypes.POINTER(Z)], I),
        "tmx_pack": ([P, P, P, I, I, I], I),
        "tmx_unpack": ([P, P, P, I, I, I], I),
        "tmx_apply_D": ([P, P, P, I, I], I),
        "tmx_apply_mhat": ([P, P, P, I, I, I, I], I),
        "tmx_apply_mdagm": ([P, P, P, I, I, I], I),
        "tmx_apply_mhat_noalloc": ([P, P, P, I, I, I, I], I),
        "tmx_solve": ([P, P, P, I, ctypes.POINTER(tmx_solver_cfg), P], I),
        "tmx_solve_mhat": ([P, P, P, I, ctypes.POINTER(tmx_solver_cfg), P], I),
        "tmx_multishift_solve": ([P, P, P, P, I, ctypes.POINTER(tmx_solver_cfg), P], I),
        "tmx_rational_apply": ([P, P, P, D, P, P, I, ctypes.POINTER(tmx_solver_cfg), P], I),
        "tmx_rational_force": ([P, P, P, P, P, I, ctypes.POINTER(tmx_solver_cfg), I, P], I),
        "tmx_hop_force": ([P, P, P, P, I, D, I], I),
        "tmx_clover_force": ([P, P, P, P, I, D, I], I),
        "tmx_rational_correction": ([P, P, D, P, P, I, D, I, ctypes.POINTER(tmx_solver_cfg), ctypes.POINTER(D),
                                     ctypes.POINTER(I)], I),
        "tmx_pc_num_params": ([P, ctypes.POINTER(Z)], I),
        "tmx_pc_set_weights": ([P, P, Z], I),
        "tmx_pc_get_weights": ([P, P, Z], I),
        "tmx_pc_apply": ([P, P, P, I], I),
        "tmx_pc_train": ([P, P, P, I, ctypes.POINTER(tmx_train_cfg), P], I),
        "tmx_pc_adam_step": ([P, P, Z, ctypes.POINTER(tmx_train_cfg)], I),
        "tmx_pc_loss_grad": ([P, P, P, I, I, I, ctypes.POINTER(D), P], I),
        "tmx_tune": ([P, I, I, I], I),
        "tmx_tuned_config": ([P, ctypes.c_char_p, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                              ctypes.POINTER(I)], I),
        "tmx_kstats_enable": ([P, I], I),
        "tmx_kstats_get": ([P, I, ctypes.c_char_p, Z, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(D)], I),
        "tmx_trace_enable": ([P, I], I),
        "tmx_trace_push": ([P, ctypes.c_char_p], I),
        "tmx_trace_pop": ([P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()
EXPORTED = [n for n in dir(lib) if n.startswith("tmx_")]


def _ptr(t) -> int:
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream_handle():
    import torch

    return torch.cuda.current_stream().cuda_stream


class TorchAllocator:
    """Device buffers of a context from torch's caching allocator.

    The library calls ``alloc(bytes)`` for every device buffer it needs (links,
    clover blocks, inverses, workspaces, network state) and ``release(ptr)``
    when it is done with one; each buffer is a torch uint8 tensor kept alive
    here until released.  Counts and bytes are kept for inspection."""

    def __init__(self):
        import torch

        self.torch = torch
        self.live = {}
        self.n_alloc = 0
        self.n_release = 0
        self.bytes_alloc = 0

        def _alloc(nbytes, user):
            try:
                t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device="cuda")
            except Exception:  # out of memory: the library reports TMX_ENOMEM
                return None
            p = t.data_ptr()
            self.live[p] = t
            self.n_alloc += 1
            self.bytes_alloc += int(nbytes)
            return p

        def _release(ptr, user):
            if self.live.pop(ptr, None) is not None:
                self.n_release += 1

        # the ctypes function objects must outlive every call into the library
        self.alloc_fn = ALLOC_FN(_alloc)
        self.release_fn = RELEASE_FN(_release)

    @property
    def live_bytes(self):
        return sum(t.numel() for t in self.live.values())


@dataclass
class Params:
    kappa: float
    csw: float
    mu: float = 0.0
    mubar: float = 0.0
    epsbar: float = 0.0
    t_bc: int = -1
    rho: float = 0.0


class Context:
    """One lattice geometry on the current device; device memory via torch."""

    def __init__(self, dims, stream=None, allocator="torch"):
        """allocator: "torch" (default) routes every device buffer of the
        library through torch's caching allocator (tmx_set_allocator); "hip"
        leaves the library on hipMalloc."""
        import torch

        self.torch = torch
        self.dims = tuple(int(d) for d in dims)
        self.V = int(np.prod(self.dims))
        self.Vh = self.V // 2
        h = ctypes.c_void_p()
        arr = (ctypes.c_int * 4)(*self.dims)
        st = stream if stream is not None else _stream_handle()
        rc = lib.tmx_create(arr, ctypes.c_void_p(st), ctypes.byref(h))
        if rc != TMX_OK:
            raise TmxError(rc, "tmx_create failed")
        self.h = h
        self.allocator = None
        if allocator == "torch":
            self.allocator = TorchAllocator()
            self.check(lib.tmx_set_allocator(self.h, self.allocator.alloc_fn, self.allocator.release_fn, None))
        elif allocator != "hip":
            raise ValueError(f"unknown allocator {allocator!r}")

    # -- plumbing ----------------------------------------------------------
    def check(self, rc, allow_noconv=False):
        if rc == TMX_OK or (allow_noconv and rc == TMX_ENOCONV):
            return rc
        raise TmxError(rc, lib.tmx_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib.tmx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream=None):
        return self.check(lib.tmx_set_stream(self.h, ctypes.c_void_p(stream if stream is not None else _stream_handle())))

    # -- state ---------------------------------------------------------------
    def set_params(self, p: Params):
        cp = tmx_params(p.kappa, p.csw, p.mu, p.mubar, p.epsbar, p.t_bc, p.rho)
        return self.check(lib.tmx_set_params(self.h, ctypes.byref(cp)))

    def load_gauge(self, U: np.ndarray, gauge_id: float):
        U = np.ascontiguousarray(U, dtype=np.complex128)
        assert U.size == self.V * 36
        return self.check(lib.tmx_load_gauge(self.h, U.ctypes.data, float(gauge_id)))

    def gauge_uploads(self):
        return lib.tmx_gauge_uploads(self.h)

    def load_clover(self, T=None):
        if T is None:
            return self.check(lib.tmx_load_clover(self.h, None))
        T = np.ascontiguousarray(T, dtype=np.complex128)
        return self.check(lib.tmx_load_clover(self.h, T.ctypes.data))

    def get_clover(self):
        T = np.empty((self.V, 2, 6, 6), dtype=np.complex128)
        self.check(lib.tmx_get_clover(self.h, T.ctypes.data))
        return T

    # -- fields --------------------------------------------------------------
    def field_bytes(self, kind, prec):
        n = ctypes.c_size_t()
        self.check(lib.tmx_field_bytes(self.h, kind, prec, ctypes.byref(n)))
        return n.value

    def empty(self, kind, prec, nvec=1):
        return self.torch.empty(self.field_bytes(kind, prec) * nvec, dtype=self.torch.uint8, device="cuda")

    def pack(self, canon, kind, prec, nvec=1):
        out = self.empty(kind, prec, nvec)
        canon = canon.contiguous()
        self.check(lib.tmx_pack(self.h, _ptr(out), _ptr(canon), kind, prec, nvec))
        return out

    def unpack(self, internal, kind, prec, nvec=1):
        n = (self.V if kind >= 2 else self.Vh) * (2 if kind in (1, 3) else 1) * 12 * nvec
        out = self.torch.empty(n, dtype=self.torch.complex128, device="cuda")
        self.check(lib.tmx_unpack(self.h, _ptr(out), _ptr(internal), kind, prec, nvec))
        return out

    # -- operators (internal layout) ------------------------------------------
    def apply_D(self, out, inp, op, prec):
        return self.check(lib.tmx_apply_D(self.h, _ptr(out), _ptr(inp), op, prec))

    def apply_mhat(self, out, inp, op, prec, dagger=0, nrhs=1):
        return self.check(lib.tmx_apply_mhat(self.h, _ptr(out), _ptr(inp), op, prec, int(dagger), nrhs))

    def apply_mhat_noalloc(self, out, inp, op, prec, dagger=0, nrhs=1):
        return self.check(lib.tmx_apply_mhat_noalloc(self.h, _ptr(out), _ptr(inp), op, prec, int(dagger), nrhs))

    def apply_mdagm(self, out, inp, op, prec, nrhs=1):
        return self.check(lib.tmx_apply_mdagm(self.h, _ptr(out), _ptr(inp), op, prec, nrhs))

    # -- solvers (canonical complex128 device tensors) -----------------------
    @staticmethod
    def cfg(kind=TMX_SOLVER_CG, op=TMX_OP_PLUS, tol=1e-10, maxiter=10000, delta=0.0, restart=16,
            use_initial_guess=0, inner_tol=0.0, inner_prec=TMX_F32):
        return tmx_solver_cfg(kind, op, tol, maxiter, delta, restart, use_initial_guess, inner_tol, inner_prec)

    def solve(self, x, b, nrhs=1, **kw):
        cfg = self.cfg(**kw)
        info = (tmx_info * nrhs)()
        rc = self.check(lib.tmx_solve(self.h, _ptr(x), _ptr(b), nrhs, ctypes.byref(cfg), info), allow_noconv=True)
        return rc, [i.as_dict() for i in info]

    def solve_mhat(self, x, b, dagger=0, **kw):
        cfg = self.cfg(**kw)
        info = tmx_info()
        rc = self.check(lib.tmx_solve_mhat(self.h, _ptr(x), _ptr(b), int(dagger), ctypes.byref(cfg),
                                           ctypes.byref(info)), allow_noconv=True)
        return rc, info.as_dict()

    def multishift_solve(self, x, b, shifts, **kw):
        cfg = self.cfg(**kw)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        info = (tmx_info * len(sh))()
        rc = self.check(lib.tmx_multishift_solve(self.h, _ptr(x), _ptr(b), sh.ctypes.data, len(sh),
                                                 ctypes.byref(cfg), info), allow_noconv=True)
        return rc, [i.as_dict() for i in info]

    def hop_force(self, force, x, y, op=TMX_OP_PLUS, coeff=1.0, accumulate=0):
        """force (= or +=) coeff * TA link derivative of Re<y, Mhat(op) x> (hopping terms)."""
        self._check_force_sizes(force, x, y, 2 if op == TMX_OP_ND else 1)
        return self.check(lib.tmx_hop_force(self.h, _ptr(force), _ptr(x), _ptr(y), int(op), float(coeff),
                                            int(accumulate)))

    def clover_force(self, force, x, y, op=TMX_OP_PLUS, coeff=1.0, accumulate=0):
        """force (= or +=) coeff * TA link derivative of Re<y, Mhat(op) x> (clover term)."""
        self._check_force_sizes(force, x, y, 2 if op == TMX_OP_ND else 1)
        return self.check(lib.tmx_clover_force(self.h, _ptr(force), _ptr(x), _ptr(y), int(op), float(coeff),
                                               int(accumulate)))

    def _check_force_sizes(self, force, x, y, nf=1):
        # the library takes plain device pointers and writes V * 36 complex128
        # values through `force`: only contiguous complex128 device tensors of
        # at least the needed size are passed on
        check_device_complex128(force, self.V * 36, "force")
        check_device_complex128(x, self.Vh * 12 * nf, "x")
        if y is not None:
            check_device_complex128(y, self.Vh * 12 * nf, "y")

    def rational_force(self, force, phi, coeffs, shifts, accumulate=0, **kw):
        """force (= or +=) the link derivative of <phi, R(N) phi>, R = a0 + sum_k coeffs[k] (N + shifts[k])^{-1}."""
        cfg = self.cfg(**kw)
        self._check_force_sizes(force, phi, None, 2 if cfg.op == TMX_OP_ND else 1)
        a = np.ascontiguousarray(coeffs, dtype=np.float64)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        if a.shape != sh.shape:
            raise ValueError("coeffs and shifts differ in length")
        info = (tmx_info * len(sh))()
        rc = self.check(lib.tmx_rational_force(self.h, _ptr(force), _ptr(phi), a.ctypes.data, sh.ctypes.data,
                                               len(sh), ctypes.byref(cfg), int(accumulate), info), allow_noconv=True)
        return rc, [i.as_dict() for i in info]

    def rational_apply(self, out, b, a0, coeffs, shifts, **kw):
        """out = a0 b + sum_k coeffs[k] (N + shifts[k])^{-1} b (device odd fields)."""
        cfg = self.cfg(**kw)
        a = np.ascontiguousarray(coeffs, dtype=np.float64)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        if a.shape != sh.shape:
            raise ValueError("coeffs and shifts differ in length")
        info = (tmx_info * len(sh))()
        rc = self.check(lib.tmx_rational_apply(self.h, _ptr(out), _ptr(b), float(a0), a.ctypes.data, sh.ctypes.data,
                                               len(sh), ctypes.byref(cfg), info), allow_noconv=True)
        return rc, [i.as_dict() for i in info]

    def rational_correction(self, eta, a0, coeffs, shifts, series_tol=1e-12, maxterms=8, **kw):
        """E = sum_k binom(-1/2, k) <eta, Z^k eta>, Z = N R(N)^2 - 1; returns (rc, E, terms).
        series_tol stops the series; kw are the solver settings (tol, inner_prec, op, ...)."""
        cfg = self.cfg(**kw)
        a = np.ascontiguousarray(coeffs, dtype=np.float64)
        sh = np.ascontiguousarray(shifts, dtype=np.float64)
        if a.shape != sh.shape:
            raise ValueError("coeffs and shifts differ in length")
        e, n = ctypes.c_double(), ctypes.c_int()
        rc = self.check(lib.tmx_rational_correction(self.h, _ptr(eta), float(a0), a.ctypes.data, sh.ctypes.data,
                                                    len(sh), float(series_tol), int(maxterms), ctypes.byref(cfg),
                                                    ctypes.byref(e), ctypes.byref(n)), allow_noconv=True)
        return rc, e.value, n.value

    # -- learned preconditioner ---------------------------------------------
    def pc_num_params(self):
        n = ctypes.c_size_t()
        self.check(lib.tmx_pc_num_params(self.h, ctypes.byref(n)))
        return n.value

    def pc_set_weights(self, w: np.ndarray):
        w = np.ascontiguousarray(w, dtype=np.float32)
        return self.check(lib.tmx_pc_set_weights(self.h, w.ctypes.data, w.size))

    def pc_get_weights(self):
        w = np.empty(self.pc_num_params(), dtype=np.float32)
        self.check(lib.tmx_pc_get_weights(self.h, w.ctypes.data, w.size))
        return w

    def free_workspaces(self):
        """Give the context's scratch buffers back (tmx_free_workspaces)."""
        return self.check(lib.tmx_free_workspaces(self.h))

    def pc_apply(self, out, inp, dagger=0):
        return self.check(lib.tmx_pc_apply(self.h, _ptr(out), _ptr(inp), int(dagger)))

    def pc_adam_step(self, grad: np.ndarray, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        g = np.ascontiguousarray(grad, dtype=np.float32)
        cfg = tmx_train_cfg(1, 1, lr, beta1, beta2, eps, 0, 0, 0)
        return self.check(lib.tmx_pc_adam_step(self.h, g.ctypes.data, g.size, ctypes.byref(cfg)))

    def pc_train(self, b, x, npairs, epochs=10, batch=8, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, seed=0,
                 loss_kind=0, op=TMX_OP_PLUS):
        cfg = tmx_train_cfg(epochs, batch, lr, beta1, beta2, eps, seed, loss_kind, op)
        loss = np.zeros(epochs, dtype=np.float32)
        self.check(lib.tmx_pc_train(self.h, _ptr(b), _ptr(x), npairs, ctypes.byref(cfg), loss.ctypes.data))
        return loss

    # -- autotuner ------------------------------------------------------------
    def tune(self, prec, op, nrhs=1):
        return self.check(lib.tmx_tune(self.h, prec, op, nrhs))

    def tuned_config(self, key):
        b, x, s, g = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        rc = lib.tmx_tuned_config(self.h, key.encode(), ctypes.byref(b), ctypes.byref(x), ctypes.byref(s),
                                  ctypes.byref(g))
        return {"block": b.value, "xcd": x.value, "spt": s.value, "rg": g.value, "tuned": rc == TMX_OK}

    # -- kernel timing --------------------------------------------------------
    def kstats_enable(self, on=True):
        return self.check(lib.tmx_kstats_enable(self.h, int(on)))

    def kstats(self):
        """{kernel name: (launches, total ms)} recorded with HIP events."""
        out = {}
        i = 0
        buf = ctypes.create_string_buffer(128)
        while True:
            n = ctypes.c_long()
            ms = ctypes.c_double()
            if lib.tmx_kstats_get(self.h, i, buf, 128, ctypes.byref(n), ctypes.byref(ms)) != TMX_OK:
                break
            out[buf.value.decode()] = (n.value, ms.value)
            i += 1
        return out

    def pc_loss_grad(self, b, x, npairs, loss_kind=0, op=TMX_OP_PLUS):
        loss = ctypes.c_double()
        g = np.zeros(self.pc_num_params(), dtype=np.float32)
        self.check(lib.tmx_pc_loss_grad(self.h, _ptr(b), _ptr(x), npairs, loss_kind, op, ctypes.byref(loss),
                                        g.ctypes.data))
        return loss.value, g

    # -- tracing ----------------------------------------------------------------
    def trace_enable(self, on=True):
        return self.check(lib.tmx_trace_enable(self.h, int(on)))

    def trace_push(self, name):
        return self.check(lib.tmx_trace_push(self.h, name.encode()))

    def trace_pop(self):
        return self.check(lib.tmx_trace_pop(self.h))


def check_device_complex128(t, n, name):
    """Raise ValueError unless t is a contiguous complex128 CUDA tensor of at
    least n elements (16 n bytes): what a kernel writing through its pointer needs."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor on the GPU, not {type(t).__name__}")
    if t.dtype != torch.complex128:
        raise ValueError(f"{name} must be complex128, not {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.element_size() * t.numel() < 16 * n:
        raise ValueError(f"{name} holds {t.numel()} complex128 values, needs {n}")


def canonical_gauge_order(U: np.ndarray) -> np.ndarray:
    """Links as the C ABI takes them: [t][z][y][x][mu][3][3] complex128."""
    return np.ascontiguousarray(U, dtype=np.complex128)
