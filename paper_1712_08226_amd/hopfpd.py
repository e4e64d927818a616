"""Thin ctypes binding of libhopfpd.so (the C-ABI in include/hopfpd.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Host arrays are NumPy float64/int32; the ``*_dev`` calls take torch
CUDA tensors (torch is used for device memory and streams only).  Importing
this module fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhopfpd.so")

U_L2, U_BOX = 0, 1
Q_TRAP, Q_LEFT = 0, 1
FP64, FP32, BF16X3 = 0, 1, 2
WARM_COLD, WARM_CONT, WARM_MLP, WARM_MLP_LAM, WARM_MLP_FIRST = 0, 1, 2, 3, 4
ROOT_BISECT, ROOT_NEWTON = 0, 1
PT_OK, PT_INSIDE, PT_UNREACH, PT_NOCONV, PT_NONFINITE = 0, 1, 2, 3, 4

EXPORTS = ["hopf_default_opts", "hopf_create", "hopf_destroy", "hopf_strerror", "hopf_last_error",
           "hopf_set_systems", "hopf_set_opts", "hopf_value", "hopf_value_dev", "hopf_min_time", "hopf_min_time_dev",
           "hopf_min_time_dev_noalloc",
           "hopf_trajectory", "hopf_last_timing", "hopf_warm_init", "hopf_warm_params",
           "hopf_warm_loss_grad", "hopf_warm_train", "hopf_warm_save", "hopf_warm_load"]


class HopfSystem(C.Structure):
    _fields_ = [("n", C.c_int), ("m", C.c_int), ("N", C.c_int), ("t_max", C.c_double),
                ("quad", C.c_int), ("uset", C.c_int),
                ("A", C.POINTER(C.c_double)), ("B", C.POINTER(C.c_double)),
                ("Qu", C.POINTER(C.c_double)), ("W", C.POINTER(C.c_double)),
                ("c", C.POINTER(C.c_double)), ("c_tau", C.c_double)]


class HopfOpts(C.Structure):
    _fields_ = [("c_tau", C.c_double), ("gap_tol", C.c_double), ("t_rel_tol", C.c_double),
                ("t_abs_frac", C.c_double), ("max_iter", C.c_int), ("check_every", C.c_int),
                ("warm", C.c_int), ("prec", C.c_int), ("root", C.c_int), ("newton_after", C.c_int),
                ("newton_rho", C.c_double), ("tail_max", C.c_int), ("adapt", C.c_int), ("scan", C.c_int),
                ("wide_min", C.c_int), ("deep_max", C.c_int), ("structure", C.c_int)]


class HopfTiming(C.Structure):
    _fields_ = [("total_s", C.c_double), ("iter_kernel_s", C.c_double), ("iter_launches", C.c_long),
                ("iter_point_rows", C.c_double), ("alg_flops", C.c_double), ("tail_kernel_s", C.c_double),
                ("tail_point_rows", C.c_double), ("tail_points", C.c_long), ("wide_kernel_s", C.c_double),
                ("wide_launches", C.c_long), ("wide_point_rows", C.c_double)]


class HopfError(RuntimeError):
    pass


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library; raises if it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise HopfError(f"{path} is not built: run `python -m paper_1712_08226_amd.build`")
    # When PyTorch is installed its HIP runtime is loaded first, so the library
    # binds to the same runtime and the device-pointer calls can share torch's
    # tensors and streams; loaded the other way round, torch's own device
    # initialisation fails later in the process ("No HIP GPUs are available").
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.c_void_p
    lib.hopf_default_opts.argtypes = [C.POINTER(HopfOpts)]
    lib.hopf_create.argtypes = [C.c_int, C.POINTER(vp)]
    lib.hopf_destroy.argtypes = [vp]
    lib.hopf_destroy.restype = None
    lib.hopf_strerror.argtypes = [C.c_int]
    lib.hopf_strerror.restype = C.c_char_p
    lib.hopf_last_error.argtypes = [vp]
    lib.hopf_last_error.restype = C.c_char_p
    lib.hopf_set_systems.argtypes = [vp, C.c_int, C.POINTER(HopfSystem)]
    lib.hopf_set_opts.argtypes = [vp, C.POINTER(HopfOpts)]
    lib.hopf_value.argtypes = [vp, C.c_long, ip, dp, dp, dp, dp, dp, ip, ip]
    lib.hopf_min_time.argtypes = [vp, C.c_long, ip, dp, dp, dp, dp, dp, dp, ip, ip, ip]
    lib.hopf_min_time_dev.argtypes = [vp, C.c_long, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hopf_value_dev.argtypes = [vp, C.c_long, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hopf_min_time_dev_noalloc.argtypes = [vp, C.c_long, C.c_int, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.hopf_trajectory.argtypes = [vp, C.c_int, dp, C.c_double, ip, dp, dp, dp, dp, dp, dp]
    lib.hopf_last_timing.argtypes = [vp, C.POINTER(HopfTiming)]
    fp = C.POINTER(C.c_float)
    lib.hopf_warm_init.argtypes = [vp, C.c_int, C.c_uint]
    lib.hopf_warm_save.argtypes = [vp, C.c_int, C.c_char_p]
    lib.hopf_warm_load.argtypes = [vp, C.c_int, C.c_char_p]
    lib.hopf_warm_params.argtypes = [vp, C.c_int, C.c_int, fp, C.c_long, fp]
    lib.hopf_warm_loss_grad.argtypes = [vp, C.c_int, C.c_int, fp, fp, dp, fp]
    lib.hopf_warm_train.argtypes = [vp, C.c_int, C.c_long, dp, C.c_int, C.c_int, C.c_float, C.c_uint, dp,
                                    C.POINTER(C.c_long)]
    for name in EXPORTS:
        if name not in ("hopf_destroy", "hopf_strerror", "hopf_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def _iptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_int)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def default_opts() -> HopfOpts:
    o = HopfOpts()
    load().hopf_default_opts(C.byref(o))
    return o


class Solver:
    """Owns one hopf_ctx (one device, one stream)."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.hopf_create(device, C.byref(h))
        if st != 0:
            raise HopfError(f"hopf_create failed: {self.lib.hopf_strerror(st).decode()}")
        self.h = h
        self._keep = []

    def close(self):
        if self.h:
            self.lib.hopf_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, what):
        if st != 0:
            msg = self.lib.hopf_last_error(self.h).decode()
            raise HopfError(f"{what}: {self.lib.hopf_strerror(st).decode()}: {msg}")

    # -------------------------------------------------------------- setup
    def set_systems(self, systems):
        """systems: iterable of objects/dicts with A, B, W, c, uset, N, t_max,
        quad (and optionally Qu and c_tau, the system's step ratio); uset
        'l2'/'box', quad 'trap'/'left'."""
        arr = (HopfSystem * len(systems))()
        keep = []
        for k, s in enumerate(systems):
            g = (lambda key, d=None: s.get(key, d) if isinstance(s, dict) else getattr(s, key, d))
            A, B, W = _f64(g("A")), _f64(g("B")), _f64(g("W"))
            if B.ndim == 1:
                B = B[:, None].copy()
            c = g("c", None)
            c = _f64(c) if c is not None else None
            Qu = g("Qu", None)
            Qu = _f64(Qu) if Qu is not None else None
            keep += [A, B, W, c, Qu]
            uset = g("uset")
            quad = g("quad")
            arr[k] = HopfSystem(A.shape[0], B.shape[1], int(g("N")), float(g("t_max")),
                                Q_TRAP if quad in ("trap", Q_TRAP) else Q_LEFT,
                                U_L2 if uset in ("l2", U_L2) else U_BOX,
                                _dptr(A), _dptr(B), _dptr(Qu), _dptr(W), _dptr(c), float(g("c_tau", 0.0) or 0.0))
        self._check(self.lib.hopf_set_systems(self.h, len(systems), arr), "hopf_set_systems")
        self.n = [int(arr[k].n) for k in range(len(systems))]
        self.m = [int(arr[k].m) for k in range(len(systems))]
        self.N = [int(arr[k].N) for k in range(len(systems))]

    def set_opts(self, **kw):
        o = default_opts()
        names = {f[0] for f in HopfOpts._fields_}
        for k, v in kw.items():
            if k not in names:
                raise TypeError(f"unknown solver option {k!r}")
            if k == "prec":
                v = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}.get(v, v)
            if k == "warm":
                v = {"cold": WARM_COLD, "cont": WARM_CONT, "mlp": WARM_MLP, "mlp_lam": WARM_MLP_LAM,
                     "mlp_first": WARM_MLP_FIRST}.get(v, v)
            if k == "root":
                v = {"bisect": ROOT_BISECT, "newton": ROOT_NEWTON}.get(v, v)
            setattr(o, k, v)
        self._check(self.lib.hopf_set_opts(self.h, C.byref(o)), "hopf_set_opts")

    # -------------------------------------------------------------- solves
    def _stride(self, sid):
        """Row width of x and lam: the largest n among the systems used."""
        if sid is None or len(sid) == 0:
            return self.n[0]
        return max(self.n[int(k)] for k in np.unique(sid) if 0 <= int(k) < len(self.n))

    def value(self, x, t, sys_id=None):
        x = _f64(x)
        npts, n = x.shape
        t = _f64(np.broadcast_to(np.asarray(t, dtype=np.float64), (npts,)))
        sid = None if sys_id is None else np.ascontiguousarray(np.asarray(sys_id, dtype=np.int32))
        if npts and n != self._stride(sid):
            raise ValueError(f"x must have {self._stride(sid)} columns (the largest n of the systems used)")
        lo, hi = np.empty(npts), np.empty(npts)
        lam = np.empty((npts, n))
        iters = np.empty(npts, dtype=np.int32)
        stat = np.empty(npts, dtype=np.int32)
        self._check(self.lib.hopf_value(self.h, npts, _iptr(sid), _dptr(x), _dptr(t), _dptr(lo), _dptr(hi),
                                        _dptr(lam), _iptr(iters), _iptr(stat)), "hopf_value")
        return dict(phi_lo=lo, phi_hi=hi, lam=lam, iters=iters, status=stat)

    def value_at_horizon(self, system, x, t):
        """Value solves of many points at one shared horizon t in the paper's
        per-horizon layout (Sec. III-A: the N nodes spread over [0, t]): the
        system's node table is rebuilt over [0, t], which replaces the
        context's systems, and every point is solved at t = t_max of that
        table.  Level sets on a grid at a few horizons (Sec. VI-A) are the
        intended use; for per-point horizons use value()."""
        g = (lambda key, d=None: system.get(key, d) if isinstance(system, dict) else getattr(system, key, d))
        sysd = {k: g(k) for k in ("A", "B", "W", "c", "Qu", "uset", "N", "quad", "c_tau")}
        sysd["t_max"] = float(t)
        self.set_systems([sysd])
        x = _f64(x)
        return self.value(x, np.full(x.shape[0], float(t)))

    def min_time(self, x, sys_id=None, lam0=None, t_bracket=None):
        """lam0: optional (npts, n_max) starting costates of the first probes;
        t_bracket: optional (npts, 2) probe hints (a, b) inside the first cell."""
        x = _f64(x)
        npts, n = x.shape
        sid = None if sys_id is None else np.ascontiguousarray(np.asarray(sys_id, dtype=np.int32))
        if npts and n != self._stride(sid):
            raise ValueError(f"x must have {self._stride(sid)} columns (the largest n of the systems used)")
        if lam0 is not None:
            lam0 = _f64(lam0)
            if lam0.shape != (npts, n):
                raise ValueError(f"lam0 must have shape {(npts, n)}")
        if t_bracket is not None:
            t_bracket = _f64(t_bracket)
            if t_bracket.shape != (npts, 2):
                raise ValueError(f"t_bracket must have shape {(npts, 2)}")
        T, gap = np.empty(npts), np.empty(npts)
        lam = np.empty((npts, n))
        probes = np.empty(npts, dtype=np.int32)
        iters = np.empty(npts, dtype=np.int32)
        stat = np.empty(npts, dtype=np.int32)
        self._check(self.lib.hopf_min_time(self.h, npts, _iptr(sid), _dptr(x), _dptr(lam0), _dptr(t_bracket),
                                           _dptr(T), _dptr(gap), _dptr(lam), _iptr(probes), _iptr(iters),
                                           _iptr(stat)), "hopf_min_time")
        return dict(T=T, gap=gap, lam=lam, probes=probes, iters=iters, status=stat)

    def _dev_ptr(self, t, name, dtype, rows, cols=None):
        """Pointer of a device tensor after checking what the library will
        assume of it (device, dtype, contiguity, at least rows x cols items),
        so that a mismatched tensor fails here instead of on the device."""
        if t is None:
            return None
        if not (getattr(t, "is_cuda", False) and str(t.dtype) == dtype and t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")
        need = rows * (cols or 1)
        if t.numel() < need or (cols is not None and (t.dim() != 2 or t.shape[1] != cols)):
            raise ValueError(f"{name} must hold {rows} rows" + (f" of {cols} entries" if cols else ""))
        return C.c_void_p(t.data_ptr())

    def _dev_common(self, x, sys_id, stream):
        if x.dim() != 2:
            raise ValueError("x must be 2-D (points x n_max)")
        npts, n = x.shape
        if npts and n != self._stride(None if sys_id is None else sys_id.cpu().numpy()):
            raise ValueError("x must have as many columns as the largest n of the systems used")
        s = C.c_void_p(stream.cuda_stream) if stream is not None else None
        return npts, n, s

    def min_time_dev(self, x, T, gap, status, lam=None, probes=None, iters=None, sys_id=None, stream=None,
                     lam0=None, t_bracket=None):
        """Device twin: torch CUDA tensors (float64 x/T/gap/lam/lam0/t_bracket,
        int32 others)."""
        npts, n, s = self._dev_common(x, sys_id, stream)
        d = self._dev_ptr
        self._check(self.lib.hopf_min_time_dev(
            self.h, npts, d(sys_id, "sys_id", "torch.int32", npts), d(x, "x", "torch.float64", npts, n),
            d(lam0, "lam0", "torch.float64", npts, n), d(t_bracket, "t_bracket", "torch.float64", npts, 2),
            d(T, "T", "torch.float64", npts), d(gap, "gap", "torch.float64", npts),
            d(lam, "lam", "torch.float64", npts, n), d(probes, "probes", "torch.int32", npts),
            d(iters, "iters", "torch.int32", npts), d(status, "status", "torch.int32", npts), s),
            "hopf_min_time_dev")

    def min_time_dev_noalloc(self, x, T, gap, status, lam=None, probes=None, iters=None, sys=0, stream=None,
                             lam0=None, t_bracket=None):
        """min_time_dev for the points of one system with the solver state in
        the library's fixed device scratch (no allocation in the call)."""
        if x.dim() != 2:
            raise ValueError("x must be 2-D (points x n)")
        npts, n = x.shape
        if npts and n != self.n[sys]:
            raise ValueError(f"x must have {self.n[sys]} columns")
        s = C.c_void_p(stream.cuda_stream) if stream is not None else None
        d = self._dev_ptr
        self._check(self.lib.hopf_min_time_dev_noalloc(
            self.h, npts, int(sys), d(x, "x", "torch.float64", npts, n),
            d(lam0, "lam0", "torch.float64", npts, n), d(t_bracket, "t_bracket", "torch.float64", npts, 2),
            d(T, "T", "torch.float64", npts), d(gap, "gap", "torch.float64", npts),
            d(lam, "lam", "torch.float64", npts, n), d(probes, "probes", "torch.int32", npts),
            d(iters, "iters", "torch.int32", npts), d(status, "status", "torch.int32", npts), s),
            "hopf_min_time_dev_noalloc")

    def value_dev(self, x, t, phi_lo, phi_hi, status, lam=None, iters=None, sys_id=None, stream=None):
        """Device twin of value(): torch CUDA tensors (float64 x/t/phi/lam,
        int32 others); results are in place when the call returns."""
        npts, n, s = self._dev_common(x, sys_id, stream)
        d = self._dev_ptr
        self._check(self.lib.hopf_value_dev(
            self.h, npts, d(sys_id, "sys_id", "torch.int32", npts), d(x, "x", "torch.float64", npts, n),
            d(t, "t", "torch.float64", npts), d(phi_lo, "phi_lo", "torch.float64", npts),
            d(phi_hi, "phi_hi", "torch.float64", npts), d(lam, "lam", "torch.float64", npts, n),
            d(iters, "iters", "torch.int32", npts), d(status, "status", "torch.int32", npts), s),
            "hopf_value_dev")

    def trajectory(self, x0, T, sys_id=0):
        """Control u(s) and state x(s) at the quadrature nodes (rows sorted by
        physical time s) and the costate p* = e^{T A^T} lam*."""
        x0 = _f64(x0)
        n = x0.shape[0]
        rows = self.N[sys_id] + 1
        m = self.m[sys_id]
        nn = C.c_int(0)
        s = np.empty(rows)
        u = np.empty((rows, m))
        xs = np.empty((rows, n))
        p = np.empty(n)
        lo, hi = C.c_double(0), C.c_double(0)
        self._check(self.lib.hopf_trajectory(self.h, sys_id, _dptr(x0), float(T), C.byref(nn), _dptr(s), _dptr(u),
                                             _dptr(xs), _dptr(p), C.byref(lo), C.byref(hi)), "hopf_trajectory")
        k = nn.value
        return dict(s=s[:k], u=u[:k], xs=xs[:k], p_star=p, phi_lo=lo.value, phi_hi=hi.value)

    # -------------------------------------------------------------- learned warm start
    def warm_nparams(self, sys_id=0, H=256):
        n = self.n[sys_id]
        return (n + 1) * H + H + 2 * (H * H + H) + H * (n + 2) + (n + 2)

    def warm_init(self, sys_id=0, seed=0):
        self._check(self.lib.hopf_warm_init(self.h, sys_id, seed), "hopf_warm_init")

    def warm_get(self, sys_id=0):
        """Returns (theta, norm) with norm = [x_mean, x_std, t_scale, lam_scale]."""
        th = np.empty(self.warm_nparams(sys_id), dtype=np.float32)
        norm = np.empty(2 * self.n[sys_id] + 2, dtype=np.float32)
        self._check(self.lib.hopf_warm_params(self.h, sys_id, 0, th.ctypes.data_as(C.POINTER(C.c_float)), th.size,
                                              norm.ctypes.data_as(C.POINTER(C.c_float))), "hopf_warm_params")
        return th, norm

    def warm_set(self, theta, norm=None, sys_id=0):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        self._check(self.lib.hopf_warm_params(self.h, sys_id, 1, th.ctypes.data_as(C.POINTER(C.c_float)), th.size,
                                              None if nm is None else nm.ctypes.data_as(C.POINTER(C.c_float))),
                    "hopf_warm_params")

    def warm_save(self, path, sys_id=0):
        """Write the trained network of sys_id to a checkpoint file
        (hopf_warm_save; format in include/hopfpd.h)."""
        self._check(self.lib.hopf_warm_save(self.h, sys_id, os.fsencode(path)), "hopf_warm_save")

    def warm_load(self, path, sys_id=0):
        """Read a checkpoint written by warm_save into sys_id (hopf_warm_load)."""
        self._check(self.lib.hopf_warm_load(self.h, sys_id, os.fsencode(path)), "hopf_warm_load")

    def warm_loss_grad(self, Z, Y, sys_id=0):
        Z = np.ascontiguousarray(Z, dtype=np.float32)
        Y = np.ascontiguousarray(Y, dtype=np.float32)
        g = np.empty(self.warm_nparams(sys_id), dtype=np.float32)
        loss = C.c_double()
        fp = C.POINTER(C.c_float)
        self._check(self.lib.hopf_warm_loss_grad(self.h, sys_id, Z.shape[0], Z.ctypes.data_as(fp),
                                                 Y.ctypes.data_as(fp), C.byref(loss), g.ctypes.data_as(fp)),
                    "hopf_warm_loss_grad")
        return loss.value, g

    def warm_train(self, x, epochs=20, batch=4096, lr=1e-3, seed=0, sys_id=0):
        x = _f64(x)
        el = np.zeros(max(epochs, 1))
        pairs = C.c_long()
        self._check(self.lib.hopf_warm_train(self.h, sys_id, x.shape[0], _dptr(x), epochs, batch, lr, seed,
                                             _dptr(el), C.byref(pairs)), "hopf_warm_train")
        return dict(epoch_loss=el[:epochs], pairs=pairs.value)

    def last_timing(self):
        t = HopfTiming()
        self._check(self.lib.hopf_last_timing(self.h, C.byref(t)), "hopf_last_timing")
        return dict(total_s=t.total_s, iter_kernel_s=t.iter_kernel_s, iter_launches=t.iter_launches,
                    point_rows=t.iter_point_rows, alg_flops=t.alg_flops, tail_kernel_s=t.tail_kernel_s,
                    tail_point_rows=t.tail_point_rows, tail_points=t.tail_points, wide_kernel_s=t.wide_kernel_s,
                    wide_launches=t.wide_launches, wide_point_rows=t.wide_point_rows)
