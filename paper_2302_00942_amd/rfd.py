"""Python binding of librfd.so (the C ABI declared in include/rfd.h).

Argument marshalling only: every step of the integrator runs in the HIP
kernels of the library. torch supplies device memory and streams. Loading
fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librfd.so")

OK, INVALID_ARG, RANGE, OUT_OF_BUDGET, NONFINITE, DEVICE, NOT_READY, SHUTDOWN = range(8)
BALL_L2, BOX_LINF = 0, 1
FP32, BF16 = 0, 1
_PREC = {"fp32": FP32, "bf16": BF16, FP32: FP32, BF16: BF16}
_SHAPE = {"ball": BALL_L2, "box": BOX_LINF, BALL_L2: BALL_L2, BOX_LINF: BOX_LINF}


class RfdError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {status_string(status)} ({status})")


class Params(C.Structure):
    _fields_ = [("m", C.c_int32), ("shape", C.c_int32), ("precision", C.c_int32), ("dim", C.c_int32),
                ("eps", C.c_double), ("lam", C.c_double), ("sigma", C.c_double), ("radius", C.c_double),
                ("seed", C.c_uint64), ("omega", C.POINTER(C.c_float))]


class Request(C.Structure):
    _fields_ = [("X", C.c_void_p), ("N", C.c_int64), ("F", C.c_void_p), ("ldF", C.c_int64), ("d", C.c_int32),
                ("reserved", C.c_int32), ("out", C.c_void_p), ("ldO", C.c_int64), ("params", Params),
                ("cloud_key", C.c_uint64)]


class Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("reserved", C.c_int32), ("t_submit", C.c_double), ("t_start", C.c_double),
                ("t_done", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    """The loaded librfd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2302_00942_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double
        sigs = {
            "rfd_status_string": ([i32], C.c_char_p),
            "rfd_plan_create": ([C.POINTER(Params), C.POINTER(vp)], i32),
            "rfd_params_frequencies": ([C.POINTER(Params), vp, vp], i32),
            "rfd_plan_export": ([vp, vp, vp], i32),
            "rfd_features": ([vp, vp, i64, vp], i32),
            "rfd_integrate": ([vp, vp, i64, i32, vp, i64, vp], i32),
            "rfd_integrate_scaled": ([vp, vp, i64, i32, vp, i64, vp, vp], i32),
            "rfd_integrate_oneshot": ([vp, vp, i64, vp, i64, i32, vp, i64, vp], i32),
            "rfd_loop_create": ([vp, vp, i32, vp, i64, i32, i32, C.POINTER(vp)], i32),
            "rfd_loop_launch": ([vp, vp], i32),
            "rfd_loop_destroy": ([vp], None),
            "rfd_plan_spectrum": ([vp, i32, i64, vp, vp], i32),
            "rfd_spectrum_batch": ([vp, i32, i32, i64, vp, vp], i32),
            "rfd_gw_create": ([vp, vp, C.POINTER(vp)], i32),
            "rfd_gw_loss": ([vp, vp, i64, vp, i64, vp], i32),
            "rfd_gw_terms": ([vp, vp, i64, vp, vp, vp, i64, vp], i32),
            "rfd_gw_destroy": ([vp], None),
            "rfd_plan_check": ([vp, vp], i32),
            "rfd_plan_core": ([vp, vp, vp, vp, vp], i32),
            "rfd_plan_info": ([vp, vp, vp, vp], i32),
            "rfd_features_sync": ([vp, vp, i64, vp], i32),
            "rfd_plan_workspace_size": ([vp, i64, i32, vp], i32),
            "rfd_plan_create_in": ([vp, vp, C.c_size_t, i64, i32, C.POINTER(vp)], i32),
            "rfd_bary_create": ([vp, vp, vp, i64, i32, vp, i32, dbl, vp, C.POINTER(vp)], i32),
            "rfd_bary_launch": ([vp, vp], i32),
            "rfd_bary_floored": ([vp, vp, vp], i32),
            "rfd_bary_destroy": ([vp], None),
            "rfd_integrate_oneshot_noalloc": ([vp, vp, i64, vp, i64, i32, vp, i64, vp], i32),
            "rfd_plan_action": ([vp, vp, vp, vp, vp], i32),
            "rfd_plan_destroy": ([vp], None),
            "rfd_integrate_batch": ([vp, vp, vp, vp, vp, vp, vp, vp, i32, vp], i32),
            "rfd_batch_create": ([vp, vp, vp, vp, vp, vp, vp, vp, i32, C.POINTER(vp)], i32),
            "rfd_batch_launch": ([vp, vp], i32),
            "rfd_batch_destroy": ([vp], None),
            "rfd_batch_tune": ([vp, i32, vp], i32),
            "rfd_batch_tiles_per_item": ([vp], i32),
            "rfd_autotune": ([vp, vp, i64, i32, vp, i64, i32, vp], i32),
            "rfd_autotune_phi1": ([vp, i32, vp], i32),
            "rfd_tune_export": ([vp, i32], i32),
            "rfd_tune_import": ([C.c_char_p], i32),
            "rfd_tune_reset": ([], None),
            "rfd_server_create": ([C.c_size_t, i32, C.POINTER(vp)], i32),
            "rfd_submit": ([vp, C.POINTER(Request), C.POINTER(u64)], i32),
            "rfd_wait": ([vp, u64, dbl, C.POINTER(Result)], i32),
            "rfd_server_stats": ([vp, vp, vp, vp, vp], i32),
            "rfd_server_destroy": ([vp], None),
            "rfd_profile_enable": ([C.c_int], None),
            "rfd_profile_read": ([vp, vp, i32, i32], i32),
            "rfd_profile_kernel_name": ([i32], C.c_char_p),
            "rfd_library_release": ([], None),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().rfd_status_string(int(s)).decode()


def _check(s: int, what: str) -> None:
    if s != OK:
        raise RfdError(s, what)


def make_params(m: int, eps: float, lam: float, seed: int = 0, shape="ball", precision="fp32",
                sigma: float = 0.0, radius: float = 0.0, omega: Optional[np.ndarray] = None, dim: int = 3):
    p = Params()
    p.m, p.shape, p.precision, p.dim = int(m), _SHAPE[shape], _PREC[precision], int(dim)
    p.eps, p.lam, p.sigma, p.radius, p.seed = float(eps), float(lam), float(sigma), float(radius), int(seed)
    keep = None
    if omega is not None:
        keep = np.ascontiguousarray(omega, dtype=np.float32)
        p.omega = keep.ctypes.data_as(C.POINTER(C.c_float))
    else:
        p.omega = None
    return p, keep


def workspace_size(m: int, eps: float, N_max: int, d_max: int, seed: int = 0, shape="ball", precision="fp32",
                   sigma: float = 0.0, radius: float = 0.0, dim: int = 3) -> int:
    """Device bytes of a plan in a caller's arena (rfd_plan_workspace_size; host only)."""
    p, _ = make_params(m, eps, 0.0, seed, shape, precision, sigma, radius, dim=dim)
    n = C.c_size_t()
    _check(lib().rfd_plan_workspace_size(C.byref(p), int(N_max), int(d_max), C.byref(n)), "rfd_plan_workspace_size")
    return int(n.value)


def frequencies(m: int, eps: float, seed: int = 0, shape="ball", sigma: float = 0.0, radius: float = 0.0,
                dim: int = 3):
    """(omega f x D float32, w f float64) as the library samples them (host only)."""
    p, _ = make_params(m, eps, 0.0, seed, shape, "fp32", sigma, radius, dim=dim)
    f = m // 2
    om = np.zeros((f, dim if dim else 3), dtype=np.float32)
    w = np.zeros(f, dtype=np.float64)
    _check(lib().rfd_params_frequencies(C.byref(p), om.ctypes.data, w.ctypes.data), "rfd_params_frequencies")
    return om, w


def _stream_handle(stream) -> int:
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


def _dev_f32(t, what: str, cols: Optional[int] = None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32:
        raise TypeError(f"{what} must be a float32 CUDA tensor")
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError(f"{what} must be 2-D with unit column stride")
    if cols is not None and t.shape[1] != cols:
        raise ValueError(f"{what} must have {cols} columns")
    return t


class Plan:
    """An RFD plan: frequencies, weights and (after features) the m x m core."""

    def __init__(self, m: int, eps: float, lam: float, seed: int = 0, shape="ball", precision="fp32",
                 sigma: float = 0.0, radius: float = 0.0, omega: Optional[np.ndarray] = None, dim: int = 3):
        p, keep = make_params(m, eps, lam, seed, shape, precision, sigma, radius, omega, dim)
        h = C.c_void_p()
        _check(lib().rfd_plan_create(C.byref(p), C.byref(h)), "rfd_plan_create")
        self._h = h
        self.m, self.eps, self.lam, self.seed = m, eps, lam, seed
        self.dim = int(dim) if dim else 3
        self.precision = _PREC[precision]

    @classmethod
    def in_arena(cls, m: int, eps: float, lam: float, N_max: int, d_max: int, seed: int = 0, shape="ball",
                 precision="fp32", sigma: float = 0.0, radius: float = 0.0, omega: Optional[np.ndarray] = None):
        """A plan whose device memory is one torch tensor (rfd_plan_create_in),
        sized for clouds of up to N_max points and fields of up to d_max channels."""
        import torch
        p, keep = make_params(m, eps, lam, seed, shape, precision, sigma, radius, omega)
        nbytes = workspace_size(m, eps, N_max, d_max, seed, shape, precision, sigma, radius)
        arena = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = (arena.data_ptr() + 255) & ~255
        self = cls.__new__(cls)
        h = C.c_void_p()
        _check(lib().rfd_plan_create_in(C.byref(p), base, nbytes, int(N_max), int(d_max), C.byref(h)),
               "rfd_plan_create_in")
        self._h = h
        self._arena = arena
        self.m, self.eps, self.lam, self.seed = m, eps, lam, seed
        self.dim = 3
        self.precision = _PREC[precision]
        return self

    @property
    def handle(self) -> C.c_void_p:
        return self._h

    def export(self):
        f = self.m // 2
        om = np.zeros((f, self.dim), dtype=np.float32)
        w = np.zeros(f, dtype=np.float64)
        _check(lib().rfd_plan_export(self._h, om.ctypes.data, w.ctypes.data), "rfd_plan_export")
        return om, w

    def features(self, X, stream=None, sync: bool = False) -> None:
        """rfd_features (async), or with sync=True rfd_features_sync: waits and
        raises on what the device found (non-finite points or core)."""
        X = _dev_f32(X, "X", self.dim)
        if X.stride(0) != self.dim:
            raise ValueError(f"X must be contiguous N x {self.dim}")
        fn = lib().rfd_features_sync if sync else lib().rfd_features
        _check(fn(self._h, X.data_ptr(), X.shape[0], _stream_handle(stream)),
               "rfd_features_sync" if sync else "rfd_features")

    @property
    def points(self) -> int:
        """The plan's cloud size as the library holds it (-1 before any features)."""
        n = C.c_int64()
        _check(lib().rfd_plan_info(self._h, C.byref(n), None, None), "rfd_plan_info")
        return int(n.value)

    def _rows(self, F, out) -> None:
        # the library reads and writes N rows of F and out: shorter tensors
        # would be accessed out of bounds, so refuse them before any launch
        n = self.points
        if n >= 0 and F.shape[0] != n:
            raise ValueError(f"F has {F.shape[0]} rows; the plan's cloud has {n} points")
        if out.shape[0] != F.shape[0]:
            raise ValueError("out must have as many rows as F")

    def integrate(self, F, out=None, stream=None):
        import torch
        F = _dev_f32(F, "F")
        if out is None:
            out = torch.empty_like(F)
        out = _dev_f32(out, "out", F.shape[1])
        self._rows(F, out)
        _check(lib().rfd_integrate(self._h, F.data_ptr(), F.stride(0), F.shape[1], out.data_ptr(), out.stride(0),
                                   _stream_handle(stream)), "rfd_integrate")
        return out

    def integrate_scaled(self, F, scale, out=None, stream=None):
        """out = diag(scale) (F + A S B^T F); scale a float32 CUDA vector of N entries or None."""
        import torch
        F = _dev_f32(F, "F")
        if out is None:
            out = torch.empty_like(F)
        out = _dev_f32(out, "out", F.shape[1])
        self._rows(F, out)
        sp = 0
        if scale is not None:
            if not (isinstance(scale, torch.Tensor) and scale.is_cuda and scale.dtype == torch.float32
                    and scale.is_contiguous() and scale.numel() == F.shape[0]):
                raise ValueError("scale must be a contiguous float32 CUDA vector with one entry per row")
            sp = scale.data_ptr()
        _check(lib().rfd_integrate_scaled(self._h, F.data_ptr(), F.stride(0), F.shape[1], out.data_ptr(),
                                          out.stride(0), sp or None, _stream_handle(stream)), "rfd_integrate_scaled")
        return out

    def oneshot(self, X, F, out=None, stream=None):
        import torch
        X = _dev_f32(X, "X", 3)
        if X.stride(0) != 3:
            raise ValueError("X must be contiguous N x 3")
        F = _dev_f32(F, "F")
        if F.shape[0] != X.shape[0]:
            raise ValueError("X and F must have the same number of rows")
        if out is None:
            out = torch.empty_like(F)
        out = _dev_f32(out, "out", F.shape[1])
        if out.shape[0] != F.shape[0]:
            raise ValueError("out must have as many rows as F")
        _check(lib().rfd_integrate_oneshot(self._h, X.data_ptr(), X.shape[0], F.data_ptr(), F.stride(0), F.shape[1],
                                           out.data_ptr(), out.stride(0), _stream_handle(stream)),
               "rfd_integrate_oneshot")
        return out

    def oneshot_noalloc(self, X, F, out=None, stream=None):
        """rfd_integrate_oneshot_noalloc: the one-shot integration with no device
        allocation by the library (its buffers live in a fixed device array)."""
        import torch
        X = _dev_f32(X, "X", 3)
        if X.stride(0) != 3:
            raise ValueError("X must be contiguous N x 3")
        F = _dev_f32(F, "F")
        if F.shape[0] != X.shape[0]:
            raise ValueError("X and F must have the same number of rows")
        if out is None:
            out = torch.empty_like(F)
        out = _dev_f32(out, "out", F.shape[1])
        if out.shape[0] != F.shape[0]:
            raise ValueError("out must have as many rows as F")
        _check(lib().rfd_integrate_oneshot_noalloc(self._h, X.data_ptr(), X.shape[0], F.data_ptr(), F.stride(0),
                                                   F.shape[1], out.data_ptr(), out.stride(0), _stream_handle(stream)),
               "rfd_integrate_oneshot_noalloc")
        return out

    def autotune(self, F, out, reps: int = 10, stream=None):
        """Tunes the expansion geometry for this cloud and F's width; out gets integrate(F)."""
        F = _dev_f32(F, "F")
        out = _dev_f32(out, "out", F.shape[1])
        self._rows(F, out)
        _check(lib().rfd_autotune(self._h, F.data_ptr(), F.stride(0), F.shape[1], out.data_ptr(), out.stride(0),
                                  int(reps), _stream_handle(stream)), "rfd_autotune")
        return out

    def autotune_phi1(self, reps: int = 5, stream=None) -> None:
        """Tunes the workgroup count of the phi_1 kernel (needs features)."""
        _check(lib().rfd_autotune_phi1(self._h, int(reps), _stream_handle(stream)), "rfd_autotune_phi1")

    def spectrum(self, k: int, which: str = "smallest", stream=None):
        """The k smallest (ascending) or largest (descending) eigenvalues of
        exp(lambda A B^T) on the plan's cloud (rfd_plan_spectrum), float64 CUDA."""
        import torch
        w = {"smallest": 0, "largest": 1}[which]
        out = torch.empty(max(int(k), 1), dtype=torch.float64, device="cuda")
        _check(lib().rfd_plan_spectrum(self._h, w, int(k), out.data_ptr(), _stream_handle(stream)),
               "rfd_plan_spectrum")
        return out[: int(k)]

    def check(self, stream=None) -> int:
        """Synchronises and returns the device status code (OK, NONFINITE, RANGE, DEVICE)."""
        return int(lib().rfd_plan_check(self._h, _stream_handle(stream)))

    def core(self, stream=None):
        """(M, S, s): M = B^T A and S = lambda phi_1(lambda M), FP64 m x m, and the scaling power."""
        M = np.zeros((self.m, self.m))
        S = np.zeros((self.m, self.m))
        s = C.c_int32()
        _check(lib().rfd_plan_core(self._h, M.ctypes.data, S.ctypes.data, C.byref(s), _stream_handle(stream)),
               "rfd_plan_core")
        return M, S, int(s.value)

    def action(self, stream=None):
        """(H, G): the FP64 field block H = B^T F (m x d) and G = lambda phi_1(lambda M) H
        of the last call whose phi_1 ran in action form (rfd_plan_action)."""
        d = C.c_int32()
        _check(lib().rfd_plan_action(self._h, None, None, C.byref(d), _stream_handle(stream)), "rfd_plan_action")
        H = np.zeros((self.m, d.value))
        G = np.zeros((self.m, d.value))
        _check(lib().rfd_plan_action(self._h, H.ctypes.data, G.ctypes.data, None, _stream_handle(stream)),
               "rfd_plan_action")
        return H, G

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rfd_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many one-shot integrations in one launch per stage (rfd_batch_*).

    plans, Xs, Fs, outs: equal-length lists; every X (N x 3), F (N x d) and
    out (N x d) a float32 CUDA tensor that stays alive with the batch."""

    def __init__(self, plans, Xs, Fs, outs):
        n = len(plans)
        if not (len(Xs) == len(Fs) == len(outs) == n) or n == 0:
            raise ValueError("plans, Xs, Fs and outs must have the same non-zero length")
        for X, F, o in zip(Xs, Fs, outs):
            _dev_f32(X, "X", 3)
            _dev_f32(F, "F")
            _dev_f32(o, "out", F.shape[1])
            if X.shape[0] != F.shape[0] or X.stride(0) != 3:
                raise ValueError("X must be contiguous N x 3 with N = F.shape[0]")
            if o.shape[0] != F.shape[0]:
                raise ValueError("each out must have as many rows as its F")
        self._keep = (plans, Xs, Fs, outs)
        P = C.c_void_p * n
        self._arrs = dict(
            plans=P(*[p.handle.value for p in plans]), Xs=P(*[X.data_ptr() for X in Xs]),
            Ns=(C.c_int64 * n)(*[X.shape[0] for X in Xs]), Fs=P(*[F.data_ptr() for F in Fs]),
            ldFs=(C.c_int64 * n)(*[F.stride(0) for F in Fs]), ds=(C.c_int32 * n)(*[F.shape[1] for F in Fs]),
            outs=P(*[o.data_ptr() for o in outs]), ldOs=(C.c_int64 * n)(*[o.stride(0) for o in outs]))
        a = self._arrs
        h = C.c_void_p()
        _check(lib().rfd_batch_create(a["plans"], a["Xs"], a["Ns"], a["Fs"], a["ldFs"], a["ds"], a["outs"], a["ldOs"],
                                      n, C.byref(h)), "rfd_batch_create")
        self._h = h

    def launch(self, stream=None) -> None:
        _check(lib().rfd_batch_launch(self._h, _stream_handle(stream)), "rfd_batch_launch")

    def tune(self, reps: int = 5, stream=None) -> int:
        """Autotunes the expansion tiles per workgroup; returns the chosen value."""
        _check(lib().rfd_batch_tune(self._h, int(reps), _stream_handle(stream)), "rfd_batch_tune")
        return int(lib().rfd_batch_tiles_per_item(self._h))

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rfd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Loop:
    """`iterations` in-place steps v <- diag(s_k) exp(lambda_k A_k B_k^T) v,
    k = t mod len(plans) (rfd_loop_*). Every plan has its features computed on
    a cloud of v.shape[0] points; scales holds float32 CUDA vectors or None."""

    def __init__(self, plans, scales, v, iterations: int):
        import torch
        _dev_f32(v, "v")
        n = len(plans)
        if scales is None:
            scales = [None] * n
        if len(scales) != n or n == 0:
            raise ValueError("one scale (or None) per plan")
        for s in scales:
            if s is not None and not (isinstance(s, torch.Tensor) and s.is_cuda and s.dtype == torch.float32
                                      and s.is_contiguous() and s.numel() == v.shape[0]):
                raise ValueError("each scale must be a contiguous float32 CUDA vector with one entry per row")
        for p in plans:
            if p.points >= 0 and p.points != v.shape[0]:
                raise ValueError(f"v has {v.shape[0]} rows; a plan's cloud has {p.points} points")
        self._keep = (plans, scales, v)
        P = C.c_void_p * n
        self._plans = P(*[p.handle.value for p in plans])
        self._scales = P(*[(s.data_ptr() if s is not None else None) for s in scales])
        h = C.c_void_p()
        _check(lib().rfd_loop_create(self._plans, self._scales, n, v.data_ptr(), v.stride(0), v.shape[1],
                                     int(iterations), C.byref(h)), "rfd_loop_create")
        self._h = h

    def launch(self, stream=None) -> None:
        _check(lib().rfd_loop_launch(self._h, _stream_handle(stream)), "rfd_loop_launch")

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rfd_loop_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Barycenter:
    """Wasserstein barycenter of k distributions on a resident plan's cloud
    (rfd_bary_*; App. D, Alg. 1). a: area weights (N float32 CUDA vector),
    mus: N x k float32 CUDA tensor (one distribution per column), alpha: k
    weights, floor: the safeguard factor (None: no floor). launch() runs the
    iterations and returns mu (N float32, the tensor the object owns)."""

    def __init__(self, plan: "Plan", a, mus, alpha, iterations: int, floor: Optional[float] = 1.0):
        import torch
        _dev_f32(mus, "mus")
        n, k = mus.shape
        if plan.points >= 0 and plan.points != n:
            raise ValueError(f"mus has {n} rows; the plan's cloud has {plan.points} points")
        if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float32 and a.is_contiguous()
                and a.numel() == n):
            raise ValueError("a must be a contiguous float32 CUDA vector with one entry per point")
        if len(alpha) != k:
            raise ValueError("one weight per distribution")
        self.mu = torch.empty(n, dtype=torch.float32, device=mus.device)
        self._keep = (plan, a, mus)
        al = (C.c_double * k)(*[float(x) for x in alpha])
        h = C.c_void_p()
        _check(lib().rfd_bary_create(plan.handle, a.data_ptr(), mus.data_ptr(), mus.stride(0), k, al, int(iterations),
                                     -1.0 if floor is None else float(floor), self.mu.data_ptr(), C.byref(h)),
               "rfd_bary_create")
        self._h = h

    def launch(self, stream=None):
        _check(lib().rfd_bary_launch(self._h, _stream_handle(stream)), "rfd_bary_launch")
        return self.mu

    def floored(self, stream=None) -> int:
        c = C.c_int64()
        _check(lib().rfd_bary_floored(self._h, C.byref(c), _stream_handle(stream)), "rfd_bary_floored")
        return int(c.value)

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rfd_bary_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spectrum_batch(plans, k: int, which: str = "smallest", stream=None):
    """rfd_spectrum_batch: the k smallest (or largest) kernel eigenvalues of
    every plan's cloud in one launch; a list of float64 CUDA tensors."""
    import torch
    w = {"smallest": 0, "largest": 1}[which]
    n = len(plans)
    outs = [torch.empty(max(int(k), 1), dtype=torch.float64, device="cuda") for _ in range(n)]
    P = C.c_void_p * max(n, 1)
    hp = P(*[p.handle.value for p in plans])
    ho = P(*[o.data_ptr() for o in outs])
    _check(lib().rfd_spectrum_batch(hp, n, w, int(k), ho, _stream_handle(stream)), "rfd_spectrum_batch")
    return [o[: int(k)] for o in outs]


class GW:
    """Loss matrix of the Gromov-Wasserstein iterations (rfd_gw_*): the source
    plan pc and target plan pd have their features computed on clouds of n and
    m points; loss(T) returns L = v1 1^T + 1 v2^T - 2 C T D^T (n x m)."""

    def __init__(self, pc: "Plan", pd: "Plan"):
        h = C.c_void_p()
        _check(lib().rfd_gw_create(pc.handle, pd.handle, C.byref(h)), "rfd_gw_create")
        self._keep = (pc, pd)
        self._h = h
        self.n, self.m = pc.points, pd.points

    def _coupling(self, T):
        _dev_f32(T, "T", self.m)
        if T.shape[0] != self.n:
            raise ValueError(f"T must be {self.n} x {self.m}")
        return T

    def loss(self, T, out=None, stream=None):
        import torch
        self._coupling(T)
        if out is None:
            out = torch.empty(T.shape, dtype=torch.float32, device=T.device)
        _dev_f32(out, "out", self.m)
        if out.shape[0] != self.n:
            raise ValueError(f"out must be {self.n} x {self.m}")
        _check(lib().rfd_gw_loss(self._h, T.data_ptr(), T.stride(0), out.data_ptr(), out.stride(0),
                                 _stream_handle(stream)), "rfd_gw_loss")
        return out

    def terms(self, T, stream=None):
        """(v1 = C^(o2) p, v2 = D^(o2) q, W3 = C T D^T) as rfd_gw_terms returns them."""
        import torch
        self._coupling(T)
        n, m = T.shape
        v1 = torch.empty(n, dtype=torch.float32, device=T.device)
        v2 = torch.empty(m, dtype=torch.float32, device=T.device)
        W3 = torch.empty((n, m), dtype=torch.float32, device=T.device)
        _check(lib().rfd_gw_terms(self._h, T.data_ptr(), T.stride(0), v1.data_ptr(), v2.data_ptr(), W3.data_ptr(),
                                  W3.stride(0), _stream_handle(stream)), "rfd_gw_terms")
        return v1, v2, W3

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rfd_gw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request server (rfd_server_*): submit() waits for
    torch's current stream (the server's streams are not ordered after it),
    queues a request and returns its ticket; wait() returns (status,
    t_submit, t_start, t_done). The tensors of a request are kept alive until
    it has been waited for."""

    def __init__(self, hbm_budget_bytes: int, max_inflight: int = 8):
        h = C.c_void_p()
        _check(lib().rfd_server_create(int(hbm_budget_bytes), int(max_inflight), C.byref(h)), "rfd_server_create")
        self._h = h
        self._keep = {}

    def submit(self, X, F, out, m: int, eps: float, lam: float, seed: int = 0, precision="fp32", shape="ball",
               cloud_key: int = 0, sigma: float = 0.0, radius: float = 0.0) -> int:
        X = _dev_f32(X, "X", 3)
        F = _dev_f32(F, "F")
        out = _dev_f32(out, "out", F.shape[1])
        if X.stride(0) != 3 or X.shape[0] != F.shape[0] or out.shape[0] != F.shape[0]:
            raise ValueError("X must be contiguous N x 3 and F, out N x d")
        r = Request()
        r.X, r.N, r.F, r.ldF, r.d, r.reserved = X.data_ptr(), X.shape[0], F.data_ptr(), F.stride(0), F.shape[1], 0
        r.out, r.ldO = out.data_ptr(), out.stride(0)
        r.params, _ = make_params(m, eps, lam, seed, shape, precision, sigma, radius)
        r.cloud_key = int(cloud_key)
        # the server's streams do not wait for torch's: the inputs must be complete now
        import torch
        torch.cuda.current_stream().synchronize()
        t = C.c_uint64()
        _check(lib().rfd_submit(self._h, C.byref(r), C.byref(t)), "rfd_submit")
        self._keep[t.value] = (X, F, out)
        return t.value

    def wait(self, ticket: int, timeout: float = -1.0):
        res = Result()
        s = lib().rfd_wait(self._h, C.c_uint64(ticket), float(timeout), C.byref(res))
        if s == NOT_READY:
            return NOT_READY, None, None, None
        if s == INVALID_ARG:  # unknown or already collected ticket
            raise RfdError(s, "rfd_wait")
        self._keep.pop(ticket, None)
        return int(s), res.t_submit, res.t_start, res.t_done

    def stats(self) -> dict:
        b = C.c_size_t()
        p, q, i = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().rfd_server_stats(self._h, C.byref(b), C.byref(p), C.byref(q), C.byref(i)), "rfd_server_stats")
        return {"device_bytes": b.value, "plans": p.value, "queued": q.value, "inflight": i.value}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().rfd_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_export() -> str:
    n = lib().rfd_tune_export(None, 0)
    buf = C.create_string_buffer(n)
    lib().rfd_tune_export(buf, n)
    return buf.value.decode()


def tune_import(text: str) -> None:
    _check(lib().rfd_tune_import(text.encode()), "rfd_tune_import")


def tune_reset() -> None:
    lib().rfd_tune_reset()


def profile_enable(on: bool) -> None:
    lib().rfd_profile_enable(1 if on else 0)


def profile_read(reset: bool = True) -> dict:
    """{kernel name: (total ms, launches)} since the last reset (synchronises the device)."""
    n = 32
    tot = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    k = lib().rfd_profile_read(tot.ctypes.data, cnt.ctypes.data, n, 1 if reset else 0)
    return {lib().rfd_profile_kernel_name(i).decode(): (float(tot[i]), int(cnt[i])) for i in range(k) if cnt[i]}


def declared_symbols(header: Optional[str] = None) -> list[str]:
    """Function names declared in include/rfd.h."""
    import re
    header = header or os.path.join(os.path.dirname(_HERE), "include", "rfd.h")
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rfd_[a-z_]+)\s*\(", text)))
