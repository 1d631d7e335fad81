"""ctypes binding of libqoc (include/qoc.h).

Argument marshalling only: every step of the GRAPE path runs in the HIP
kernels of libqoc.so.  PyTorch provides device memory and streams for the
device entry points.  There is no fallback: if the library is not built, or
it reports an error, the call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqoc.so")

QOC_OK = 0
FP64, FP32, BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16x3": BF16X3}

_ERRORS = {
    -1: "QOC_ERR_ARG",
    -2: "QOC_ERR_NOT_HERMITIAN",
    -3: "QOC_ERR_NONFINITE",
    -4: "QOC_ERR_OOM",
    -5: "QOC_ERR_DEVICE",
    -6: "QOC_ERR_UNSUPPORTED",
    -7: "QOC_ERR_NOT_UNITARY",
}

# Every symbol include/qoc.h declares.
EXPORTS = (
    "qoc_default_options",
    "qoc_propagate",
    "qoc_fidelity",
    "qoc_gradient",
    "qoc_workspace_size",
    "qoc_default_chunk",
    "qoc_engine_chunk",
    "qoc_propagate_dev",
    "qoc_fidelity_dev",
    "qoc_gradient_dev",
    "qoc_gradient_dev_noalloc",
    "qoc_trace_gradient_dev",
    "qoc_slice_plan",
    "qoc_state_workspace_size",
    "qoc_state_propagate",
    "qoc_state_gradient",
    "qoc_state_propagate_dev",
    "qoc_state_gradient_dev",
    "qoc_stage_timing",
    "qoc_stage_times",
    "qoc_stage_name",
    "qoc_engine_footprint",
    "qoc_engine_create",
    "qoc_engine_destroy",
    "qoc_engine_submit",
    "qoc_engine_step",
    "qoc_engine_poll",
    "qoc_engine_fetch",
    "qoc_engine_stats",
    "qoc_last_error",
    "qoc_version",
)


class QocError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("validate", ctypes.c_int32),
        ("hbm_budget", ctypes.c_uint64),
        ("reunitarise_tol", ctypes.c_double),
        ("stream", ctypes.c_void_p),
        ("chunk", ctypes.c_int32),
        ("dense_controls", ctypes.c_int32),
        ("diagnostics", ctypes.c_void_p),
        ("generators", ctypes.c_int32),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libqoc.so (after torch, so both use one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2208_12187_amd/build.py")
    try:
        import torch  # noqa: F401  (loads the HIP runtime torch was built with)
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, dbl, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    opt = ctypes.POINTER(Options)
    L.qoc_default_options.argtypes = [opt]
    L.qoc_default_options.restype = None
    L.qoc_propagate.argtypes = [i32, i32, i32, vp, vp, vp, dbl, vp, opt]
    L.qoc_fidelity.argtypes = [i32, i32, i32, vp, vp, vp, dbl, vp, vp, opt]
    L.qoc_gradient.argtypes = [i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, opt]
    L.qoc_workspace_size.argtypes = [i32, i32, i32, i32, i32, i32, ctypes.c_uint64]
    L.qoc_workspace_size.restype = sz
    L.qoc_default_chunk.argtypes = [i32, i32]
    L.qoc_default_chunk.restype = i32
    L.qoc_engine_chunk.argtypes = [i32, i32]
    L.qoc_engine_chunk.restype = i32
    L.qoc_propagate_dev.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, sz, opt]
    L.qoc_fidelity_dev.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, sz, opt]
    L.qoc_gradient_dev.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp, sz, opt]
    L.qoc_gradient_dev_noalloc.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, opt]
    L.qoc_trace_gradient_dev.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp, sz, opt]
    L.qoc_slice_plan.argtypes = [i32, i32, i32, vp, vp, vp, dbl, i32, i32, vp]
    L.qoc_state_workspace_size.argtypes = [i32, i32, i32, i32, i32]
    L.qoc_state_workspace_size.restype = sz
    L.qoc_state_propagate.argtypes = [i32, i32, i32, vp, vp, vp, dbl, vp, vp, opt]
    L.qoc_state_gradient.argtypes = [i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp, opt]
    L.qoc_state_propagate_dev.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, sz, opt]
    L.qoc_state_gradient_dev.argtypes = [i32, i32, i32, i32, vp, vp, vp, dbl, vp, vp, vp, vp, vp, sz, opt]
    L.qoc_stage_timing.argtypes = [i32]
    L.qoc_stage_times.argtypes = [i32, vp, vp]
    L.qoc_stage_name.argtypes = [i32]
    L.qoc_stage_name.restype = ctypes.c_char_p
    u64, i64p = ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64)
    L.qoc_engine_footprint.argtypes = [i32, i32, i32, i32]
    L.qoc_engine_footprint.restype = u64
    L.qoc_engine_create.argtypes = [i32, u64, u64, i32, ctypes.POINTER(vp)]
    L.qoc_engine_destroy.argtypes = [vp]
    L.qoc_engine_submit.argtypes = [vp, i32, i32, i32, vp, vp, vp, dbl, vp, i64p]
    L.qoc_engine_step.argtypes = [vp, i32]
    L.qoc_engine_poll.argtypes = [vp, i32, vp, vp, ctypes.POINTER(ctypes.c_int)]
    L.qoc_engine_fetch.argtypes = [vp, ctypes.c_int64, vp]
    L.qoc_engine_stats.argtypes = [vp, i64p, i64p, ctypes.POINTER(u64)]
    for name in ("qoc_engine_create", "qoc_engine_destroy", "qoc_engine_submit", "qoc_engine_step",
                 "qoc_engine_poll", "qoc_engine_fetch", "qoc_engine_stats"):
        getattr(L, name).restype = ctypes.c_int
    L.qoc_last_error.restype = ctypes.c_char_p
    L.qoc_version.restype = ctypes.c_char_p
    for name in ("qoc_stage_timing", "qoc_stage_times", "qoc_propagate", "qoc_fidelity", "qoc_gradient", "qoc_propagate_dev", "qoc_fidelity_dev",
                 "qoc_gradient_dev", "qoc_gradient_dev_noalloc", "qoc_trace_gradient_dev", "qoc_slice_plan",
                 "qoc_state_propagate",
                 "qoc_state_gradient", "qoc_state_propagate_dev", "qoc_state_gradient_dev"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != QOC_OK:
        raise QocError(rc, lib().qoc_last_error().decode())


def options(precision="fp64", validate=False, chunk=0, stream=None, hbm_budget=0, dense_controls=False,
            generators=False) -> Options:
    o = Options()
    lib().qoc_default_options(ctypes.byref(o))
    o.generators = 1 if generators else 0
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.validate = 1 if validate else 0
    o.chunk = int(chunk)
    o.stream = stream
    o.hbm_budget = int(hbm_budget)
    o.dense_controls = 1 if dense_controls else 0
    return o


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------ host entry points

def propagate(H0, Hc, u, dt, precision="fp64", validate=False, chunk=0, hbm_budget=0, dense_controls=False, generators=False) -> np.ndarray:
    """X_N = U_{N-1} ... U_0 (host arrays in, host array out)."""
    H0, Hc, u = _c128(H0), _c128(Hc), _f64(u)
    d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
    out = np.empty((d, d), dtype=np.complex128)
    o = options(precision, validate, chunk, None, hbm_budget, dense_controls, generators)
    _check(lib().qoc_propagate(d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), _ptr(out), ctypes.byref(o)))
    return out


def fidelity(H0, Hc, u, dt, V, precision="fp64", validate=False, chunk=0, hbm_budget=0, dense_controls=False, generators=False) -> float:
    H0, Hc, u, V = _c128(H0), _c128(Hc), _f64(u), _c128(V)
    d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
    F = np.zeros(1)
    o = options(precision, validate, chunk, None, hbm_budget, dense_controls, generators)
    _check(lib().qoc_fidelity(d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), _ptr(V), _ptr(F), ctypes.byref(o)))
    return float(F[0])


def gradient(H0, Hc, u, dt, V, precision="fp64", validate=False, chunk=0, hbm_budget=0, dense_controls=False, generators=False):
    """(F, grad) with grad[j, k] = dF/du[j, k]."""
    H0, Hc, u, V = _c128(H0), _c128(Hc), _f64(u), _c128(V)
    d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
    F = np.zeros(1)
    grad = np.empty((m, N))
    o = options(precision, validate, chunk, None, hbm_budget, dense_controls, generators)
    _check(lib().qoc_gradient(d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), _ptr(V), _ptr(F), _ptr(grad),
                              ctypes.byref(o)))
    return float(F[0]), grad


def state_propagate(H0, Hc, u, dt, psi0, precision="fp64", validate=False, dense_controls=False) -> np.ndarray:
    """psi_N = U_{N-1} ... U_0 psi0 (host arrays in, host array out)."""
    H0, Hc, u, psi0 = _c128(H0), _c128(Hc), _f64(u), _c128(psi0)
    d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
    out = np.empty(d, dtype=np.complex128)
    o = options(precision, validate, 0, None, 0, dense_controls)
    _check(lib().qoc_state_propagate(d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), _ptr(psi0), _ptr(out),
                                     ctypes.byref(o)))
    return out


def state_gradient(H0, Hc, u, dt, psi0, chi, precision="fp64", validate=False, dense_controls=False):
    """(F, grad) of the state transfer psi0 -> chi, F = |<chi|psi_N>|^2."""
    H0, Hc, u, psi0, chi = _c128(H0), _c128(Hc), _f64(u), _c128(psi0), _c128(chi)
    d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
    F = np.zeros(1)
    grad = np.empty((m, N))
    o = options(precision, validate, 0, None, 0, dense_controls)
    _check(lib().qoc_state_gradient(d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), _ptr(psi0), _ptr(chi),
                                    _ptr(F), _ptr(grad), ctypes.byref(o)))
    return float(F[0]), grad


def state_workspace_size(B, d, m, N, precision="fp64") -> int:
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = lib().qoc_state_workspace_size(B, d, m, N, p)
    if n == 0:
        _check(-1)
    return int(n)


def slice_plan(H0, Hc, u, dt, precision="fp64", with_gradient=True) -> np.ndarray:
    """(N, 3) array of (s, q, qb) per slice, as the kernels choose them."""
    H0, Hc, u = _c128(H0), _c128(Hc), _f64(u)
    d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
    out = np.empty((N, 3), dtype=np.int32)
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(lib().qoc_slice_plan(d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), p, 1 if with_gradient else 0,
                                _ptr(out)))
    return out


def default_chunk(d, N) -> int:
    """Slices per scan chunk when the chunk option is 0."""
    n = lib().qoc_default_chunk(d, N)
    if n == 0:
        _check(-1)
    return int(n)


def engine_chunk(d, N) -> int:
    """Slices per scan chunk the serving engine uses for a request."""
    n = lib().qoc_engine_chunk(d, N)
    if n == 0:
        _check(-1)
    return int(n)


def workspace_size(B, d, m, N, precision="fp64", chunk=0, hbm_budget=0) -> int:
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    n = lib().qoc_workspace_size(B, d, m, N, p, chunk, int(hbm_budget))
    if n == 0:
        _check(-1)
    return int(n)


# ------------------------------------------------------------ device entry points

class Batch:
    """B problems with shared (d, m, N, dt) resident on a torch device.

    H0 [B, d, d], Hc [B, m, d, d], V [B, d, d] complex128; u [B, m, N] float64.
    """

    def __init__(self, H0, Hc, u, dt, V=None):
        import torch

        self.H0 = H0.contiguous()
        self.Hc = Hc.contiguous()
        self.u = u.contiguous()
        self.V = None if V is None else V.contiguous()
        self.dt = float(dt)
        assert self.H0.dtype == torch.complex128 and self.Hc.dtype == torch.complex128
        assert self.u.dtype == torch.float64
        self.B, self.d = self.H0.shape[0], self.H0.shape[1]
        self.m, self.N = self.u.shape[1], self.u.shape[2]
        assert tuple(self.Hc.shape) == (self.B, self.m, self.d, self.d)
        assert tuple(self.u.shape) == (self.B, self.m, self.N)
        if self.V is not None:
            assert self.V.dtype == torch.complex128 and tuple(self.V.shape) == (self.B, self.d, self.d)

    @staticmethod
    def from_problems(problems, device="cuda"):
        import torch

        H0 = torch.from_numpy(np.stack([p.H0 for p in problems])).to(device)
        Hc = torch.from_numpy(np.stack([p.Hc for p in problems])).to(device)
        u = torch.from_numpy(np.stack([p.u for p in problems])).to(device)
        V = torch.from_numpy(np.stack([p.V for p in problems])).to(device)
        dts = {p.dt for p in problems}
        assert len(dts) == 1, "a batch shares dt"
        return Batch(H0, Hc, u, dts.pop(), V)


class Runner:
    """Owns a device workspace for repeated calls on batches of one shape."""

    def __init__(self, B, d, m, N, precision="fp64", chunk=0, device="cuda", hbm_budget=0, dense_controls=False,
                 generators=False):
        import torch

        self.generators = bool(generators)
        self.B, self.d, self.m, self.N = B, d, m, N
        self.precision = precision
        self.chunk = chunk
        self.hbm_budget = int(hbm_budget)
        self.dense_controls = bool(dense_controls)
        self.ws_bytes = workspace_size(B, d, m, N, precision, chunk, hbm_budget)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)
        self.device = device

    def _opt(self, stream):
        import torch

        st = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        return options(self.precision, False, self.chunk, ctypes.c_void_p(st.cuda_stream), self.hbm_budget,
                       self.dense_controls, self.generators)

    def _shape_ok(self, b: Batch):
        if (b.B, b.d, b.m, b.N) != (self.B, self.d, self.m, self.N):
            raise ValueError("batch shape does not match the runner")

    def gradient(self, b: Batch, F=None, grad=None, stream=None):
        """Enqueue F [B] and grad [B, m, N] (float64 device tensors)."""
        import torch

        self._shape_ok(b)
        if F is None:
            F = torch.empty(b.B, dtype=torch.float64, device=self.ws.device)
        if grad is None:
            grad = torch.empty((b.B, b.m, b.N), dtype=torch.float64, device=self.ws.device)
        o = self._opt(stream)
        _check(lib().qoc_gradient_dev(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(), b.dt,
                                      b.V.data_ptr(), F.data_ptr(), grad.data_ptr(), self.ws.data_ptr(),
                                      self.ws_bytes, ctypes.byref(o)))
        return F, grad

    def trace_gradient(self, b: Batch, g=None, dg=None, stream=None):
        """Enqueue g [B] = Tr(V^dag X_N) and dg [B, m, N] = dg/du (complex128
        device tensors); V need not be unitary."""
        import torch

        self._shape_ok(b)
        if g is None:
            g = torch.empty(b.B, dtype=torch.complex128, device=self.ws.device)
        if dg is None:
            dg = torch.empty((b.B, b.m, b.N), dtype=torch.complex128, device=self.ws.device)
        o = self._opt(stream)
        _check(lib().qoc_trace_gradient_dev(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(),
                                            b.dt, b.V.data_ptr(), g.data_ptr(), dg.data_ptr(), self.ws.data_ptr(),
                                            self.ws_bytes, ctypes.byref(o)))
        return g, dg

    def fidelity(self, b: Batch, F=None, stream=None):
        import torch

        self._shape_ok(b)
        if F is None:
            F = torch.empty(b.B, dtype=torch.float64, device=self.ws.device)
        o = self._opt(stream)
        _check(lib().qoc_fidelity_dev(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(), b.dt,
                                      b.V.data_ptr(), F.data_ptr(), self.ws.data_ptr(), self.ws_bytes,
                                      ctypes.byref(o)))
        return F

    def propagate(self, b: Batch, out=None, stream=None):
        import torch

        self._shape_ok(b)
        if out is None:
            out = torch.empty((b.B, b.d, b.d), dtype=torch.complex128, device=self.ws.device)
        o = self._opt(stream)
        _check(lib().qoc_propagate_dev(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(), b.dt,
                                       out.data_ptr(), self.ws.data_ptr(), self.ws_bytes, ctypes.byref(o)))
        return out


class StateBatch:
    """B state-transfer problems with shared (d, m, N, dt) on a torch device:
    H0 [B, d, d], Hc [B, m, d, d] complex128, u [B, m, N] float64,
    psi0 [B, d], chi [B, d] complex128."""

    def __init__(self, H0, Hc, u, dt, psi0, chi):
        import torch

        self.H0, self.Hc, self.u = H0.contiguous(), Hc.contiguous(), u.contiguous()
        self.psi0, self.chi = psi0.contiguous(), chi.contiguous()
        self.dt = float(dt)
        self.B, self.d = self.H0.shape[0], self.H0.shape[1]
        self.m, self.N = self.u.shape[1], self.u.shape[2]
        assert self.H0.dtype == torch.complex128 and self.psi0.dtype == torch.complex128
        assert tuple(self.psi0.shape) == (self.B, self.d) and tuple(self.chi.shape) == (self.B, self.d)
        assert tuple(self.Hc.shape) == (self.B, self.m, self.d, self.d)

    @staticmethod
    def from_problems(problems, device="cuda"):
        import torch

        st = lambda xs: torch.from_numpy(np.stack(xs)).to(device)
        dts = {p.dt for p in problems}
        assert len(dts) == 1, "a batch shares dt"
        return StateBatch(st([p.H0 for p in problems]), st([p.Hc for p in problems]), st([p.u for p in problems]),
                          dts.pop(), st([p.psi0 for p in problems]), st([p.chi for p in problems]))


class StateRunner:
    """Owns a device workspace for repeated state-transfer calls of one shape."""

    def __init__(self, B, d, m, N, precision="fp64", device="cuda", dense_controls=False):
        import torch

        self.B, self.d, self.m, self.N, self.precision = B, d, m, N, precision
        self.dense_controls = bool(dense_controls)
        self.ws_bytes = state_workspace_size(B, d, m, N, precision)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def _opt(self, stream):
        import torch

        st = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        return options(self.precision, False, 0, ctypes.c_void_p(st.cuda_stream), 0, self.dense_controls)

    def gradient(self, b: StateBatch, F=None, grad=None, stream=None):
        import torch

        if (b.B, b.d, b.m, b.N) != (self.B, self.d, self.m, self.N):
            raise ValueError("batch shape does not match the runner")
        if F is None:
            F = torch.empty(b.B, dtype=torch.float64, device=self.ws.device)
        if grad is None:
            grad = torch.empty((b.B, b.m, b.N), dtype=torch.float64, device=self.ws.device)
        o = self._opt(stream)
        _check(lib().qoc_state_gradient_dev(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(),
                                            b.dt, b.psi0.data_ptr(), b.chi.data_ptr(), F.data_ptr(),
                                            grad.data_ptr(), self.ws.data_ptr(), self.ws_bytes, ctypes.byref(o)))
        return F, grad

    def propagate(self, b: StateBatch, out=None, stream=None):
        import torch

        if out is None:
            out = torch.empty((b.B, b.d), dtype=torch.complex128, device=self.ws.device)
        o = self._opt(stream)
        _check(lib().qoc_state_propagate_dev(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(),
                                             b.dt, b.psi0.data_ptr(), out.data_ptr(), self.ws.data_ptr(),
                                             self.ws_bytes, ctypes.byref(o)))
        return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # QOC_NOALLOC_SCRATCH_BYTES in include/qoc.h


def gradient_noalloc(b: Batch, F, grad, precision="fp64", chunk=0, hbm_budget=0, dense_controls=False,
                     stream=None):
    """qoc_gradient_dev_noalloc: F [B] and grad [B, m, N] (float64 device
    tensors, caller-allocated) with libqoc's static device scratch as the
    workspace; no device memory is allocated by the call."""
    import torch

    st = stream if stream is not None else torch.cuda.current_stream(F.device)
    o = options(precision, False, chunk, ctypes.c_void_p(st.cuda_stream), hbm_budget, dense_controls)
    _check(lib().qoc_gradient_dev_noalloc(b.B, b.d, b.m, b.N, b.H0.data_ptr(), b.Hc.data_ptr(), b.u.data_ptr(),
                                          b.dt, b.V.data_ptr(), F.data_ptr(), grad.data_ptr(), ctypes.byref(o)))
    return F, grad


STAGES = ("prep", "plan", "expm", "scan", "carry", "mc", "bscan", "adjoint", "state_chain", "state_grad")


class Engine:
    """Continuous-batching serving engine of libqoc (see include/qoc.h)."""

    def __init__(self, precision="fp32", pool_bytes=64 << 30, host_bytes=8 << 30, max_active=256):
        self._p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        h = ctypes.c_void_p()
        _check(lib().qoc_engine_create(self._p, int(pool_bytes), int(host_bytes), int(max_active), ctypes.byref(h)))
        self._h = h
        self._shape = {}
        self._ids = np.zeros(4096, dtype=np.int64)
        self._F = np.zeros(4096)

    def close(self):
        if self._h:
            lib().qoc_engine_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def footprint(precision, d, m, N) -> int:
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        return int(lib().qoc_engine_footprint(p, d, m, N))

    def submit(self, H0, Hc, u, dt, V) -> int:
        H0, Hc, u, V = _c128(H0), _c128(Hc), _f64(u), _c128(V)
        d, m, N = H0.shape[0], Hc.shape[0], u.shape[1]
        rid = ctypes.c_int64()
        _check(lib().qoc_engine_submit(self._h, d, m, N, _ptr(H0), _ptr(Hc), _ptr(u), float(dt), _ptr(V),
                                       ctypes.byref(rid)))
        self._shape[rid.value] = (m, N)
        return rid.value

    def step(self, wait=False):
        _check(lib().qoc_engine_step(self._h, 1 if wait else 0))

    def poll(self):
        """[(id, F)] of requests finished since the last poll."""
        n = ctypes.c_int()
        _check(lib().qoc_engine_poll(self._h, len(self._ids), _ptr(self._ids), _ptr(self._F), ctypes.byref(n)))
        return [(int(self._ids[i]), float(self._F[i])) for i in range(n.value)]

    def fetch(self, rid) -> np.ndarray:
        m, N = self._shape.pop(rid)
        g = np.empty((m, N))
        _check(lib().qoc_engine_fetch(self._h, int(rid), _ptr(g)))
        return g

    def stats(self):
        q, a, u = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_uint64()
        _check(lib().qoc_engine_stats(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(u)))
        return {"queued": q.value, "active": a.value, "pool_used": u.value}


def stage_timing(enable: bool):
    """Record hipEvents around every kernel stage of subsequent launches."""
    _check(lib().qoc_stage_timing(1 if enable else 0))


def stage_times() -> dict:
    """{stage: (total_ms, launches)} since the last call; waits for the events."""
    n = len(STAGES)
    ms = np.zeros(n)
    cnt = np.zeros(n, dtype=np.int64)
    _check(lib().qoc_stage_times(n, _ptr(ms), _ptr(cnt)))
    return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}


def version() -> str:
    return lib().qoc_version().decode()
