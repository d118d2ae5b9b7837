"""ctypes binding of libfmnmf.so (the C ABI declared in include/fmnmf.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  PyTorch provides device memory (the mixture, the workspace,
the separated output) and the HIP stream.  The binding fails loudly when the
library has not been built; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmnmf.so")

FP64, FP32, MIXED_BF16 = 0, 1, 2
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": MIXED_BF16, "mixed": MIXED_BF16}
NORMALIZE, TIE_G_OVER_F, WITH_DERIVED, FCA = 1, 2, 4, 8

OK, E_INVAL, E_UNSUPPORTED, E_WORKSPACE, E_HIP, E_SINGULAR, E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
EXPORTS = ("fmnmf_workspace_bytes", "fmnmf_footprint_bytes", "fmnmf_init", "fmnmf_step",
           "fmnmf_loglik", "fmnmf_separate", "fmnmf_get_state", "fmnmf_set_state",
           "fmnmf_get_derived", "fmnmf_destroy", "fmnmf_last_error", "fmnmf_profile_step",
           "fmnmf_kernel_name", "fmnmf_step_batch", "fmnmf_init_scm", "fmnmf_init_noalloc")
KERNELS = ("wpass", "mu_w", "hpass", "mu_h", "gpass", "mu_g", "vpass", "ip", "norm", "proj", "lam")


class Dims(ctypes.Structure):
    _fields_ = [("F", ctypes.c_int), ("T", ctypes.c_int), ("M", ctypes.c_int),
                ("N", ctypes.c_int), ("K", ctypes.c_int), ("precision", ctypes.c_int),
                ("flags", ctypes.c_uint), ("delta", ctypes.c_double)]


class FmnmfError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fmnmf error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libfmnmf.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it first (python -c "
                           "'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(LIB_PATH)
    vp, dp, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_size_t
    L.fmnmf_workspace_bytes.argtypes = [ctypes.POINTER(Dims)]
    L.fmnmf_workspace_bytes.restype = sz
    L.fmnmf_footprint_bytes.argtypes = [ctypes.POINTER(Dims)]
    L.fmnmf_footprint_bytes.restype = sz
    L.fmnmf_init.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Dims), vp, vp, sz, dp, dp, dp, dp, vp]
    L.fmnmf_init_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(Dims), vp, dp, dp, dp, dp, vp]
    L.fmnmf_init_noalloc.restype = ctypes.c_int
    L.fmnmf_step.argtypes = [vp, ctypes.c_int]
    L.fmnmf_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.c_int, ctypes.c_int]
    L.fmnmf_step_batch.restype = ctypes.c_int
    L.fmnmf_loglik.argtypes = [vp, dp]
    L.fmnmf_init_scm.argtypes = [vp]
    L.fmnmf_init_scm.restype = ctypes.c_int
    L.fmnmf_separate.argtypes = [vp, vp]
    L.fmnmf_get_state.argtypes = [vp, dp, dp, dp, dp]
    L.fmnmf_set_state.argtypes = [vp, dp, dp, dp, dp]
    L.fmnmf_get_derived.argtypes = [vp, ctypes.c_int, dp]
    L.fmnmf_destroy.argtypes = [vp]
    L.fmnmf_destroy.restype = None
    L.fmnmf_profile_step.argtypes = [vp, ctypes.c_int, dp]
    L.fmnmf_profile_step.restype = ctypes.c_int
    L.fmnmf_kernel_name.argtypes = [ctypes.c_int]
    L.fmnmf_kernel_name.restype = ctypes.c_char_p
    L.fmnmf_last_error.argtypes = []
    L.fmnmf_last_error.restype = ctypes.c_char_p
    for name in ("fmnmf_init", "fmnmf_step", "fmnmf_loglik", "fmnmf_separate", "fmnmf_get_state",
                 "fmnmf_set_state", "fmnmf_get_derived"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != OK:
        raise FmnmfError(rc, lib().fmnmf_last_error().decode())


def _dp(a):
    if a is None:
        return ctypes.POINTER(ctypes.c_double)()
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_dims(F, T, M, N, K, precision="fp64", delta=0.0, flags=0) -> Dims:
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return Dims(F, T, M, N, K, p, flags, float(delta))


def workspace_bytes(dims: Dims) -> int:
    return int(lib().fmnmf_workspace_bytes(ctypes.byref(dims)))


def footprint_bytes(dims: Dims) -> int:
    return int(lib().fmnmf_footprint_bytes(ctypes.byref(dims)))


def _f64c(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _q_as_f64(Q) -> np.ndarray:
    q = np.ascontiguousarray(np.asarray(Q, dtype=np.complex128))
    return q.view(np.float64)


def step_batch(models, n: int = 1):
    """Enqueue n iterations of every model in `models` as batched launches
    (fmnmf_step_batch): work goes on the first model's stream; the others'
    streams are joined before and after."""
    ms = list(models)
    arr = (ctypes.c_void_p * len(ms))(*[m._ctx.value for m in ms])
    _check(lib().fmnmf_step_batch(arr, len(ms), int(n)))


class FastMNMF:
    """One separation problem resident on the device.

    X        torch complex tensor [F, T, M] on a HIP device (complex128 for
             "fp64", complex64 for "fp32" / "bf16"); borrowed for the
             lifetime of the object.
    init     (W0 [N,K,F], H0 [N,K,T], G0 [N,F,M], Q0 [F,M,M] complex) host arrays.
    normalize / tie_g  the FMNMF_NORMALIZE / FMNMF_TIE_G_OVER_F options.
    noalloc  use fmnmf_init_noalloc: the workspace is the library's static
             device array (one such model per device at a time).
    """

    def __init__(self, X, N: int, K: int, init, precision="fp64", delta=0.0,
                 derived=False, stream=None, normalize=False, tie_g=False, noalloc=False):
        flags = (WITH_DERIVED if derived else 0) | (NORMALIZE if normalize else 0) | (TIE_G_OVER_F if tie_g else 0)
        self._open(X, N, K, init, precision, delta, flags, stream, noalloc)

    def _open(self, X, N, K, init, precision, delta, flags, stream, noalloc=False):
        import torch

        F, T, M = X.shape
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        want = torch.complex128 if p == FP64 else torch.complex64
        if X.dtype != want or not X.is_cuda or not X.is_contiguous():
            raise ValueError(f"X must be a contiguous {want} HIP tensor")
        self.dims = make_dims(F, T, M, N, K, p, delta, flags)
        self.precision = p
        self.shape = (F, T, M, N, K)
        self.X = X
        nbytes = workspace_bytes(self.dims)
        if nbytes == 0:
            raise FmnmfError(E_INVAL, lib().fmnmf_last_error().decode())
        self.ws = None if noalloc else torch.empty(nbytes, dtype=torch.uint8, device=X.device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=X.device)
        torch.cuda.current_stream(X.device).synchronize()  # X / ws are ready before our stream uses them
        W0, H0, G0, Q0 = init
        self._ctx = ctypes.c_void_p()
        args = (_dp(_f64c(W0)), _dp(None if H0 is None else _f64c(H0)), _dp(_f64c(G0)), _dp(_q_as_f64(Q0)),
                ctypes.c_void_p(self.stream.cuda_stream))
        if noalloc:
            with torch.cuda.device(X.device):
                _check(lib().fmnmf_init_noalloc(ctypes.byref(self._ctx), ctypes.byref(self.dims),
                                                ctypes.c_void_p(X.data_ptr()), *args))
        else:
            _check(lib().fmnmf_init(ctypes.byref(self._ctx), ctypes.byref(self.dims),
                                    ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(self.ws.data_ptr()),
                                    nbytes, *args))

    # -- iteration ---------------------------------------------------------
    def step(self, n: int = 1):
        _check(lib().fmnmf_step(self._ctx, int(n)))

    def profile(self, n: int = 1) -> dict:
        """n instrumented iterations; mean kernel durations in ms (HIP events)."""
        ms = np.zeros(len(KERNELS))
        _check(lib().fmnmf_profile_step(self._ctx, int(n), _dp(ms)))
        return dict(zip(KERNELS, ms.tolist()))

    def init_scm(self):
        """Replace Q and G~ by the paper's initialisation from the average
        observed SCM (fmnmf_init_scm)."""
        _check(lib().fmnmf_init_scm(self._ctx))

    def loglik(self) -> float:
        v = ctypes.c_double()
        _check(lib().fmnmf_loglik(self._ctx, ctypes.byref(v)))
        return v.value

    def separate(self, out=None):
        """Wiener-filtered source images [N, F, T, M] (complex, X's dtype).
        ``out`` may be a preallocated contiguous tensor of that shape."""
        import torch

        F, T, M, N, _ = self.shape
        dt = torch.complex128 if self.precision == FP64 else torch.complex64
        if out is None:
            out = torch.empty((N, F, T, M), dtype=dt, device=self.X.device)
            torch.cuda.current_stream(self.X.device).synchronize()
        elif out.shape != (N, F, T, M) or out.dtype != dt or not out.is_contiguous():
            raise ValueError("out must be a contiguous [N, F, T, M] tensor of X's dtype")
        _check(lib().fmnmf_separate(self._ctx, ctypes.c_void_p(out.data_ptr())))
        return out

    # -- state ---------------------------------------------------------------
    def get_state(self):
        F, T, M, N, K = self.shape
        W = np.empty((N, K, F))
        H = np.empty((N, K, T))
        G = np.empty((N, F, M))
        Q = np.empty((F, M, M), dtype=np.complex128)
        _check(lib().fmnmf_get_state(self._ctx, _dp(W), _dp(H), _dp(G), _dp(Q.view(np.float64))))
        return W, H, G, Q

    def set_state(self, W, H, G, Q):
        _check(lib().fmnmf_set_state(self._ctx, _dp(_f64c(W)), _dp(_f64c(H)), _dp(_f64c(G)),
                                     _dp(_q_as_f64(Q))))

    def derived(self, which: int) -> np.ndarray:
        F, T, M, _, _ = self.shape
        out = np.empty((F, T, M))
        _check(lib().fmnmf_get_derived(self._ctx, int(which), _dp(out)))
        return out

    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            lib().fmnmf_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FastFCA(FastMNMF):
    """FastFCA (flag FMNMF_FCA): the unconstrained source model, lambda [N, F, T]
    updated by Eq. (22), with the same spatial model and IP step.

    init     (lam0 [N,F,T], G0 [N,F,M], Q0 [F,M,M] complex) host arrays.
    """

    def __init__(self, X, N: int, init, precision="fp64", delta=0.0, derived=False, stream=None,
                 tie_g=False):
        lam0, G0, Q0 = init
        flags = FCA | (WITH_DERIVED if derived else 0) | (TIE_G_OVER_F if tie_g else 0)
        self._open(X, N, 0, (lam0, None, G0, Q0), precision, delta, flags, stream)

    def get_state(self):
        F, T, M, N, _ = self.shape
        lam = np.empty((N, F, T))
        G = np.empty((N, F, M))
        Q = np.empty((F, M, M), dtype=np.complex128)
        _check(lib().fmnmf_get_state(self._ctx, _dp(lam), _dp(None), _dp(G), _dp(Q.view(np.float64))))
        return lam, G, Q

    def set_state(self, lam, G, Q):
        _check(lib().fmnmf_set_state(self._ctx, _dp(_f64c(lam)), _dp(None), _dp(_f64c(G)), _dp(_q_as_f64(Q))))
