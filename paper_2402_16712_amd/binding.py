"""Thin ctypes binding of the C ABI in include/l1line.h.

Argument marshalling only: device memory and the current stream come from
PyTorch, every step of the method runs in the library's HIP kernels.  There
is no fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_build", "libl1line.so")

OK, EINVAL, EHIP, ENONFINITE, ERANGE, ENOMEM, EWIDE, ESIZE, EINTERNAL, EIO, ENOMODEL = \
    0, -1, -2, -3, -4, -5, -6, -7, -8, -9, -10
MAX_N = 65535
BP_MAX_N = 16384
MAX_LAMBDAS = 128
NOALLOC_MAX_M = 1024

EXPORTS = ["l1line_create", "l1line_destroy", "l1line_strerror", "l1line_last_error", "l1line_column_stats",
           "l1line_fit", "l1line_fit_noalloc", "l1line_fit_path", "l1line_fit_batch", "l1line_autotune",
           "l1line_tune_get",
           "l1line_tune_set", "l1line_profile", "l1line_profile_read", "l1line_ranker_features",
           "l1line_ranker_signsums", "l1line_mlp_forward", "l1line_mlp_grad", "l1line_mlp_adam",
           "l1line_fit_ranked", "l1line_ranker_load",
           "l1line_ranker_save", "l1line_ranker_set_params", "l1line_ranker_get_params", "l1line_ranker_train",
           "l1line_breakpoints", "l1line_components", "l1line_solution_path", "l1line_measure_peaks",
           "l1line_tune_lookup"]
BATCH_GRAPH = 1
FEATURES = 32
MLP_PARAMS = 20865


class Problem(ctypes.Structure):
    """l1line_problem of include/l1line.h."""
    _fields_ = [("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("ld", ctypes.c_int64), ("lambdas", ctypes.c_void_p), ("L", ctypes.c_int64),
                ("V", ctypes.c_void_p), ("J", ctypes.c_void_p), ("OBJ", ctypes.c_void_p),
                ("ROW", ctypes.c_void_p), ("ZALL", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class L1LineError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


_lib = None


def lib() -> ctypes.CDLL:
    """Load the built library (build it with paper_2402_16712_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build() or python -m paper_2402_16712_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        P, I64, I32, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
        L.l1line_create.argtypes = [ctypes.POINTER(P), I32, ctypes.c_char_p]
        L.l1line_last_error.argtypes = [P]
        L.l1line_ranker_load.argtypes = [P, ctypes.c_char_p]
        L.l1line_ranker_save.argtypes = [P, ctypes.c_char_p]
        L.l1line_ranker_set_params.argtypes = [P, P, P]
        L.l1line_ranker_get_params.argtypes = [P, P, P]
        L.l1line_ranker_train.argtypes = [P, ctypes.c_char_p, I64, ctypes.c_uint64]
        L.l1line_breakpoints.argtypes = [P, P, I64, I64, I64, P, P, P, P, P, I64, P, P]
        L.l1line_components.argtypes = [P, P, I64, I64, I64, D, I64, P, P, P, P, P, P]
        L.l1line_solution_path.argtypes = [P, P, I64, I64, I64, I64, P, P, P, P, P, P, P, P, P, P]
        L.l1line_destroy.argtypes = [P]
        L.l1line_strerror.argtypes = [I32]
        L.l1line_strerror.restype = ctypes.c_char_p
        L.l1line_column_stats.argtypes = [P, P, I64, I64, I64, P, P, P, P]
        L.l1line_fit.argtypes = [P, P, I64, I64, I64, D, P, P, P, P, P, P, P]
        L.l1line_fit_noalloc.argtypes = [P, P, I64, I64, I64, D, P, P, P, P, P, P, P]
        L.l1line_fit_path.argtypes = [P, P, I64, I64, I64, P, I64, P, P, P, P, P, P, P]
        L.l1line_fit_batch.argtypes = [P, P, I64, I32, P]
        L.l1line_autotune.argtypes = [P, P, I64, P, P]
        L.l1line_tune_get.argtypes = [P, P]
        L.l1line_tune_set.argtypes = [P, P]
        L.l1line_tune_lookup.argtypes = [P, P, I64, P, P]
        F32 = ctypes.c_float
        L.l1line_ranker_features.argtypes = [P, P, I64, I64, I64, D, P, P]
        L.l1line_ranker_signsums.argtypes = [P, P, I64, I64, I64, P, P]
        L.l1line_mlp_forward.argtypes = [P, P, P, I64, P, P]
        L.l1line_mlp_grad.argtypes = [P, P, P, P, I64, P, P, P]
        L.l1line_mlp_adam.argtypes = [P, P, P, P, P, I64, F32, P]
        L.l1line_fit_ranked.argtypes = [P, P, I64, I64, I64, D, I32, D, P, P, P, P, P, P, P, P]
        L.l1line_profile.argtypes = [P, I32]
        L.l1line_measure_peaks.argtypes = [P, P]
        L.l1line_profile_read.argtypes = [P, ctypes.c_char_p, ctypes.POINTER(D),
                                          ctypes.POINTER(I64), I32]
        for f in ("l1line_create", "l1line_destroy", "l1line_column_stats", "l1line_fit", "l1line_fit_noalloc",
                  "l1line_fit_path", "l1line_fit_batch", "l1line_autotune", "l1line_tune_get",
                  "l1line_tune_set", "l1line_profile", "l1line_profile_read", "l1line_ranker_features",
                  "l1line_ranker_signsums", "l1line_mlp_forward", "l1line_mlp_grad", "l1line_mlp_adam",
                  "l1line_fit_ranked",
                  "l1line_last_error", "l1line_ranker_load", "l1line_ranker_save", "l1line_ranker_set_params",
                  "l1line_ranker_get_params", "l1line_ranker_train", "l1line_breakpoints",
                  "l1line_components", "l1line_measure_peaks", "l1line_tune_lookup"):
            getattr(L, f).restype = I32
        _lib = L
    return _lib


def strerror(code: int) -> str:
    try:
        return lib().l1line_strerror(int(code)).decode()
    except RuntimeError:
        return f"status {code}"


def _check(code: int, what: str):
    if code != OK:
        raise L1LineError(code, what)


def _torch():
    import torch
    return torch


def device_matrix(X: np.ndarray, device="cuda:0"):
    """Copy an n x m numpy matrix to a column-major FP64 device tensor
    (strides (1, n)), the layout the library takes."""
    torch = _torch()
    X = np.asfortranarray(np.asarray(X, dtype=np.float64))
    n, m = X.shape
    t = torch.empty_strided((n, m), (1, max(n, 1)), dtype=torch.float64, device=device)
    t.copy_(torch.from_numpy(X))
    return t


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_matrix(X):
    torch = _torch()
    if not isinstance(X, torch.Tensor) or X.dtype != torch.float64 or not X.is_cuda or X.dim() != 2:
        raise TypeError("X must be a 2-D float64 CUDA tensor")
    n, m = X.shape
    if X.stride(0) != 1 or (m > 1 and X.stride(1) < n):
        raise ValueError("X must be column-major: stride(0) == 1, stride(1) >= n")
    ld = X.stride(1) if m > 1 else max(n, 1)
    return n, m, max(ld, n)


class Context:
    """One library context (workspace) on one device."""

    def __init__(self, device: int = 0, tune_cache_path=None):
        torch = _torch()
        self.device = int(device)
        self._torch_device = torch.device("cuda", self.device)
        h = ctypes.c_void_p()
        path = None if tune_cache_path is None else os.fsencode(tune_cache_path)
        _check(lib().l1line_create(ctypes.byref(h), self.device, path), "l1line_create")
        self._h = h

    def last_error(self) -> int:
        """The context's sticky error (then cleared); call after synchronising."""
        return int(lib().l1line_last_error(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().l1line_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def measure_peaks(self):
        """Measured ceilings: dict hbm_GBps, lds_GBps, fp64_valu_TFLOPs,
        fp64_mfma_TFLOPs, bf16_mfma_TFLOPs (l1line_measure_peaks)."""
        out = (ctypes.c_double * 5)()
        _check(lib().l1line_measure_peaks(self._h, ctypes.cast(out, ctypes.c_void_p)), "l1line_measure_peaks")
        return dict(zip(("hbm_GBps", "lds_GBps", "fp64_valu_TFLOPs", "fp64_mfma_TFLOPs", "bf16_mfma_TFLOPs"),
                        list(out)))

    def profile(self, enable: bool):
        _check(lib().l1line_profile(self._h, int(bool(enable))), "l1line_profile")

    def profile_read(self, kernel=None, reset=False):
        """(total ms, launches) of the recorded launches of `kernel`."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        _check(lib().l1line_profile_read(self._h, None if kernel is None else kernel.encode(),
                                         ctypes.byref(ms), ctypes.byref(cnt), int(bool(reset))),
               "l1line_profile_read")
        return ms.value, cnt.value

    def _stream(self):
        return ctypes.c_void_p(_torch().cuda.current_stream(self._torch_device).cuda_stream)

    def _empty(self, shape, dtype):
        return _torch().empty(shape, dtype=dtype, device=self._torch_device)

    def column_stats(self, X):
        """(W [m] fp64, zeros [m] int32, status [1] int32) on the device."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        W = self._empty((m,), torch.float64)
        Z = self._empty((m,), torch.int32)
        st = self._empty((1,), torch.int32)
        _check(lib().l1line_column_stats(self._h, _ptr(X), n, m, ld, _ptr(W), _ptr(Z), _ptr(st),
                                         self._stream()), "l1line_column_stats")
        return W, Z, st

    def fit(self, X, lam: float, rows: bool = True, z_all: bool = True):
        """Algorithm 1 for one penalty: dict of device tensors v, j, obj,
        row, z_all, status."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        out = dict(v=self._empty((m,), torch.float64), j=self._empty((1,), torch.int64),
                   obj=self._empty((1,), torch.float64),
                   row=self._empty((m,), torch.int32) if rows else None,
                   z_all=self._empty((m,), torch.float64) if z_all else None,
                   status=self._empty((1,), torch.int32))
        _check(lib().l1line_fit(self._h, _ptr(X), n, m, ld, float(lam), _ptr(out["v"]), _ptr(out["j"]),
                                _ptr(out["obj"]), _ptr(out["row"]), _ptr(out["z_all"]),
                                _ptr(out["status"]), self._stream()), "l1line_fit")
        return out

    def fit_noalloc(self, X, lam: float, out=None):
        """l1line_fit_noalloc: as fit(), the workspace in the library's fixed
        device array.  `out` (optional): a dict from an earlier call whose
        tensors are reused, so the call itself allocates nothing."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        if out is None:
            out = dict(v=self._empty((m,), torch.float64), j=self._empty((1,), torch.int64),
                       obj=self._empty((1,), torch.float64), row=self._empty((m,), torch.int32),
                       z_all=self._empty((m,), torch.float64), status=self._empty((1,), torch.int32))
        _check(lib().l1line_fit_noalloc(self._h, _ptr(X), n, m, ld, float(lam), _ptr(out["v"]), _ptr(out["j"]),
                                        _ptr(out["obj"]), _ptr(out["row"]), _ptr(out["z_all"]),
                                        _ptr(out["status"]), self._stream()), "l1line_fit_noalloc")
        return out

    def fit_path(self, X, lambdas, rows: bool = True, z_all: bool = True):
        """Algorithm 1 along a path: dict V [L,m], J [L], OBJ [L], ROW [L,m],
        ZALL [L,m], status."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
        L = lam.size
        out = dict(V=self._empty((L, m), torch.float64), J=self._empty((L,), torch.int64),
                   OBJ=self._empty((L,), torch.float64),
                   ROW=self._empty((L, m), torch.int32) if rows else None,
                   ZALL=self._empty((L, m), torch.float64) if z_all else None,
                   status=self._empty((1,), torch.int32))
        _check(lib().l1line_fit_path(self._h, _ptr(X), n, m, ld,
                                     lam.ctypes.data_as(ctypes.c_void_p), L, _ptr(out["V"]),
                                     _ptr(out["J"]), _ptr(out["OBJ"]), _ptr(out["ROW"]),
                                     _ptr(out["ZALL"]), _ptr(out["status"]), self._stream()),
               "l1line_fit_path")
        return out

    # ------------------------------------------------------------- batches
    def _batch_args(self, problems, rows, z_all):
        torch = _torch()
        arr = (Problem * len(problems))()
        outs, keep = [], []
        for q, (X, lambdas) in enumerate(problems):
            n, m, ld = _check_matrix(X)
            lam = np.ascontiguousarray(np.atleast_1d(np.asarray(lambdas, dtype=np.float64)))
            L = lam.size
            o = dict(V=self._empty((L, m), torch.float64), J=self._empty((L,), torch.int64),
                     OBJ=self._empty((L,), torch.float64),
                     ROW=self._empty((L, m), torch.int32) if rows else None,
                     ZALL=self._empty((L, m), torch.float64) if z_all else None,
                     status=self._empty((1,), torch.int32))
            keep.append(lam)
            arr[q] = Problem(X.data_ptr(), n, m, ld, lam.ctypes.data, L, o["V"].data_ptr(),
                             o["J"].data_ptr(), o["OBJ"].data_ptr(),
                             o["ROW"].data_ptr() if rows else None,
                             o["ZALL"].data_ptr() if z_all else None, o["status"].data_ptr())
            outs.append(o)
        return arr, outs, keep

    def fit_batch(self, problems, graph: bool = False, rows: bool = True, z_all: bool = True):
        """problems: list of (X device tensor, lambdas).  Returns one dict per
        problem, as fit_path."""
        arr, outs, keep = self._batch_args(problems, rows, z_all)
        _check(lib().l1line_fit_batch(self._h, ctypes.cast(arr, ctypes.c_void_p), len(problems),
                                      BATCH_GRAPH if graph else 0, self._stream()), "l1line_fit_batch")
        del keep
        return outs

    def fit_batch_prepared(self, arr, n, graph: bool = False):
        """Submit an already built Problem array (reuse of the same layout)."""
        _check(lib().l1line_fit_batch(self._h, ctypes.cast(arr, ctypes.c_void_p), n,
                                      BATCH_GRAPH if graph else 0, self._stream()), "l1line_fit_batch")

    def autotune(self, problems):
        arr, outs, keep = self._batch_args(problems, True, True)
        params = (ctypes.c_int32 * 3)()
        _check(lib().l1line_autotune(self._h, ctypes.cast(arr, ctypes.c_void_p), len(problems),
                                     self._stream(), params), "l1line_autotune")
        return list(params)

    def tune_lookup(self, problems):
        """((workgroups per CU, fewest k per item, items per CU), tuned) a
        call with these problems (list of (X, lambdas)) launches with."""
        arr, outs, keep = self._batch_args(problems, False, False)
        params = (ctypes.c_int32 * 3)()
        tuned = ctypes.c_int32()
        _check(lib().l1line_tune_lookup(self._h, ctypes.cast(arr, ctypes.c_void_p), len(problems),
                                        ctypes.cast(params, ctypes.c_void_p), ctypes.byref(tuned)),
               "l1line_tune_lookup")
        del keep, outs
        return tuple(params), bool(tuned.value)

    def tune_get(self):
        params = (ctypes.c_int32 * 3)()
        _check(lib().l1line_tune_get(self._h, params), "l1line_tune_get")
        return list(params)

    def tune_set(self, params):
        arr = (ctypes.c_int32 * 3)(*[int(x) for x in params])
        _check(lib().l1line_tune_set(self._h, arr), "l1line_tune_set")

    # -------------------------------------------------------------- ranker
    def features(self, X, lam: float):
        """[m, 32] FP32 per-column features (device)."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        F = self._empty((m, FEATURES), torch.float32)
        _check(lib().l1line_ranker_features(self._h, _ptr(X), n, m, ld, float(lam), _ptr(F),
                                            self._stream()), "l1line_ranker_features")
        return F

    def feature_signsums(self, X):
        """[m, m, 2] FP64 (D_jk, Zr_jk) behind the features (device; BF16
        matrix units, error bounds in the header)."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        DZ = self._empty((m, m, 2), torch.float64)
        _check(lib().l1line_ranker_signsums(self._h, _ptr(X), n, m, ld, _ptr(DZ), self._stream()),
               "l1line_ranker_signsums")
        return DZ

    @staticmethod
    def _f32(t, shape=None):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_cuda or \
                not t.is_contiguous():
            raise TypeError("expected a contiguous float32 CUDA tensor")
        if shape is not None and tuple(t.shape) != tuple(shape):
            raise ValueError(f"expected shape {shape}, got {tuple(t.shape)}")
        return t

    def mlp_forward(self, params, F):
        torch = _torch()
        self._f32(params, (MLP_PARAMS,))
        self._f32(F)
        N = F.shape[0]
        out = self._empty((N,), torch.float32)
        _check(lib().l1line_mlp_forward(self._h, _ptr(params), _ptr(F), N, _ptr(out), self._stream()),
               "l1line_mlp_forward")
        return out

    def mlp_grad(self, params, F, y):
        torch = _torch()
        self._f32(params, (MLP_PARAMS,))
        self._f32(F)
        self._f32(y, (F.shape[0],))
        grad = self._empty((MLP_PARAMS,), torch.float32)
        loss = self._empty((1,), torch.float32)
        _check(lib().l1line_mlp_grad(self._h, _ptr(params), _ptr(F), _ptr(y), F.shape[0], _ptr(grad),
                                     _ptr(loss), self._stream()), "l1line_mlp_grad")
        return grad, loss

    def mlp_adam(self, params, m1, m2, grad, step: int, lr: float):
        for t in (params, m1, m2, grad):
            self._f32(t, (MLP_PARAMS,))
        _check(lib().l1line_mlp_adam(self._h, _ptr(params), _ptr(m1), _ptr(m2), _ptr(grad), int(step),
                                     float(lr), self._stream()), "l1line_mlp_adam")

    def fit_ranked(self, X, lam: float, K: int = 32, margin: float = 0.05):
        """Ranked fit with the context's ranker weights."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        out = dict(v=self._empty((m,), torch.float64), j=self._empty((1,), torch.int64),
                   obj=self._empty((1,), torch.float64), row=self._empty((m,), torch.int32),
                   used_fallback=self._empty((1,), torch.int32),
                   scores=self._empty((m,), torch.float32), status=self._empty((1,), torch.int32))
        _check(lib().l1line_fit_ranked(self._h, _ptr(X), n, m, ld, float(lam), int(K), float(margin),
                                       _ptr(out["v"]), _ptr(out["j"]), _ptr(out["obj"]), _ptr(out["row"]),
                                       _ptr(out["used_fallback"]), _ptr(out["scores"]), _ptr(out["status"]),
                                       self._stream()), "l1line_fit_ranked")
        return out

    def breakpoints(self, X):
        """Algorithm 2 for every segment: dict offsets [m*m+1], lambda_max
        [m*m], lam, v, row [total], status (device tensors).  Two calls: the
        first sizes the outputs (one host synchronisation)."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        offsets = self._empty((m * m + 1,), torch.int64)
        lmax = self._empty((m * m,), torch.float64)
        status = self._empty((1,), torch.int32)
        _check(lib().l1line_breakpoints(self._h, _ptr(X), n, m, ld, _ptr(offsets), _ptr(lmax), None, None, None,
                                        0, _ptr(status), self._stream()), "l1line_breakpoints")
        total = int(offsets[-1].item())
        out = dict(offsets=offsets, lambda_max=lmax, lam=self._empty((total,), torch.float64),
                   v=self._empty((total,), torch.float64), row=self._empty((total,), torch.int32), status=status)
        if total > 0:
            _check(lib().l1line_breakpoints(self._h, _ptr(X), n, m, ld, _ptr(offsets), _ptr(lmax), _ptr(out["lam"]),
                                            _ptr(out["v"]), _ptr(out["row"]), total, _ptr(status),
                                            self._stream()), "l1line_breakpoints")
        return out

    def solution_path(self, X, capacity: int | None = None):
        """Algorithm 3: the records of the exact solution path (dict of device
        tensors lam, j, k, v, row, E, P, and count).  Without a capacity the
        library is asked for the count first (two calls)."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        cnt = ctypes.c_int64(0)
        status = self._empty((1,), torch.int32)
        if capacity is None:
            _check(lib().l1line_solution_path(self._h, _ptr(X), n, m, ld, 0, ctypes.byref(cnt), None, None, None,
                                              None, None, None, None, _ptr(status), self._stream()),
                   "l1line_solution_path")
            capacity = cnt.value
        c = max(int(capacity), 1)
        out = dict(lam=self._empty((c,), torch.float64), j=self._empty((c,), torch.int64),
                   k=self._empty((c,), torch.int32), v=self._empty((c,), torch.float64),
                   row=self._empty((c,), torch.int32), E=self._empty((c,), torch.float64),
                   P=self._empty((c,), torch.float64), status=status)
        _check(lib().l1line_solution_path(self._h, _ptr(X), n, m, ld, c, ctypes.byref(cnt), _ptr(out["lam"]),
                                          _ptr(out["j"]), _ptr(out["k"]), _ptr(out["v"]), _ptr(out["row"]),
                                          _ptr(out["E"]), _ptr(out["P"]), _ptr(status), self._stream()),
               "l1line_solution_path")
        out["count"] = cnt.value
        for key in ("lam", "j", "k", "v", "row", "E", "P"):
            out[key] = out[key][:cnt.value]
        return out

    def components(self, X, lam: float, p: int):
        """p successive components: dict V [p, m], J [p], OBJ [p], work (the
        projected data of the last component), status."""
        torch = _torch()
        n, m, ld = _check_matrix(X)
        out = dict(V=self._empty((p, m), torch.float64), J=self._empty((p,), torch.int64),
                   OBJ=self._empty((p,), torch.float64),
                   work=torch.empty_strided((n, m), (1, n), dtype=torch.float64, device=self._torch_device),
                   status=self._empty((1,), torch.int32))
        _check(lib().l1line_components(self._h, _ptr(X), n, m, ld, float(lam), int(p), _ptr(out["work"]),
                                       _ptr(out["V"]), _ptr(out["J"]), _ptr(out["OBJ"]), _ptr(out["status"]),
                                       self._stream()), "l1line_components")
        return out

    def ranker_load(self, path):
        _check(lib().l1line_ranker_load(self._h, os.fsencode(path)), "l1line_ranker_load")

    def ranker_save(self, path):
        _check(lib().l1line_ranker_save(self._h, os.fsencode(path)), "l1line_ranker_save")

    def ranker_set_params(self, params):
        self._f32(params, (MLP_PARAMS,))
        _check(lib().l1line_ranker_set_params(self._h, _ptr(params), self._stream()), "l1line_ranker_set_params")

    def ranker_get_params(self):
        torch = _torch()
        out = self._empty((MLP_PARAMS,), torch.float32)
        _check(lib().l1line_ranker_get_params(self._h, _ptr(out), self._stream()), "l1line_ranker_get_params")
        return out

    def ranker_train(self, steps: int, seed: int = 0, ckpt_path=None):
        """Native training loop (synchronous, default stream)."""
        _torch().cuda.synchronize(self._torch_device)
        path = None if ckpt_path is None else os.fsencode(ckpt_path)
        _check(lib().l1line_ranker_train(self._h, path, int(steps), int(seed) & 0xFFFFFFFFFFFFFFFF),
               "l1line_ranker_train")


def write_ranker_file(path, params):
    """Write FP32 weights (numpy, L1LINE_MLP_PARAMS) in the library's ranker
    file format (no optimizer state): "L1RK", version 1, count, flags 0,
    step 0, seed 0, next example 0, then the weights."""
    import struct
    w = np.ascontiguousarray(np.asarray(params, dtype="<f4"))
    if w.shape != (MLP_PARAMS,):
        raise ValueError("expected %d weights" % MLP_PARAMS)
    with open(path, "wb") as f:
        f.write(b"L1RK" + struct.pack("<IIIqQQ", 1, MLP_PARAMS, 0, 0, 0, 0))
        f.write(w.tobytes())


def read_ranker_file(path):
    """(weights, state or None, header dict) of a ranker file, numpy only."""
    import struct
    with open(path, "rb") as f:
        head = f.read(40)
        if len(head) != 40 or head[:4] != b"L1RK":
            raise ValueError("not a ranker file")
        ver, cnt, flags, step, seed, cursor = struct.unpack("<IIIqQQ", head[4:])
        if ver != 1 or cnt != MLP_PARAMS or flags & ~1:
            raise ValueError("unsupported ranker file")
        data = np.frombuffer(f.read(), dtype="<f4")
    k = 3 if flags & 1 else 1
    if data.size != k * MLP_PARAMS:
        raise ValueError("truncated ranker file")
    w = data[:MLP_PARAMS].copy()
    state = (data[MLP_PARAMS:2 * MLP_PARAMS].copy(), data[2 * MLP_PARAMS:].copy()) if k == 3 else None
    return w, state, dict(step=step, seed=seed, cursor=cursor)
