"""ctypes binding of libthx (include/thx.h) -- argument marshalling only.

Every function here forwards to the C entry point of the same name; tensors
are passed as device pointers and the current torch stream as the hipStream_t.
There is no fallback: if libthx.so is missing or fails to load, the import of
this module raises.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libthx.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
_lib = ctypes.CDLL(LIB_PATH)

# enums (include/thx.h)
LEG2CHEB, CHEB2LEG, ULTRA2ULTRA, JAC2JAC, LAG2LAG, JAC2CHEB, CHEB2JAC = 0, 1, 2, 3, 4, 5, 6
FP64, FP32_BULK, FP64_TAIL32 = 0, 1, 2
FLAG_FORCE_DIRECT, FLAG_FORCE_FFT, FLAG_NO_DENSE, FLAG_AUTOTUNE = 1, 2, 4, 8
PHASES = ["pack", "toep_lds", "col_fwd", "row", "col_inv", "row0", "unpack", "direct", "dense", "scan"]
STATUS = {0: "THX_OK", 1: "THX_INVALID_ARGUMENT", 2: "THX_UNSUPPORTED", 3: "THX_TOL_NOT_REACHED",
          4: "THX_OUT_OF_MEMORY", 5: "THX_HIP_ERROR", 6: "THX_WORKSPACE_TOO_LARGE"}

_i64, _i32, _dbl, _vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_p64 = ctypes.POINTER(ctypes.c_int64)


def _sig(name, res, *args):
    f = getattr(_lib, name)
    f.restype = res
    f.argtypes = list(args)
    return f


_sig("thx_plan_create", ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, _dp, ctypes.c_int, _i64, _dbl,
     ctypes.c_int, ctypes.c_uint32, _vp)
_sig("thx_execute", ctypes.c_int, _vp, _vp, _vp, _i64, _i64, _i64, _vp)
_sig("thx_plan_destroy", ctypes.c_int, _vp)
_sig("thx_plan_rank", _i32, _vp)
_sig("thx_plan_rank_part", _i32, _vp, ctypes.c_int)
_sig("thx_plan_fft_length", _i64, _vp)
_sig("thx_plan_path", _i32, _vp)
_sig("thx_plan_fft_geometry", ctypes.c_int, _vp, _p64, _p64, _p64)
_sig("thx_plan_autotune", ctypes.c_int, _vp, _i64, _vp)
_sig("thx_plan_launch_shape", ctypes.c_int, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_sig("thx_plan_lds_radix", _i32, _vp)
_sig("thx_plan_p1_blocks", _i32, _vp)
_sig("thx_plan_fused_columns", _i32, _vp)
_sig("thx_plan_tail_slots", _i32, _vp)
_sig("thx_plan_partial_groups", _i32, _vp, _i64)
_sig("thx_plan_achieved_tol", _dbl, _vp, ctypes.c_int)
_sig("thx_plan_factors", ctypes.c_int, _vp, ctypes.c_int, _dp, ctypes.POINTER(_i32),
     ctypes.POINTER(_i64), _vp)
_sig("thx_leg2cheb", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, ctypes.c_int, _vp)
_sig("thx_cheb2leg", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, ctypes.c_int, _vp)
_sig("thx_ultra2ultra", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, _dbl, _dbl, ctypes.c_int, _vp)
_sig("thx_lag2lag", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, _dbl, _dbl, ctypes.c_int, _vp)
_sig("thx_jac2jac", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, _dbl, _dbl, _dbl, _dbl, ctypes.c_int, _vp)
_sig("thx_jac2cheb", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, _dbl, _dbl, ctypes.c_int, _vp)
_sig("thx_cheb2jac", ctypes.c_int, _vp, _vp, _i64, _i64, _dbl, _dbl, _dbl, ctypes.c_int, _vp)
_sig("thx_execute_varlen", ctypes.c_int, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _vp)
_sig("thx_execute_noalloc", ctypes.c_int, _vp, _vp, _vp, _i64, _i64, _i64, _vp)
_sig("thx_noalloc_scratch_bytes", _i64)
_sig("thx_trace_marker", ctypes.c_int, ctypes.c_int, _vp)
_sig("thx_cache_clear", ctypes.c_int)
_sig("thx_lambda_table", ctypes.c_int, _vp, _i64, _dbl, _vp)
_sig("thx_gamma_ratio_table", ctypes.c_int, _vp, _i64, _dbl, _dbl, _dbl, _vp)
_sig("thx_plan_enable_timing", ctypes.c_int, _vp, ctypes.c_uint32)
_sig("thx_plan_timings", ctypes.c_int, _vp, _dp, ctypes.POINTER(_i64), ctypes.c_int)
_sig("thx_batch_create", ctypes.c_int, ctypes.POINTER(_vp), ctypes.c_int, _dp, ctypes.c_int,
     ctypes.POINTER(_i64), _i64, _dbl, ctypes.c_int, ctypes.c_uint32, _vp)
_sig("thx_batch_execute", ctypes.c_int, _vp, _vp, _vp, ctypes.c_int, _vp)
_sig("thx_batch_destroy", ctypes.c_int, _vp)
_sig("thx_batch_coefficients", _i64, _vp)
_sig("thx_batch_buckets", _i32, _vp)
_sig("thx_batch_bucket_info", ctypes.c_int, _vp, ctypes.c_int, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
     ctypes.POINTER(_i64), ctypes.POINTER(_i32), ctypes.POINTER(_i32))
_sig("thx_status_string", ctypes.c_char_p, ctypes.c_int)
_sig("thx_last_hip_error", ctypes.c_int)   # hipError_t (an enum of int size)


class ThxError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)} (hip error {_lib.thx_last_hip_error()})")


def _check(st: int, where: str, allow=(0,)) -> int:
    if st not in allow:
        raise ThxError(st, where)
    return st


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_tensor(t, name):
    import torch
    if not (t.is_cuda and t.dtype == torch.float64):
        raise TypeError(f"{name} must be a float64 tensor on the GPU")


class Plan:
    """Owns a thx_plan* (thx_plan_create / thx_plan_destroy)."""

    def __init__(self, kind: int, degree: int, tol: float, prec: int = FP64, params=(), flags: int = 0,
                 stream=None):
        self._h = _vp()
        arr = (ctypes.c_double * max(1, len(params)))(*params)
        self.status = _check(_lib.thx_plan_create(ctypes.byref(self._h), kind, arr, len(params), degree, tol,
                                                  prec, flags, _stream(stream)), "thx_plan_create", (0, 3))
        self.kind, self.degree, self.tol, self.prec = kind, degree, tol, prec

    def __del__(self):
        h = getattr(self, "_h", None)
        if _lib is None:  # interpreter shutdown: the process exit releases the device memory
            return
        if h is not None and h.value:
            _lib.thx_plan_destroy(h)
            self._h = _vp()

    @property
    def handle(self):
        return self._h

    rank = property(lambda self: _lib.thx_plan_rank(self._h))
    fft_length = property(lambda self: _lib.thx_plan_fft_length(self._h))
    path = property(lambda self: _lib.thx_plan_path(self._h))

    def autotune(self, batch: int, stream=None):
        """Choose launch shapes / dense vs FFT for executions of `batch` vectors."""
        _check(_lib.thx_plan_autotune(self._h, int(batch), _stream(stream)), "thx_plan_autotune")
        return self

    def launch_shape(self):
        """(lds_blocks, p3_blocks): workgroups targeted per launch (set by autotune)."""
        a, c = _i32(), _i32()
        _check(_lib.thx_plan_launch_shape(self._h, ctypes.byref(a), ctypes.byref(c)), "thx_plan_launch_shape")
        return a.value, c.value

    @property
    def p1_blocks(self) -> int:
        """Workgroups targeted per forward column pass (0: one per tile, slot and vector)."""
        return int(_lib.thx_plan_p1_blocks(self._h))

    @property
    def fused_columns(self) -> bool:
        """True if the forward column pass runs inside the row pass (columns of 2 or 4)."""
        return int(_lib.thx_plan_fused_columns(self._h)) == 1

    @property
    def tail_slots(self) -> int:
        """FFT slots run in single precision (FP64_TAIL32 plans; 0 otherwise)."""
        return int(_lib.thx_plan_tail_slots(self._h))

    @property
    def lds_radix(self) -> int:
        """Largest FFT radix of the single-workgroup path (set by autotune)."""
        return int(_lib.thx_plan_lds_radix(self._h))

    def partial_groups(self, batch: int = 1) -> int:
        return int(_lib.thx_plan_partial_groups(self._h, int(batch)))

    def fft_geometry(self):
        """(rows, cols, tile_cols) of the three-pass FFT (path 2 only)."""
        r, c, t = _i64(), _i64(), _i64()
        _check(_lib.thx_plan_fft_geometry(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(t)),
               "thx_plan_fft_geometry")
        return r.value, c.value, t.value

    def rank_part(self, part: int) -> int:
        return _lib.thx_plan_rank_part(self._h, part)

    def achieved_tol(self, part: int) -> float:
        return _lib.thx_plan_achieved_tol(self._h, part)

    def factors(self, part: int, stream=None):
        """(ell [K, n] normalised Cholesky columns, pivots [K]) of Hankel part `part`."""
        import numpy as np
        n = _i64()
        _check(_lib.thx_plan_factors(self._h, part, None, None, ctypes.byref(n), _stream(stream)), "thx_plan_factors")
        K = self.rank_part(part)
        ell = np.zeros((max(K, 0), n.value), dtype=np.float64)
        piv = np.zeros(max(K, 1), dtype=np.int32)
        _check(_lib.thx_plan_factors(self._h, part, ell.ctypes.data_as(_dp),
                                     piv.ctypes.data_as(ctypes.POINTER(_i32)), ctypes.byref(n),
                                     _stream(stream)), "thx_plan_factors")
        return ell, piv[:max(K, 0)]

    def enable_timing(self, on: bool = True, phases=None):
        """Time every phase (phases=None) or only the named ones (names from PHASES)."""
        mask = 0
        if on:
            mask = (1 << len(PHASES)) - 1 if phases is None else sum(1 << PHASES.index(p) for p in set(phases))
        _check(_lib.thx_plan_enable_timing(self._h, mask), "thx_plan_enable_timing")

    def timings(self, reset: bool = True):
        """{phase: (total_ms, launches)} of the timed executions since the last reset."""
        n = len(PHASES)
        ms = (ctypes.c_double * n)()
        cnt = (_i64 * n)()
        _check(_lib.thx_plan_timings(self._h, ms, cnt, 1 if reset else 0), "thx_plan_timings")
        return {PHASES[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i]}

    def execute(self, alpha, beta, degree=None, stream=None):
        """thx_execute on [batch][ld] (or [N+1]) float64 device tensors."""
        _check_tensor(alpha, "alpha")
        _check_tensor(beta, "beta")
        N = self.degree if degree is None else degree
        a2 = alpha if alpha.dim() == 2 else alpha.view(1, -1)
        b2 = beta if beta.dim() == 2 else beta.view(1, -1)
        if a2.stride(1) != 1 or b2.stride(1) != 1 or a2.stride(0) != b2.stride(0) or a2.shape != b2.shape:
            raise ValueError("alpha and beta must share shape and row stride, unit column stride")
        _check(_lib.thx_execute(self._h, _ptr(a2), _ptr(b2), N, a2.shape[0], a2.stride(0), _stream(stream)),
               "thx_execute")
        return beta

    def execute_noalloc(self, alpha, beta, degree=None, stream=None):
        """thx_execute_noalloc (workspace in the library's static scratch) on [batch][ld] tensors."""
        _check_tensor(alpha, "alpha")
        _check_tensor(beta, "beta")
        N = self.degree if degree is None else degree
        a2 = alpha if alpha.dim() == 2 else alpha.view(1, -1)
        b2 = beta if beta.dim() == 2 else beta.view(1, -1)
        if a2.stride(1) != 1 or b2.stride(1) != 1 or a2.stride(0) != b2.stride(0) or a2.shape != b2.shape:
            raise ValueError("alpha and beta must share shape and row stride, unit column stride")
        _check(_lib.thx_execute_noalloc(self._h, _ptr(a2), _ptr(b2), N, a2.shape[0], a2.stride(0),
                                        _stream(stream)), "thx_execute_noalloc")
        return beta

    def execute_varlen(self, alpha, beta, offsets, skipped=None, stream=None):
        """thx_execute_varlen: members alpha[offsets[i]:offsets[i+1]] (offsets: int64 device tensor
        of count + 1 entries; skipped: optional int64 device tensor of one entry, added to)."""
        import torch
        _check_tensor(alpha, "alpha")
        _check_tensor(beta, "beta")
        if not (offsets.is_cuda and offsets.dtype == torch.int64 and offsets.is_contiguous()):
            raise TypeError("offsets must be a contiguous int64 tensor on the GPU")
        if not alpha.is_contiguous() or not beta.is_contiguous() or alpha.numel() != beta.numel():
            raise ValueError("contiguous alpha/beta of equal size required")
        if skipped is not None and not (skipped.is_cuda and skipped.dtype == torch.int64):
            raise TypeError("skipped must be an int64 tensor on the GPU")
        _check(_lib.thx_execute_varlen(self._h, _ptr(alpha), _ptr(beta), _ptr(offsets), offsets.numel() - 1,
                                       alpha.numel(), _ptr(skipped) if skipped is not None else None,
                                       _stream(stream)), "thx_execute_varlen")
        return beta


class Batch:
    """Owns a thx_batch* (thx_batch_create / thx_batch_destroy): mixed degrees, CSR layout."""

    def __init__(self, kind: int, degrees, tol: float, prec: int = FP64, params=(), flags: int = 0,
                 stream=None):
        import numpy as np
        self.degrees = np.ascontiguousarray(degrees, dtype=np.int64)
        self._h = _vp()
        arr = (ctypes.c_double * max(1, len(params)))(*params)
        self.status = _check(_lib.thx_batch_create(
            ctypes.byref(self._h), kind, arr, len(params),
            self.degrees.ctypes.data_as(ctypes.POINTER(_i64)), len(self.degrees), tol, prec, flags,
            _stream(stream)), "thx_batch_create", (0, 3))
        self.offsets = np.concatenate([[0], np.cumsum(self.degrees + 1)]).astype(np.int64)

    def __del__(self):
        h = getattr(self, "_h", None)
        if _lib is None:  # interpreter shutdown: the process exit releases the device memory
            return
        if h is not None and h.value:
            _lib.thx_batch_destroy(h)
            self._h = _vp()

    coefficients = property(lambda self: _lib.thx_batch_coefficients(self._h))

    def buckets(self):
        out = []
        for i in range(_lib.thx_batch_buckets(self._h)):
            L, m, nmax = _i64(), _i64(), _i64()
            path, rank = _i32(), _i32()
            _check(_lib.thx_batch_bucket_info(self._h, i, ctypes.byref(L), ctypes.byref(m), ctypes.byref(nmax),
                                              ctypes.byref(path), ctypes.byref(rank)), "thx_batch_bucket_info")
            out.append({"L": L.value, "members": m.value, "max_degree": nmax.value, "path": path.value,
                        "rank": rank.value})
        return out

    def execute(self, alpha, beta, graph: bool = False, stream=None):
        _check_tensor(alpha, "alpha")
        _check_tensor(beta, "beta")
        n = int(self.offsets[-1])
        if alpha.numel() < n or beta.numel() < n or not alpha.is_contiguous() or not beta.is_contiguous():
            raise ValueError("alpha / beta must be contiguous with sum(degree+1) entries")
        _check(_lib.thx_batch_execute(self._h, _ptr(alpha), _ptr(beta), 1 if graph else 0, _stream(stream)),
               "thx_batch_execute")
        return beta


def thx_execute(plan: Plan, alpha, beta, degree=None, stream=None):
    return plan.execute(alpha, beta, degree, stream)


def _oneshot(fname, alpha, beta, *args, stream=None):
    _check_tensor(alpha, "alpha")
    _check_tensor(beta, "beta")
    a2 = alpha if alpha.dim() == 2 else alpha.view(1, -1)
    if not a2.is_contiguous() or not beta.is_contiguous() or beta.numel() != a2.numel():
        raise ValueError("contiguous alpha/beta of equal size required")
    N = a2.shape[1] - 1
    _check(getattr(_lib, fname)(_ptr(a2), _ptr(beta), N, a2.shape[0], *args, _stream(stream)), fname)
    return beta


def thx_leg2cheb(alpha, beta, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_leg2cheb", alpha, beta, tol, prec, stream=stream)


def thx_cheb2leg(alpha, beta, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_cheb2leg", alpha, beta, tol, prec, stream=stream)


def thx_ultra2ultra(alpha, beta, lambda1, lambda2, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_ultra2ultra", alpha, beta, lambda1, lambda2, tol, prec, stream=stream)


def thx_lag2lag(alpha, beta, alpha1, alpha2, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_lag2lag", alpha, beta, alpha1, alpha2, tol, prec, stream=stream)


def thx_jac2jac(alpha, beta, a, b, g, d, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_jac2jac", alpha, beta, a, b, g, d, tol, prec, stream=stream)


def thx_jac2cheb(alpha, beta, a, b, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_jac2cheb", alpha, beta, a, b, tol, prec, stream=stream)


def thx_cheb2jac(alpha, beta, g, d, tol=1e-15, prec=FP64, stream=None):
    return _oneshot("thx_cheb2jac", alpha, beta, g, d, tol, prec, stream=stream)


def thx_cache_clear():
    return _check(_lib.thx_cache_clear(), "thx_cache_clear")


def thx_lambda_table(out, z0=0.0, stream=None):
    _check_tensor(out, "out")
    _check(_lib.thx_lambda_table(_ptr(out), out.numel(), z0, _stream(stream)), "thx_lambda_table")
    return out


def thx_gamma_ratio_table(out, a, b, z0=0.0, stream=None):
    _check_tensor(out, "out")
    _check(_lib.thx_gamma_ratio_table(_ptr(out), out.numel(), z0, a, b, _stream(stream)), "thx_gamma_ratio_table")
    return out


def thx_trace_marker(marker_id: int, stream=None):
    """Empty kernel with marker_id workgroups of 64 threads (cuts kernel traces into regions)."""
    return _check(_lib.thx_trace_marker(int(marker_id), _stream(stream)), "thx_trace_marker")


def thx_status_string(s: int) -> str:
    return _lib.thx_status_string(s).decode()


def raw_library():
    """The loaded ctypes.CDLL (for tests of the C ABI)."""
    return _lib
