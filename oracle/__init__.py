"""CPU oracle for the conversion matvec beta = A alpha.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct reference
implementations written from the paper (Townsend, Webb, Olver,
arXiv:1604.07486).  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the GPU library
never does, and this package never imports the GPU library.

Contents
--------
* ``matvec`` / ``dense`` -- O(N^2) beta = A alpha from the closed-form entries
  (``oracle.c``: eq. (M), eq. (FormulaL), eq. (UltraSconversion), the Jacobi
  case-2 formula of Sec. 5.3 and the Laguerre formula of Sec. 5.4).
* ``jac2jac`` / ``jac2cheb`` -- the general Jacobi conversion assembled the way
  Sec. 5.3 describes: a change of the second parameter through the reflection
  P_k^{(a,b)}(-x) = (-1)^k P_k^{(b,a)}(x), then a change of the first one, and
  for Chebyshev targets the normalisation T_k = P_k^{(-1/2,-1/2)}/P_k^{(-1/2,-1/2)}(1).
* ``jacobi_step`` / ``jac2jac_rows`` / ``jac2cheb_rows`` -- the whole-number
  change of the first Jacobi parameter (Sec. 5.3, case 1) by its bidiagonal
  factor in O(N), and a sampled-row Jacobi conversion that takes that step first
  (the expansion in the target basis is unique, so the order of the steps does
  not change the result): the reference for long vectors.
* ``pivoted_cholesky`` -- the O(K^2 N) pivoted Cholesky of Sec. 2.1 (Fig. 3),
  in numpy float64, used to check the GPU factorisation's invariants.

Parity status: every function here is pinned by ``tests/test_oracle_pins.py``
(exact rational basis changes, extended-precision polynomial evaluation,
mpmath values of Lambda, and the invariants of Sec. 2.1).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

KINDS = {"leg2cheb": 0, "cheb2leg": 1, "ultra2ultra": 2, "jac2jac_b": 3, "lag2lag": 4}

_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, OpenMP, libquadmath)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", SRC_PATH,
             "-lquadmath", "-o", tmp])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i64, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
        lib.orc_matvec.argtypes = [ctypes.c_int, dp, i64, dp, dp,
                                   ctypes.POINTER(ctypes.c_int64), i64, ctypes.c_int]
        lib.orc_matvec.restype = ctypes.c_int
        lib.orc_matvec_abs.argtypes = lib.orc_matvec.argtypes
        lib.orc_matvec_abs.restype = ctypes.c_int
        lib.orc_dense.argtypes = [ctypes.c_int, dp, i64, dp]
        lib.orc_dense.restype = ctypes.c_int
        lib.orc_absmax.argtypes = [ctypes.c_int, dp, i64]
        lib.orc_absmax.restype = ctypes.c_double
        lib.orc_lambda.argtypes = [i64, dp]
        lib.orc_lambda.restype = ctypes.c_int
        lib.orc_lambda_str.argtypes = [i64, ctypes.c_char_p, ctypes.c_int]
        lib.orc_lambda_str.restype = ctypes.c_int
        lib.orc_jacobi_step.argtypes = [ctypes.c_double, ctypes.c_double, i64, dp, dp, ctypes.c_int]
        lib.orc_jacobi_step.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _params(kind: str, params) -> np.ndarray:
    p = np.zeros(4, dtype=np.float64)
    for i, v in enumerate(params or ()):
        p[i] = float(v)
    return p


def matvec(kind: str, alpha, params=(), rows=None, nthreads: int = 0, absolute: bool = False) -> np.ndarray:
    """beta = A alpha (all rows, or only ``rows``) for one coefficient vector.

    kind: 'leg2cheb', 'cheb2leg', 'ultra2ultra' (params l1, l2), 'jac2jac_b'
    (params a, b, g: Jacobi (a,b) -> (g,b)), 'lag2lag' (params a1, a2).
    absolute: return |A| |alpha| instead (the rounding scale of each row, for
    error bars).
    """
    lib = _load()
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    N = a.shape[0] - 1
    p = _params(kind, params)
    if rows is None:
        out = np.empty(N + 1, dtype=np.float64)
        rp, nr = None, 0
    else:
        r = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.empty(r.shape[0], dtype=np.float64)
        rp, nr = r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), r.shape[0]
    fn = lib.orc_matvec_abs if absolute else lib.orc_matvec
    rc = fn(KINDS[kind], _dptr(p), N, _dptr(a), _dptr(out), rp, nr, int(nthreads))
    if rc != 0:
        raise ValueError(f"oracle matvec failed (rc={rc}) for {kind} {params} N={N}")
    return out


def dense(kind: str, N: int, params=()) -> np.ndarray:
    """The full (N+1)x(N+1) conversion matrix A (small N only)."""
    lib = _load()
    A = np.empty((N + 1, N + 1), dtype=np.float64)
    rc = lib.orc_dense(KINDS[kind], _dptr(_params(kind, params)), N, _dptr(A))
    if rc != 0:
        raise ValueError(f"oracle dense failed (rc={rc})")
    return A


def absmax(kind: str, N: int, params=()) -> float:
    """max_{j,k} |A_jk| of the (N+1)x(N+1) conversion matrix (O(N^2))."""
    v = _load().orc_absmax(KINDS[kind], _dptr(_params(kind, params)), N)
    if v < 0:
        raise ValueError("orc_absmax failed")
    return float(v)


def lambda_table(M: int) -> np.ndarray:
    """Lambda(n) = Gamma(n+1/2)/Gamma(n+1), n = 0..M (binary128, rounded)."""
    out = np.empty(M + 1, dtype=np.float64)
    if _load().orc_lambda(M, _dptr(out)) != 0:
        raise ValueError("orc_lambda failed")
    return out


def lambda_str(n: int) -> str:
    """Lambda(n) to 34 significant digits."""
    buf = ctypes.create_string_buffer(64)
    if _load().orc_lambda_str(n, buf, 64) != 0:
        raise ValueError("orc_lambda_str failed")
    return buf.value.decode()


# --------------------------------------------------------------------------
# General Jacobi conversions (Sec. 5.3) assembled from the beta = delta kernel
# --------------------------------------------------------------------------

def jac2jac(alpha, a: float, b: float, g: float, d: float, rows=None) -> np.ndarray:
    """Coefficients in P^{(g,d)} of sum_k alpha_k P_k^{(a,b)}.

    When b != d the second parameter is changed first (Sec. 5.3, footnote): by
    the reflection P_k^{(a,b)}(-x) = (-1)^k P_k^{(b,a)}(x), the conversion
    (a,b) -> (a,d) equals R A[(b,a) -> (d,a)] R with R = diag((-1)^k).
    """
    x = np.ascontiguousarray(alpha, dtype=np.float64)
    if b != d:
        sgn = np.where(np.arange(x.shape[0]) % 2 == 0, 1.0, -1.0)
        x = sgn * matvec("jac2jac_b", sgn * x, (b, a, d))
    if a == g:
        return x if rows is None else x[np.asarray(rows)]
    return matvec("jac2jac_b", x, (a, d, g), rows=rows)


def cheb_norm(N: int) -> np.ndarray:
    """P_k^{(-1/2,-1/2)}(1) = (1/2)_k / k! = Lambda(k)/sqrt(pi), k = 0..N."""
    return lambda_table(N) / np.sqrt(np.pi)


def jac2cheb(alpha, a: float, b: float) -> np.ndarray:
    """Chebyshev coefficients of sum_k alpha_k P_k^{(a,b)} (Sec. 5.3, last part)."""
    x = np.ascontiguousarray(alpha, dtype=np.float64)
    y = jac2jac(x, a, b, -0.5, -0.5)
    return y * cheb_norm(x.shape[0] - 1)


def cheb2jac(alpha, g: float, d: float) -> np.ndarray:
    """Coefficients in P^{(g,d)} of sum_k alpha_k T_k: T_k = P_k^{(-1/2,-1/2)} / P_k^{(-1/2,-1/2)}(1)."""
    x = np.ascontiguousarray(alpha, dtype=np.float64)
    return jac2jac(x / cheb_norm(x.shape[0] - 1), -0.5, -0.5, g, d)


def jacobi_step(alpha, a: float, b: float, up: bool) -> np.ndarray:
    """Coefficients in P^(a+1,b) (up) or P^(a-1,b) (down) of sum_k alpha_k P_k^(a,b).

    Sec. 5.3, case 1: the upper-bidiagonal factor S_(a,b) of the textbook
    connection relation, applied directly for a rise and by backward
    substitution for a drop; O(N) in binary128 (``orc_jacobi_step``).
    """
    x = np.ascontiguousarray(alpha, dtype=np.float64)
    out = np.empty_like(x)
    rc = _load().orc_jacobi_step(float(a), float(b), x.shape[0] - 1, _dptr(x), _dptr(out), 1 if up else -1)
    if rc != 0:
        raise ValueError(f"orc_jacobi_step failed (rc={rc}) for a={a} b={b}")
    return out


def jac2jac_rows(alpha, a: float, b: float, g: float, d: float, rows) -> np.ndarray:
    """Rows ``rows`` of the coefficients in P^(g,d) of sum_k alpha_k P_k^(a,b), a - g whole.

    The first parameter moves a -> g in unit steps (Sec. 5.3, case 1, O(N) per
    step), then the second b -> d through the reflection of Sec. 5.3 with the
    case-2 closed form evaluated on the requested rows only.  Sec. 5.3 takes the
    other order (second parameter first); the expansion is unique, so both
    orders give the same coefficients.
    """
    x = np.ascontiguousarray(alpha, dtype=np.float64)
    steps = g - a
    if steps != round(steps):
        raise ValueError("jac2jac_rows needs a whole-number change of the first parameter")
    cur = a
    for _ in range(int(abs(round(steps)))):
        up = g > cur
        x = jacobi_step(x, cur, b, up)
        cur = cur + 1.0 if up else cur - 1.0
    rows = np.asarray(rows, dtype=np.int64)
    if b == d:
        return x[rows]
    sgn = np.where(np.arange(x.shape[0]) % 2 == 0, 1.0, -1.0)
    y = matvec("jac2jac_b", sgn * x, (b, g, d), rows=rows)
    return np.where(rows % 2 == 0, 1.0, -1.0) * y


def jac2cheb_rows(alpha, a: float, b: float, rows) -> np.ndarray:
    """Rows ``rows`` of the Chebyshev coefficients of sum_k alpha_k P_k^(a,b), a + 1/2 whole."""
    rows = np.asarray(rows, dtype=np.int64)
    y = jac2jac_rows(alpha, a, b, -0.5, -0.5, rows)
    return y * cheb_norm(np.asarray(alpha).shape[0] - 1)[rows]


# --------------------------------------------------------------------------
# Pivoted Cholesky of a PSD matrix given by columns (Sec. 2.1, Fig. 3)
# --------------------------------------------------------------------------

def pivoted_cholesky(column, diag: np.ndarray, tol: float, kmax: int | None = None):
    """Greedy diagonal-pivoted Cholesky touching only K columns (Fig. 3).

    column(p) returns column p of the PSD matrix H; diag is its diagonal.
    Stops when the largest residual diagonal entry is <= tol * max(diag(H))
    (the paper's "sufficiently small", read relative to the largest entry of H).
    Returns (pivots, a, ells) with H ~= sum_r ells[r] ells[r]^T / a[r]: the
    update subtracts ell_j (ell_j)_{p_r} / a_j from the new column, which is the
    Schur-complement step of eq. (FirstCholeskyStep) applied to column p_r.
    """
    d = np.array(diag, dtype=np.float64)
    n = d.shape[0]
    kmax = n if kmax is None else min(kmax, n)
    dmax0 = float(d.max()) if n else 0.0
    piv, avals, ells = [], [], []
    while len(piv) < kmax:
        p = int(np.argmax(d))
        if not d[p] > tol * dmax0:
            break
        ell = np.array(column(p), dtype=np.float64)
        for lj, aj in zip(ells, avals):
            ell -= lj * (lj[p] / aj)
        a = ell[p]
        d -= ell * ell / a
        d[p] = 0.0
        np.maximum(d, 0.0, out=d)
        piv.append(p)
        avals.append(a)
        ells.append(ell)
    return np.array(piv, dtype=np.int64), np.array(avals), np.array(ells).reshape(len(piv), n)
