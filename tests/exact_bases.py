"""Exact (rational) orthogonal-polynomial bases for pinning the oracle.

Independent of the paper's closed forms: every basis is built in the monomial
basis with Python ``fractions`` from the textbook three-term recurrences
(DLMF 18.9.1 and Table 18.9.1 / 18.9.2), and a conversion matrix is obtained by
an exact triangular solve.  Also extended-precision (mpmath) evaluation of the
same recurrences at arbitrary points for larger degrees.
"""
from __future__ import annotations

from fractions import Fraction as F

import mpmath


def _mul_x(p):
    return [F(0)] + list(p)


def _axpy(a, x, y):
    n = max(len(x), len(y))
    out = [F(0)] * n
    for i, v in enumerate(x):
        out[i] += a * v
    for i, v in enumerate(y):
        out[i] += v
    return out


def _scale(a, x):
    return [a * v for v in x]


def basis(family: str, N: int, params=()):
    """Monomial coefficients (lowest first) of phi_0..phi_N as Fractions."""
    P = []
    if family == "cheb":
        P = [[F(1)], [F(0), F(1)]]
        for n in range(1, N):
            P.append(_axpy(F(-1), P[n - 1] + [F(0)] * 2, _scale(F(2), _mul_x(P[n]))))
    elif family == "leg":
        P = [[F(1)], [F(0), F(1)]]
        for n in range(1, N):
            # (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1}
            t = _axpy(F(-n), P[n - 1], _scale(F(2 * n + 1), _mul_x(P[n])))
            P.append(_scale(F(1, n + 1), t))
    elif family == "ultra":
        lam = F(params[0])
        P = [[F(1)], [F(0), 2 * lam]]
        for n in range(1, N):
            # (n+1) C_{n+1} = 2 (n+lam) x C_n - (n + 2 lam - 1) C_{n-1}
            t = _axpy(-(n + 2 * lam - 1), P[n - 1], _scale(2 * (n + lam), _mul_x(P[n])))
            P.append(_scale(F(1) / (n + 1), t))
    elif family == "jacobi":
        a, b = F(params[0]), F(params[1])
        # P_1 = (a+1) + (a+b+2)(x-1)/2
        P = [[F(1)], [(a + 1) - (a + b + 2) / 2, (a + b + 2) / 2]]
        for n in range(1, N):
            s = 2 * n + a + b
            c1 = 2 * (n + 1) * (n + a + b + 1) * s
            c2 = (s + 1) * (a * a - b * b)
            c3 = (s + 1) * (s + 2) * s
            c4 = 2 * (n + a) * (n + b) * (s + 2)
            t = _axpy(c2, P[n], _scale(c3, _mul_x(P[n])))
            t = _axpy(-c4, P[n - 1], t)
            P.append(_scale(F(1) / c1, t))
    elif family == "laguerre":
        a = F(params[0])
        P = [[F(1)], [1 + a, F(-1)]]
        for n in range(1, N):
            # (n+1) L_{n+1} = (2n + a + 1 - x) L_n - (n + a) L_{n-1}
            t = _axpy(F(2 * n + 1) + a, P[n], _scale(F(-1), _mul_x(P[n])))
            t = _axpy(-(n + a), P[n - 1], t)
            P.append(_scale(F(1, n + 1), t))
    else:
        raise ValueError(family)
    P = P[: N + 1]
    return [p + [F(0)] * (N + 1 - len(p)) for p in P]


def conversion(src, dst, N: int):
    """Exact A with phi_k = sum_j A_jk psi_j (phi = src basis, psi = dst basis)."""
    A = [[F(0)] * (N + 1) for _ in range(N + 1)]
    for k in range(N + 1):
        r = list(src[k])
        for j in range(k, -1, -1):
            c = r[j] / dst[j][j]
            A[j][k] = c
            if c:
                for i in range(j + 1):
                    r[i] -= c * dst[j][i]
        assert all(v == 0 for v in r)
    return A


def eval_recurrence(family: str, coeffs, x, params=(), dps: int = 40):
    """sum_k coeffs[k] phi_k(x) in mpmath at `dps` digits via the recurrence."""
    with mpmath.workdps(dps):
        x = mpmath.mpf(x)
        N = len(coeffs) - 1
        c = [mpmath.mpf(float(v)) for v in coeffs]
        if family == "cheb":
            p0, p1 = mpmath.mpf(1), x
        elif family == "leg":
            p0, p1 = mpmath.mpf(1), x
        elif family == "ultra":
            lam = mpmath.mpf(params[0])
            p0, p1 = mpmath.mpf(1), 2 * lam * x
        elif family == "jacobi":
            a, b = mpmath.mpf(params[0]), mpmath.mpf(params[1])
            p0, p1 = mpmath.mpf(1), (a + 1) + (a + b + 2) * (x - 1) / 2
        elif family == "laguerre":
            a = mpmath.mpf(params[0])
            p0, p1 = mpmath.mpf(1), 1 + a - x
        else:
            raise ValueError(family)
        s = c[0] * p0 + (c[1] * p1 if N >= 1 else 0)
        for n in range(1, N):
            if family == "cheb":
                p2 = 2 * x * p1 - p0
            elif family == "leg":
                p2 = ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
            elif family == "ultra":
                p2 = (2 * (n + lam) * x * p1 - (n + 2 * lam - 1) * p0) / (n + 1)
            elif family == "jacobi":
                s2 = 2 * n + a + b
                p2 = ((s2 + 1) * ((s2 + 2) * s2 * x + a * a - b * b) * p1
                      - 2 * (n + a) * (n + b) * (s2 + 2) * p0) / (2 * (n + 1) * (n + a + b + 1) * s2)
            else:
                p2 = ((2 * n + a + 1 - x) * p1 - (n + a) * p0) / (n + 1)
            s += c[n + 1] * p2
            p0, p1 = p1, p2
        return s
