"""Error bars of the GPU parity tests, computed from the oracle only.

Error measure (Sec. 4 plots the absolute error; the targets are relative):
    err = max_j |beta_gpu_j - beta_oracle_j| / ||alpha||_1
with bars 1e-13 (double precision) and 5e-6 (single-precision bulk).  For
matrices whose entries grow with the degree, one rounding unit is amplified by
the largest entry, so the bar is multiplied by max(1, max_jk |A_jk|), taken at
the tested degree (never extrapolated).  Every check also asserts the error
against the rounding scale of the vector itself,
    max_j |beta_gpu_j - beta_oracle_j| <= bar * max_j (|A| |alpha|)_j,
which is never looser than the first (max_j (|A||alpha|)_j <= max|A| ||alpha||_1)
and stays meaningful when beta is much smaller than ||alpha||_1.
"""
from __future__ import annotations

import numpy as np

import oracle

BAR64, BAR32 = 1e-13, 5e-6
DENSE_MAX = 3000   # largest degree whose composite Jacobi matrix is formed densely


def jacobi_ends(kind, params):
    """(a, b, g, d) of a Jacobi-type conversion (3 jac2jac, 5 jac2cheb, 6 cheb2jac)."""
    if kind == 3:
        return tuple(params)
    if kind == 5:
        return params[0], params[1], -0.5, -0.5
    return -0.5, -0.5, params[0], params[1]


def jacobi_matrix(kind, N, params):
    """The composite conversion matrix of a Jacobi-type kind (Sec. 5.3), densely."""
    a, b, g, d = jacobi_ends(kind, params)
    A = np.eye(N + 1)
    sgn = np.where(np.arange(N + 1) % 2 == 0, 1.0, -1.0)
    if b != d:
        A = (sgn[:, None] * oracle.dense("jac2jac_b", N, (b, a, d)) * sgn[None, :]) @ A
    if a != g:
        A = oracle.dense("jac2jac_b", N, (a, d, g)) @ A
    cn = oracle.cheb_norm(N)
    if kind == 5:
        A = cn[:, None] * A
    elif kind == 6:
        A = A / cn[None, :]
    return A


def single_stage(kind, params):
    """True when the oracle computes the kind with one closed-form matrix."""
    if kind in (0, 1, 2, 4):
        return True
    a, b, g, d = jacobi_ends(kind, params)
    return kind == 3 and b == d


ORACLE_NAME = {0: "leg2cheb", 1: "cheb2leg", 2: "ultra2ultra", 4: "lag2lag"}


def _stage(kind, params):
    if kind in ORACLE_NAME:
        return ORACLE_NAME[kind], tuple(params)
    a, b, g, d = jacobi_ends(kind, params)
    return "jac2jac_b", (a, b, g)


def entry_max(kind, N, params=()):
    """max_jk |A_jk| at degree N (O(N^2) in the oracle; dense product for Jacobi composites)."""
    if kind == 0:
        return 1.0                      # max |M_jk| = M_00 = 1 (pinned against exact bases)
    if single_stage(kind, params):
        name, p = _stage(kind, params)
        return oracle.absmax(name, N, p)
    if N > DENSE_MAX:
        raise ValueError("composite Jacobi entry maximum only up to degree %d" % DENSE_MAX)
    return float(np.max(np.abs(jacobi_matrix(kind, N, params))))


def row_scale(kind, alpha, params=(), rows=None):
    """max over the rows of (|A| |alpha|)_j (all rows, or the sampled ones)."""
    N = len(alpha) - 1
    if single_stage(kind, params):
        name, p = _stage(kind, params)
        return float(np.max(oracle.matvec(name, alpha, p, rows=rows, absolute=True)))
    if N > DENSE_MAX:
        raise ValueError("composite Jacobi row scale only up to degree %d" % DENSE_MAX)
    s = np.abs(jacobi_matrix(kind, N, params)) @ np.abs(alpha)
    return float(np.max(s if rows is None else s[np.asarray(rows)]))


def check(got, ref, alpha, bar, kind, params=(), rows=None, entry_scale=None, label=""):
    """Assert both bars (see the module docstring) and print their margins.

    entry_scale: max|A_jk| when the caller knows it (closed form); computed here otherwise.
    Returns err / ||alpha||_1.
    """
    N = len(alpha) - 1
    dif = float(np.max(np.abs(np.asarray(got) - np.asarray(ref))))
    l1 = float(np.sum(np.abs(alpha)))
    err = dif / l1
    scale = max(1.0, entry_scale if entry_scale is not None else entry_max(kind, N, params))
    rs = row_scale(kind, alpha, params, rows)
    rel = dif / max(rs, 1e-300)
    print(f"  {label}err/|a|1={err:.3e} (bar {bar * scale:.2e}, margin {bar * scale / max(err, 1e-300):.1e}) "
          f"err/max(|A||a|)={rel:.3e} (bar {bar:.0e}, margin {bar / max(rel, 1e-300):.1e}) "
          f"err/max|beta|={dif / max(float(np.max(np.abs(ref))), 1e-300):.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert err < bar * scale, (label, err, bar * scale)
    assert rel < bar, (label, rel, bar)
    return err
