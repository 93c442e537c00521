"""GPU parity on seeded random cases: kind, parameters, degree, batch, precision
and the plan's path choices (forced FFT, autotuning, row length, FFT radix,
slot grouping, fused column pass) drawn together, so that combinations the
targeted tests do not list are compared with the oracle too.  Same bars as
test_gpu_parity (tests/bars.py): 1e-13 (FP64, and FP64 with the single-precision
tail) and 5e-6 (FP32-bulk) of ||alpha||_1, scaled by the largest matrix entry at
the tested degree where entries grow with the degree, and of the rounding scale
max_j (|A| |alpha|)_j.  Every kind runs at the same Hankel tolerance, 1e-15
(FP64) or 1e-7 (FP32-bulk).
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1604_07486_amd import inputs

from . import bars
from .test_gpu_parity import _dev, _jac_ref, thx  # noqa: F401  (thx: the module fixture)

pytestmark = pytest.mark.gpu

CASES = 64


def _case(i):
    g = inputs.rng(7000 + i)
    kind = int(g.integers(0, 7))
    N = int(np.exp(g.uniform(np.log(2), np.log(25000))))
    batch = int(g.integers(1, 3))
    prec = int(g.integers(0, 3))   # FP64, FP32-bulk, FP64 with the single-precision tail
    force_fft = bool(g.integers(0, 2))
    tune = bool(g.integers(0, 2))
    env = {}
    if g.uniform() < 0.4:
        env["THX_ROW_LEN"] = str([2048, 4096][int(g.integers(0, 2))] * (2 if prec == 1 else 1))
    r = g.uniform()
    if r < 0.25:
        env["THX_P1_BLOCKS"] = "1"
    elif r < 0.5:
        env["THX_P1_BLOCKS"] = "-1"
    if g.uniform() < 0.3:
        env["THX_LDS_RADIX"] = "16"
    u = lambda lo, hi: round(float(g.uniform(lo, hi)), 3)
    if kind == 2:
        params = (u(0.2, 2.5), u(0.2, 2.5))
    elif kind == 3:
        params = (u(-0.8, 1.2), u(-0.8, 1.2), u(-0.8, 1.2), u(-0.8, 1.2))
    elif kind == 4:
        params = (u(-0.8, 1.5), u(-0.8, 1.5))
    elif kind in (5, 6):
        params = (u(-0.8, 1.2), u(-0.8, 1.2))
    else:
        params = ()
    if kind in (3, 5, 6):
        N = min(N, bars.DENSE_MAX)   # the composite matrix (for the bar scale) is formed densely
    return kind, params, N, batch, prec, force_fft, tune, env


@pytest.mark.parametrize("i", range(CASES))
def test_random_case(thx, i, monkeypatch):
    import torch
    kind, params, N, batch, prec, force_fft, tune, env = _case(i)
    print(f"[case] random {i}: kind={kind} params={params} N={N} batch={batch} prec={prec} "
          f"force_fft={force_fft} tune={tune} env={env}", flush=True)
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    p = 1.5 if kind == 1 else 1.0
    fp64 = prec != 1
    tol = 1e-15 if fp64 else 1e-7
    alpha = inputs.coeffs(N, p, seed=100 + i, batch=batch)
    plan = thx.Plan(kind, N, tol, prec, params=params, flags=thx.FLAG_FORCE_FFT if force_fft else 0)
    if tune:
        plan.autotune(batch)
    a = _dev(alpha)
    b = torch.full_like(a, float("nan"))
    plan.execute(a, b)
    torch.cuda.synchronize()
    got = b.cpu().numpy()
    bar = 1e-13 if fp64 else 5e-6
    # leg2cheb and cheb2leg: bar relative to ||alpha||_1 as it stands; the others
    # scaled by their largest entry at this degree
    scale = 1.0 if kind in (0, 1) else bars.entry_max(kind, N, params)
    for j in range(batch):
        if kind in (3, 5, 6):
            ref = _jac_ref(kind, alpha[j], params)
        else:
            ref = oracle.matvec({0: "leg2cheb", 1: "cheb2leg", 2: "ultra2ultra", 4: "lag2lag"}[kind], alpha[j],
                                params)
        print(f"  vector {j}: path={plan.path} K={plan.rank} tail={plan.tail_slots} L={plan.fft_length}", flush=True)
        bars.check(got[j], ref, alpha[j], bar, kind, params, entry_scale=scale, label=f"case {i} vector {j} ")
