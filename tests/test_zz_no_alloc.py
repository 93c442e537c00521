"""GPU test of thx_execute_noalloc (workspace in the library's static scratch,
no allocation) through the C ABI: its output against thx_execute's for the same
plan and inputs, to the parity bars (1e-13 of ||alpha||_1 in double precision,
5e-6 in FP32-bulk), on two calls in a row, the second with a smaller input, for
every path that uses a workspace; and the error for an execution whose
workspace does not fit.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_1604_07486_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def thx():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1604_07486_amd import binding
    return binding


def _pair(thx, plan, alpha, degree=None):
    import torch
    a = torch.from_numpy(np.ascontiguousarray(alpha)).to("cuda:0")
    ref = torch.full_like(a, float("nan"))
    got = torch.full_like(a, float("nan"))
    plan.execute(a, ref, degree=degree)
    plan.execute_noalloc(a, got, degree=degree)
    torch.cuda.synchronize()
    return ref.cpu().numpy().reshape(-1, a.shape[-1]), got.cpu().numpy().reshape(-1, a.shape[-1])


# (kind, params, plan degree, prec, first call (degree, batch), second call (degree, batch))
CASES = [
    (0, (), 1 << 20, 0, (1 << 20, 1), (5000, 1)),        # three-pass FFT at the headline size, then small
    (0, (), 70000, 2, (70000, 2), (40000, 1)),           # FP64 with the single-precision tail
    (0, (), 40000, 1, (40000, 4), (9000, 2)),            # FP32-bulk
    (1, (), 20000, 0, (20000, 2), (3000, 1)),            # cheb2leg: row 0 direct
    (5, (0.5, -0.25), 3000, 0, (3000, 3), (1000, 2)),    # two stages: intermediate in the scratch
    (3, (2.6, 0.3, 0.2, 1.3), 2000, 0, (2000, 2), (700, 1)),  # longer chain: two intermediates
    (2, (1.5, 0.5), 9000, 0, (9000, 2), (4000, 1)),      # unit step (suffix sums)
    (0, (), 300, 0, (300, 50), (100, 7)),                # dense path (no workspace)
]


@pytest.mark.parametrize("kind,params,N,prec,first,second", CASES)
def test_noalloc_matches_execute(thx, kind, params, N, prec, first, second):
    print(f"[case] noalloc kind={kind} params={params} N={N} prec={prec} calls={first},{second}", flush=True)
    plan = thx.Plan(kind, N, 1e-15 if prec != 1 else 1e-7, prec, params=params)
    bar = 5e-6 if prec == 1 else 1e-13
    for call, (deg, batch) in enumerate((first, second)):
        alpha = inputs.coeffs(deg, 1.0, seed=deg + call, batch=batch)
        ref, got = _pair(thx, plan, alpha, degree=deg)
        al = alpha.reshape(batch, -1)
        for i in range(batch):
            d = float(np.max(np.abs(got[i] - ref[i])) / np.sum(np.abs(al[i])))
            print(f"  call {call} degree {deg} vector {i}: |noalloc - execute|/|a|1 = {d:.3e}", flush=True)
            assert np.all(np.isfinite(got[i])) and d < bar
        if deg <= 3000 and kind in (0, 1, 2):
            name = {0: "leg2cheb", 1: "cheb2leg", 2: "ultra2ultra"}[kind]
            e = float(np.max(np.abs(got[0] - oracle.matvec(name, al[0], params))) / np.sum(np.abs(al[0])))
            scale = 2 * deg + 1 if kind == 2 else 1.0
            assert e < bar * scale


def test_noalloc_rejects_oversized_workspace(thx):
    import torch
    N = 1 << 22
    plan = thx.Plan(thx.LEG2CHEB, N, 1e-15, thx.FP64)
    a = torch.zeros(N + 1, dtype=torch.float64, device="cuda:0")
    b = torch.zeros_like(a)
    with pytest.raises(thx.ThxError) as ei:
        plan.execute_noalloc(a, b)
    assert ei.value.status == 6                      # THX_WORKSPACE_TOO_LARGE
    assert thx.thx_status_string(6) == "THX_WORKSPACE_TOO_LARGE"
    torch.cuda.synchronize()
