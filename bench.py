#!/usr/bin/env python3
"""Benchmark of the Toeplitz-dot-Hankel conversion on one MI355X.

Headline workload: Legendre -> Chebyshev, one vector of degree N = 2^20,
FP64 end to end, alpha_k = z_k (k+1)^-1.5 with z ~ N(0,1) (seeded), Hankel
parts factorised to 1e-15.  A step is one execution of Fig. 1 steps 3-5
(pack, K diagonally scaled Toeplitz products, D1) on a plan built once
(steps 1-2 and the symbol FFT; the plan is reused as Sec. 2.1 suggests), with
alpha already resident in HBM.  Plan construction is timed separately.

Printed: one JSON line with the contract fields, the roofline of the dominant
kernel (HIP-event timings of every launch in the timed region) and the CPU
oracle timed on a bounded sample of output rows.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "leg2cheb coeffs/s at N=2^20 & batched; HBM GB/s; FP32 vs FP64 at stated error"
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--log2n", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the headline timed loop (for profiler runs)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="in --headline-only mode, run the plan's default launch shapes (the same kernels in "
                         "every run: counter passes that must be combined)")
    ap.add_argument("--shapes", nargs=2, type=int, metavar=("ROW", "P1_BLOCKS"), default=None,
                    help="in --headline-only mode, fix the three-pass row length and the forward column pass's "
                         "workgroups per launch (0: one slot per workgroup) instead of autotuning, so that "
                         "counter passes that must be combined run the kernels the autotuner picks")
    ap.add_argument("--prec", choices=["fp64", "fp32", "tail32"], default="fp64",
                    help="precision of the headline loop in --headline-only mode")
    ap.add_argument("--only", choices=["batched", "config5", "sweep", "config1", "dense"], default=None,
                    help="run one secondary section only (profiler runs) and print its JSON")
    ap.add_argument("--kind", choices=["ultra", "jac2cheb"], default=None,
                    help="with --only config5: one conversion only")
    ap.add_argument("--write-traffic", nargs="+", metavar="ARG", default=None,
                    help="FETCH_DB WRITE_DB RUN_LOG [OUT]: summarise two rocprofv3 --pmc runs of "
                         "--headline-only --copy-calibration (FETCH_SIZE, WRITE_SIZE) into OUT (default: the "
                         "FP64 row-pass file under profiles/) and exit (no GPU use)")
    ap.add_argument("--write-trace", nargs="+", metavar="ARG", default=None,
                    help="DB OUT_MD TITLE COMMAND [REPLAYS]: summarise the timed region of a rocprofv3 "
                         "--kernel-trace database (the kernels between the trace markers 1 and 2) into a "
                         "markdown table, with the first execution's timeline when REPLAYS is given, and "
                         "exit (no GPU use)")
    ap.add_argument("--write-counters", nargs=4, metavar=("DB", "OUT_MD", "TITLE", "COMMAND"), default=None,
                    help="average every counter of a rocprofv3 --pmc database per kernel over the dispatches "
                         "between trace markers 1 and 2 into a markdown table and exit (no GPU use)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also time a plain device copy of 512 MiB (bandwidth ceiling and the "
                         "reference for HBM byte counters)")
    return ap.parse_args()


COPY_BYTES = 512 << 20
MFMA_FP64_TFLOPS = 78.6   # MI355X dense matrix-core peaks
MFMA_BF16_TFLOPS = 2500.0
VALU_FP64_TFLOPS = 78.6   # 256 CUs x 128 FP64 flops per clock (FMA = 2) x 2.4 GHz

# Measured HBM traffic of the dominant kernel (row pass of the headline plan),
# valid only for the device sources it was taken with, the same template
# instantiation (row length) and the same algorithmic bytes per launch.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "passes_leg2cheb_N2p20_fp64_hbm_traffic.txt")
TRAFFIC_SOURCES = ["paper_1604_07486_amd/csrc/kernels.hip", "paper_1604_07486_amd/csrc/fft_reg.hpp",
                   "paper_1604_07486_amd/csrc/thx_device.hpp", "paper_1604_07486_amd/csrc/launch.hpp"]


def row_kernel_name(plan):
    """Template instantiation of the row pass the plan launches (its row length)."""
    return f"k_mp_p2<double, {plan.fft_geometry()[0]}>" if plan.path == 2 else None


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oracle_extras(oracle, inputs, alpha, N, threads):
    """Single-thread rate on a bounded sample of rows at the headline size, and full O(N^2)
    conversions at small N with all threads (a few seconds of CPU in total)."""
    g = inputs.rng(98)
    r = g.integers(0, N + 1, size=256)
    t0 = time.perf_counter()
    oracle.matvec("leg2cheb", alpha, rows=r, nthreads=1)
    t1 = time.perf_counter() - t0
    full = []
    for n in (2048, 4096, 65536):
        a = inputs.coeffs(n, 1.0, seed=n)
        t0 = time.perf_counter()
        oracle.matvec("leg2cheb", a, nthreads=threads)
        dt = time.perf_counter() - t0
        full.append({"N": n, "seconds": round(dt, 4), "coeffs_per_s": round((n + 1) / dt, 1)})
    return {"single_thread": {"value": round(256 / t1, 2), "unit": "coeffs/s", "cores": 1,
                              "sample": "256 random output rows of leg2cheb at N=2^20"},
            "full_conversions": full, "cpu_model": cpu_model(), "nproc": os.cpu_count()}


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def pmc_dispatches(db, counter):
    """(kernel name, value in KiB) per dispatch of one rocprofv3 --pmc database, in dispatch order."""
    import re
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, value from counters_collection where counter_name = ? "
                       "order by dispatch_id", (counter,)).fetchall()
    con.close()
    return [(re.sub(r"\(.*", "", k).replace("void ", "").replace("thx::", ""), v) for _, k, v in rows]


def kernel_phase(name):
    """Phase of a library kernel by its name (None for kernels outside the execution)."""
    for prefix, phase in (("k_mp_p1", "col_fwd"), ("k_mp_p2f", "row"), ("k_mp_p2<", "row"), ("k_mp_p3", "col_inv"),
                          ("k_toep_lds", "toep_lds"), ("k_pack", "pack"), ("k_unpack", "unpack")):
        if name.startswith(prefix):
            return phase
    return None


def timed_window(d):
    """The dispatches between trace marker 1 and the next marker 2 (the timed loop)."""
    marks = [i for i, (k, _) in enumerate(d) if k.startswith("k_trace_marker")]
    return d[marks[0] + 1:marks[1]]


def write_traffic(fetch_db, write_db, run_log, out=None):
    """FETCH_SIZE / WRITE_SIZE per dispatch of every kernel of the timed loop, scaled by what the
    same counters read for the 512 MiB device copy of the same run, against each launch's
    algorithmic bytes.  `run_log` holds the JSON line of the profiled `--headline-only` run (its
    precision, row-pass instantiation and the algorithmic bytes of each phase).  The key lines
    below the table describe the row pass (read back by the bench for `roofline.traffic`)."""
    info = None
    for line in open(run_log):
        if line.startswith("{") and '"headline_only"' in line:
            info = json.loads(line)
    prec, algo_by_phase, lg = info["prec"], info["phase_bytes"], info.get("log2n", 20)
    out = out or TRAFFIC_FILE
    per = {}
    for key, db, counter in (("fetch", fetch_db, "FETCH_SIZE"), ("write", write_db, "WRITE_SIZE")):
        d = pmc_dispatches(db, counter)
        copy = max(v for k, v in d if "copyBuffer" in k)   # the 512 MiB calibration copy
        factor = (COPY_BYTES / 1024) / copy
        for k, v in timed_window(d):
            per.setdefault(k, {}).setdefault(key, []).append(v)
        per.setdefault("_factor", {})[key] = factor
    fac = per.pop("_factor")
    odd = sorted(k for k, vals in per.items() if len(vals) != 2)
    if odd:
        raise SystemExit(f"the two counter runs timed different kernels {odd}: profile a plan with fixed "
                         "launch shapes (--no-autotune)")
    rows_md, row = [], None
    for k, vals in sorted(per.items(), key=lambda kv: -sum(kv[1].get("fetch", [0]))):
        f = sum(vals["fetch"]) / len(vals["fetch"]) * 1024 * fac["fetch"]
        w = sum(vals["write"]) / len(vals["write"]) * 1024 * fac["write"]
        ph = kernel_phase(k)
        algo = algo_by_phase.get(ph) if ph else None
        ratio = f"{(f + w) / algo:.3f}" if algo else "-"
        rows_md.append(f"# | `{k}` | {ph or '-'} | {len(vals['fetch'])} | {f / 1e6:.1f} | {w / 1e6:.1f} | "
                       f"{(algo or 0) / 1e6:.1f} | {ratio} |")
        if ph == "row" and (row is None or f + w > row[1] + row[2]):
            row = (k, f, w, algo, vals)
    tuned, shapes = info.get("autotuned", True), info.get("shapes")
    fixed = f" --shapes {shapes[0]} {shapes[1]}" if shapes else " --no-autotune"
    cmd = ("rocprofv3 --pmc {c} -d $OUT/pmc/{p}_{lg}_{c} -o pmc -- python3 $R/bench.py --headline-only --steps 3 "
           "--warmup 1 --copy-calibration --prec {p} --log2n {lg}" + ("" if tuned else fixed))
    if tuned:
        how = "(autotuned for one vector)"
    elif shapes:
        p1 = f"{shapes[1]} workgroups per launch" if shapes[1] > 0 else "one slot per workgroup"
        how = (f"(launch shapes fixed at those the autotuner picks, geometry {info.get('fft_geometry')}, forward "
               f"column pass {p1}: the same kernels in both counter runs)")
    else:
        how = f"(default launch shapes, geometry {info.get('fft_geometry')}: the same kernels in both counter runs)"
    lines = [
        f"# HBM traffic per launch of the timed loop, leg2cheb N=2^{lg} {prec} plan " + how,
        "# Counters in KiB per dispatch from rocprofv3 --pmc, one counter per run, averaged over the",
        "# dispatches between trace markers 1 and 2; factors = bytes of the 512 MiB device copy in the",
        "# same run / counter.  Commands (repo root $R, output directory $OUT, from /tmp, TMPDIR=/tmp):",
        "#   " + cmd.format(c="FETCH_SIZE", p=prec, lg=lg) + f" > $OUT/pmc/{prec}_{lg}_FETCH_SIZE.log",
        "#   " + cmd.format(c="WRITE_SIZE", p=prec, lg=lg),
        f"#   python3 bench.py --write-traffic $OUT/pmc/{prec}_{lg}_FETCH_SIZE/pmc_results.db "
        f"$OUT/pmc/{prec}_{lg}_WRITE_SIZE/pmc_results.db $OUT/pmc/{prec}_{lg}_FETCH_SIZE.log "
        f"{os.path.relpath(out, ROOT)}",
        f"# fetch factor {fac['fetch']:.4f}, write factor {fac['write']:.4f}",
        "# | kernel | phase | launches | read (MB) | written (MB) | algorithmic (MB) | measured / algorithmic |",
        "# |---|---|---:|---:|---:|---:|---:|",
        *rows_md,
        f"kernel = {row[0]}",
        "phase = row",
        f"fetch_kib_per_dispatch = {sum(row[4]['fetch']) / len(row[4]['fetch']):.1f}",
        f"write_kib_per_dispatch = {sum(row[4]['write']) / len(row[4]['write']):.1f}",
        f"dispatches = {len(row[4]['fetch'])}",
        f"fetch_factor = {fac['fetch']:.4f}",
        f"write_factor = {fac['write']:.4f}",
        f"traffic_bytes_per_launch = {row[1] + row[2]:.0f}",
        f"algorithmic_bytes_per_launch = {row[3]}",
        f"source_sha256 = {source_digest()}",
    ]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def write_counters(db, out_md, title, command):
    """Per kernel of the timed loop (between trace markers 1 and 2): the average of every counter the
    run collected, per dispatch (rocprofv3 reports per-SE and per-SIMD counters summed over the chip)."""
    import re
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection "
                       "order by dispatch_id").fetchall()
    con.close()
    disp = {}
    for d, k, c, v in rows:
        disp.setdefault(d, [re.sub(r"\(.*", "", k).replace("void ", "").replace("thx::", ""), {}])[1][c] = v
    ids = sorted(disp)
    marks = [i for i in ids if disp[i][0].startswith("k_trace_marker")]
    agg = {}
    for i in ids:
        if not (marks[0] < i < marks[1]):
            continue
        name, cs = disp[i]
        a = agg.setdefault(name, {"_n": 0})
        a["_n"] += 1
        for c, v in cs.items():
            a[c] = a.get(c, 0.0) + v
    counters = sorted({c for a in agg.values() for c in a if c != "_n"})
    lines = [f"# Counters: {title}", "", "Command (repo root $R, output directory $OUT, from /tmp with TMPDIR=/tmp), "
             "then the summary:", "", "```", command,
             f"python3 $R/bench.py --write-counters <pmc_results.db> <this file> \"{title}\" \"<the command>\"",
             "```", "", "Average per dispatch of the timed loop (between trace markers 1 and 2).", "",
             "| kernel | dispatches | " + " | ".join(counters) + " |",
             "|---|---:|" + "---:|" * len(counters)]
    for name, a in agg.items():
        n = a["_n"]
        lines.append(f"| `{name}` | {n} | " + " | ".join(f"{a.get(c, 0.0) / n:.0f}" for c in counters) + " |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def measured_traffic(phase, kernel, algo_bytes):
    """Bytes per launch from the committed counter summary, or None if it is absent, for another
    phase or kernel instantiation (the plan's row length picks the template), for a launch of other
    algorithmic bytes (another rank or slot chunking), or taken with other device sources."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        if kv.get("phase") != phase or kv.get("kernel") != kernel or kv.get("source_sha256") != source_digest():
            return None
        if int(kv["algorithmic_bytes_per_launch"]) != int(algo_bytes):
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_bandwidth(torch, reps=20):
    """GB/s of a plain device-to-device copy of COPY_BYTES (read + write counted)."""
    src = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    del src, dst
    return 2 * COPY_BYTES / dt / 1e9


def phase_bytes(phase, es, S, nc, L, G, batch=1):
    """Algorithmic HBM bytes of one launch of `phase` (single rank chunk).

    es: bytes per complex element; S: FFT slots in the launch; nc: complex lanes
    of the input; L: FFT length; G: partial-sum groups.  Each term is data the
    launch must read or write at least once: the normalised Cholesky columns
    (S nc), the packed input (nc per vector), the FFT intermediates (S L per
    vector, written by the forward column pass, read and written by the row
    pass, read by the inverse column pass), the symbol spectrum (L) and the
    partial sums (G nc per vector)."""
    if phase == "col_fwd":
        return es * (S * nc + batch * nc + S * batch * L)
    if phase == "row":
        return es * (2 * S * batch * L + L)
    if phase == "col_inv":
        return es * (S * batch * L + S * nc + G * batch * nc)
    if phase == "toep_lds":
        return es * (S * nc + batch * nc + L + G * batch * nc)
    return None


def time_plan(thx, torch, plan, a, b, steps, warmup, phase=None):
    """Milliseconds per execution over `steps` timed executions.  With `phase`,
    that phase's launches are bracketed by HIP events inside the timed loop (two
    events per launch: the other phases run without markers, which would add a
    few microseconds each).  Trace markers 1 and 2 (empty kernels, outside the
    timed region) delimit the loop in a kernel trace."""
    for _ in range(warmup):
        plan.execute(a, b)
    torch.cuda.synchronize()
    plan.timings(reset=True)
    if phase is not None:
        plan.enable_timing(True, phases=(phase,))
    thx.thx_trace_marker(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.execute(a, b)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    thx.thx_trace_marker(2)
    plan.enable_timing(False)
    return (t1 - t0) * 1e3 / steps, plan.timings(reset=True)


def busy_union(iv):
    """Length of the union of [start, end) intervals (time with at least one kernel running)."""
    tot, cur_s, cur_e = 0, None, None
    for st, en in sorted(iv):
        if cur_e is None or st > cur_e:
            if cur_e is not None:
                tot += cur_e - cur_s
            cur_s, cur_e = st, en
        else:
            cur_e = max(cur_e, en)
    return tot + (cur_e - cur_s if cur_e is not None else 0)


def write_trace(db, out_md, title, command, replays=None):
    """Markdown table of the kernels between the first trace marker 1 and the next marker 2 of a
    rocprofv3 --kernel-trace database (the timed loop only: no plan, tuning or warm-up dispatches),
    with the loop's span against the sum of its kernel durations and against the time during
    which at least one kernel runs (concurrent graph branches overlap).  With `replays` (the
    number of executions in the loop, equal kernel sequences), the first execution's dispatches
    are listed with their start and end relative to its first dispatch."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select name, start, end, grid_x, grid_y * grid_z, workgroup_x * workgroup_y * workgroup_z "
                       "from kernels order by start").fetchall()
    con.close()
    marks = [(i, r[3]) for i, r in enumerate(rows) if "k_trace_marker" in r[0]]
    i0 = next(i for i, gx in marks if gx == 64)
    i1 = next(i for i, gx in marks if gx == 128 and i > i0)
    win = [r for r in rows[i0 + 1:i1] if "k_trace_marker" not in r[0]]
    stats = {}
    for n, st, en, *_ in win:
        name = n.split("(")[0].replace("void ", "")
        stats.setdefault(name, []).append((en - st) / 1e3)
    total = sum(sum(v) for v in stats.values())
    span = (max(r[2] for r in win) - min(r[1] for r in win)) / 1e3
    busy = busy_union([(r[1], r[2]) for r in win]) / 1e3
    rep_arg = f" {int(replays)}" if replays else ""
    lines = [f"# Kernel trace: {title}", "",
             "Command (repo root $R, output directory $OUT, from /tmp with TMPDIR=/tmp), then the summary:", "",
             "```", command,
             f"python3 $R/bench.py --write-trace <kt_results.db> <this file> \"{title}\" \"<the command>\"{rep_arg}",
             "```", "",
             f"Only the dispatches of the timed loop (between trace markers 1 and 2): {len(win)} launches, "
             f"{total:.1f} us of kernel time in a span of {span:.1f} us; at least one kernel runs during "
             f"{busy:.1f} us of it ({100 * (span - busy) / span:.1f}% of the span with no kernel running).", "",
             "| kernel | calls | total (us) | average (us) | min (us) | max (us) | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for name, v in sorted(stats.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{name}` | {len(v)} | {sum(v):.1f} | {sum(v) / len(v):.1f} | {min(v):.1f} | "
                     f"{max(v):.1f} | {100 * sum(v) / total:.1f} |")
    if replays and len(win) % int(replays) == 0:
        per = len(win) // int(replays)
        first = win[:per]
        t0 = first[0][1]
        fspan = (max(r[2] for r in first) - t0) / 1e3
        fbusy = busy_union([(r[1], r[2]) for r in first]) / 1e3
        lines += ["", f"First of the {int(replays)} executions: {per} dispatches in {fspan:.1f} us, at least one "
                  f"kernel running during {fbusy:.1f} us ({100 * (fspan - fbusy) / fspan:.1f}% idle).", "",
                  "| # | kernel | workgroups | start (us) | end (us) | duration (us) |",
                  "|---:|---|---:|---:|---:|---:|"]
        for i, (n, st, en, gx, gyz, wg) in enumerate(first):
            name = n.split("(")[0].replace("void ", "")
            lines.append(f"| {i} | `{name}` | {gx * gyz // max(1, wg)} | {(st - t0) / 1e3:.1f} | "
                         f"{(en - t0) / 1e3:.1f} | {(en - st) / 1e3:.1f} |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def phase_breakdown(torch, plan, a, b, steps):
    """{phase: (total_ms, launches)} from executions with every phase timed; run
    outside the timed loop, since the markers slow the step down."""
    torch.cuda.synchronize()
    plan.timings(reset=True)
    plan.enable_timing(True)
    for _ in range(steps):
        plan.execute(a, b)
    torch.cuda.synchronize()
    plan.enable_timing(False)
    return plan.timings(reset=True)


def phase_avg(tim):
    return {k: round(v[0] / v[1], 5) for k, v in tim.items()}


def sampled_error(oracle, kind, alpha, got, rows):
    ref = oracle.matvec(kind, alpha, rows=rows)
    return float(np.max(np.abs(got[rows] - ref)) / np.sum(np.abs(alpha)))


def lds_flops(S, L, nc, batch=1):
    """Algorithmic flops of one single-workgroup launch: per slot and vector a forward and an
    inverse complex FFT of length L (5 L log2 L each), the product with the symbol (6 L), the
    scaling of the input by the Cholesky column (2 nc) and the scaled accumulation (4 nc)."""
    import math
    return batch * S * (10 * L * math.log2(L) + 6 * L + 6 * nc)


def run_config1(thx, torch, inputs, oracle, dev, steps):
    """Legendre -> Chebyshev, one vector of degree 2048, FP64, Hankel tol 1e-15: one launch of the
    single-workgroup FFT path per conversion; its rate against the FP64 vector peak.  Timed as plan
    executions (one call each) and as replays of a one-member batch graph."""
    N = 2048
    alpha = inputs.coeffs(N, 1.0, seed=2048)
    a = torch.from_numpy(alpha).to(dev)
    b = torch.empty_like(a)
    plan = thx.Plan(thx.LEG2CHEB, N, 1e-15, thx.FP64, flags=thx.FLAG_FORCE_FFT)
    plan.autotune(1)
    reps = max(200, steps * 10)
    ms, _ = time_plan(thx, torch, plan, a, b, reps, 20)
    ref = oracle.matvec("leg2cheb", alpha)
    err = float(np.max(np.abs(b.cpu().numpy() - ref)) / np.sum(np.abs(alpha)))
    _, tim = time_plan(thx, torch, plan, a, b, reps, 5, phase="toep_lds")
    # the same conversion as a one-member batch replayed as a hipGraph (no launch gaps between
    # its kernels)
    bt = thx.Batch(thx.LEG2CHEB, np.array([N], dtype=np.int64), 1e-15, thx.FP64,
                   flags=thx.FLAG_FORCE_FFT | thx.FLAG_AUTOTUNE)
    bb = torch.empty_like(a)
    for _ in range(20):
        bt.execute(a, bb, graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        bt.execute(a, bb, graph=True)
    torch.cuda.synchronize()
    gms = (time.perf_counter() - t0) * 1e3 / reps
    gerr = float(np.max(np.abs(bb.cpu().numpy() - ref)) / np.sum(np.abs(alpha)))
    gbk = bt.buckets()
    del bt
    tot, cnt = tim["toep_lds"]
    kms = tot / cnt
    fl = lds_flops(plan.rank, plan.fft_length, N // 2 + 1)
    tf = fl / (kms * 1e-3) / 1e12
    return {"workload": "leg2cheb N=2048 (2049 coefficients), batch 1, FP64, alpha_k ~ N(0,1)(k+1)^-1 seed 2048, "
                        "Hankel tol 1e-15, FFT path (length 2048 complex per parity half), plan autotuned",
            "ms_per_conversion": round(ms, 5), "coeffs_per_s": round((N + 1) / (ms * 1e-3), 1),
            "K": plan.rank, "L": plan.fft_length, "lds_radix": plan.lds_radix, "max_err_over_l1": err,
            "graph_replay": {"ms_per_conversion": round(gms, 5), "coeffs_per_s": round((N + 1) / (gms * 1e-3), 1),
                             "max_err_over_l1": gerr, "buckets": gbk},
            "roofline": {"kernel": "toep_lds", "bound": "alu", "achieved": round(tf, 3),
                         "peak": VALU_FP64_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / VALU_FP64_TFLOPS, 5),
                         "flops_per_launch": int(fl), "avg_launch_ms": round(kms, 5), "launches": cnt}}


def run_sweep(thx, torch, inputs, oracle, dev, steps):
    """Precision sweep of Legendre -> Chebyshev: FP64 (Hankel tol 1e-15) against FP32-bulk (1e-7)
    at N = 2^12, 2^16, 2^20, 2^22 for coefficients decaying like (k+1)^-2 and undecayed; error
    against the oracle on every row up to 2^16, on 256 sampled rows (+ the special ones) above."""
    out = []
    for lg in (12, 16, 20, 22):
        N = 1 << lg
        for p in (2.0, 0.0):
            alpha = inputs.coeffs(N, p, seed=300 + lg)
            a = torch.from_numpy(alpha).to(dev)
            b = torch.empty_like(a)
            rows = None if lg <= 16 else inputs.sample_rows(N, 256, seed=lg)
            ref = oracle.matvec("leg2cheb", alpha, rows=rows)
            for prec, tol, name in ((thx.FP64, 1e-15, "fp64"), (thx.FP32_BULK, 1e-7, "fp32_bulk")):
                plan = thx.Plan(thx.LEG2CHEB, N, tol, prec)
                plan.autotune(1)
                n_steps = max(5, steps // (1 if lg <= 20 else 4))
                ms, _ = time_plan(thx, torch, plan, a, b, n_steps, 3)
                got = b.cpu().numpy()
                err = float(np.max(np.abs((got if rows is None else got[rows]) - ref)) / np.sum(np.abs(alpha)))
                out.append({"N": N, "decay": p, "prec": name, "K": plan.rank, "ms": round(ms, 4),
                            "coeffs_per_s": round((N + 1) / (ms * 1e-3), 1), "max_err_over_l1": err,
                            "rows_checked": N + 1 if rows is None else int(len(rows))})
                del plan
    return out


def run_batched(thx, torch, inputs, oracle, dev, steps, precs=("fp64", "fp32_bulk", "fp64_tail32")):
    """Mixed-degree batch: 4096 polynomials, degrees log-uniform in [16, 65536]."""
    degs = inputs.batch_degrees(4096, 16, 65536, seed=4)
    batch_res = {}
    for pname, prec, tolh in (("fp64", thx.FP64, 1e-15), ("fp32_bulk", thx.FP32_BULK, 1e-7),
                              ("fp64_tail32", thx.FP64_TAIL32, 1e-15)):
        if pname not in precs:
            continue
        flat = np.concatenate([inputs.coeffs(int(n), 1.0, seed=1000 + i) for i, n in enumerate(degs)])
        ab = torch.from_numpy(flat).to(dev)
        bb = torch.empty_like(ab)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bt = thx.Batch(thx.LEG2CHEB, degs, tolh, prec, flags=thx.FLAG_AUTOTUNE)
        torch.cuda.synchronize()
        bplan_ms = (time.perf_counter() - t0) * 1e3
        for _ in range(2):
            bt.execute(ab, bb, graph=True)
        torch.cuda.synchronize()
        reps = max(3, steps // 5)
        thx.thx_trace_marker(1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            bt.execute(ab, bb, graph=True)
        torch.cuda.synchronize()
        bms = (time.perf_counter() - t0) * 1e3 / reps
        thx.thx_trace_marker(2)
        got = bb.cpu().numpy()
        g = inputs.rng(5)
        worst = 0.0
        for i in g.choice(len(degs), size=24, replace=False):
            o, n = int(bt.offsets[i]), int(degs[i])
            al = flat[o:o + n + 1]
            r = inputs.sample_rows(n, 64, seed=int(i))
            worst = max(worst, sampled_error(oracle, "leg2cheb", al, got[o:o + n + 1], r))
        batch_res[pname] = {"coeffs_per_s": round(bt.coefficients / (bms * 1e-3), 1), "ms_per_batch": round(bms, 4),
                            "plan_ms": round(bplan_ms, 1), "buckets": bt.buckets(),
                            "max_err_over_l1_sampled": worst, "hankel_tol": tolh}
        del bt, ab, bb
    batch_res["workload"] = ("4096 polynomials, degrees floor(exp(U[ln 16, ln 65536])) seed 4 "
                             f"(sum of degree+1 = {int(np.sum(degs + 1))}), alpha_k ~ N(0,1)(k+1)^-1, "
                             "hipGraph replay, plans reused, buckets autotuned for their member counts "
                             "(plan_ms includes the tuning)")
    return batch_res


def dense_alone(thx, torch, dev, prec, tolh, steps, kind=None, params=(0.5, -0.25)):
    """65536 vectors of degree 255 through one dense plan (matrix cores): the config-5 Jacobi
    (1/2, -1/4) -> Chebyshev members, whose two-stage conversion is materialised as one matrix.
    Time per product (trace markers 1 and 2 around the timed loop), useful flops (the upper
    triangle: (n+1)(n+2)/2 multiply-adds per vector) against the matrix-core peak the form runs
    on, and alpha + beta bytes against HBM."""
    n, m = 255, 65536
    kind = thx.JAC2CHEB if kind is None else kind
    plan = thx.Plan(kind, n, tolh, prec, params=params)
    if plan.path != 3:
        return None
    a = torch.from_numpy(np.random.default_rng(7).standard_normal((m, n + 1))).to(dev)
    b = torch.empty_like(a)
    for _ in range(3):
        plan.execute(a, b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(10, steps)
    thx.thx_trace_marker(1)
    e0.record()
    for _ in range(reps):
        plan.execute(a, b)
    e1.record()
    thx.thx_trace_marker(2)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    flops = m * (n + 1) * (n + 2)
    # FP64 matrix cores; the split-bfloat16 form issues eight bfloat16 products per useful one
    peak = MFMA_FP64_TFLOPS if prec == thx.FP64 else MFMA_BF16_TFLOPS / 8
    tf = flops / (ms * 1e-3) / 1e12
    return {"ms": round(ms, 4), "useful_tflops": round(tf, 2), "peak_tflops": peak,
            "frac_of_peak": round(tf / peak, 4), "hbm_gbs": round(2 * m * (n + 1) * 8 / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(2 * m * (n + 1) * 8 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}


def run_config5(thx, torch, inputs, oracle, dev, steps, kinds=("ultra", "jac2cheb"),
                precs=("fp64", "fp32_bulk")):
    """65536 x degree 255 + 64 x degree 2^18 in one batch, ultraspherical and Jacobi."""
    degs5 = np.array([255] * 65536 + [1 << 18] * 64, dtype=np.int64)
    offs5 = np.concatenate([[0], np.cumsum(degs5 + 1)])
    g5 = inputs.rng(55)
    z5 = g5.standard_normal(int(offs5[-1]))
    kidx = np.arange(int(offs5[-1])) - np.repeat(offs5[:-1], degs5 + 1)
    flat5 = z5 / (kidx + 1.0)                      # alpha_k ~ N(0,1) (k+1)^-1 per member
    a5 = torch.from_numpy(flat5).to(dev)
    b5 = torch.empty_like(a5)
    conf5 = {}
    for short, kname, kind, params in (("ultra", "ultra_1.5_to_0.5", thx.ULTRA2ULTRA, (1.5, 0.5)),
                                       ("jac2cheb", "jac2cheb_0.5_-0.25", thx.JAC2CHEB, (0.5, -0.25))):
        if short not in kinds:
            continue
        for pname, prec, tolh in (("fp64", thx.FP64, 1e-15), ("fp32_bulk", thx.FP32_BULK, 1e-7)):
            if pname not in precs:
                continue
            bt = thx.Batch(kind, degs5, tolh, prec, params=params, flags=thx.FLAG_AUTOTUNE)
            for _ in range(2):
                bt.execute(a5, b5, graph=True)
            torch.cuda.synchronize()
            reps = max(3, steps // 5)
            thx.thx_trace_marker(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                bt.execute(a5, b5, graph=True)
            torch.cuda.synchronize()
            ms5 = (time.perf_counter() - t0) * 1e3 / reps
            thx.thx_trace_marker(2)
            got = b5.cpu().numpy()
            worst = 0.0
            for i in list(range(0, 65536, 8191)) + [65536, 65599]:
                o, n = int(offs5[i]), int(degs5[i])
                al, gi = flat5[o:o + n + 1], got[o:o + n + 1]
                if kind == thx.ULTRA2ULTRA:
                    r = None if n <= 4096 else inputs.sample_rows(n, 32, seed=i)
                    ref = oracle.matvec("ultra2ultra", al, params, rows=r)
                    e = np.max(np.abs((gi if r is None else gi[r]) - ref)) / np.sum(np.abs(al))
                    e /= max(1.0, 2.0 * n + 1.0)   # entries grow like 2j+1 for 3/2 -> 1/2
                elif n <= 4096:
                    e = np.max(np.abs(gi - oracle.jac2cheb(al, *params))) / np.sum(np.abs(al))
                else:
                    # degree 2^18: the oracle's sampled-row route (unit step of the first
                    # parameter by its bidiagonal factor, then the reflected stage on the rows)
                    r = inputs.sample_rows(n, 64, seed=i)
                    ref = oracle.jac2cheb_rows(al, *params, r)
                    e = np.max(np.abs(gi[r] - ref)) / np.sum(np.abs(al))
                if e is not None:
                    worst = max(worst, float(e))
            conf5[f"{kname}_{pname}"] = {"coeffs_per_s": round(bt.coefficients / (ms5 * 1e-3), 1),
                                         "ms_per_batch": round(ms5, 4), "buckets": bt.buckets(),
                                         "max_err_over_l1_sampled": worst}
            del bt
            if short == "jac2cheb":
                conf5[f"dense_alone_{pname}"] = dense_alone(thx, torch, dev, prec, tolh, steps)
    conf5["workload"] = ("65536 vectors of degree 255 + 64 of degree 2^18 in one batch (CSR), alpha_k ~ "
                         "N(0,1)(k+1)^-1 seed 55, hipGraph replay, buckets autotuned; ultraspherical errors "
                         "divided by the entry growth 2N+1; Jacobi checked on the degree-255 members")
    del a5, b5
    return conf5


def main():
    args = parse()
    if args.write_traffic:
        write_traffic(*args.write_traffic)
        return
    if args.write_trace:
        write_trace(*args.write_trace)
        return
    if args.write_counters:
        write_counters(*args.write_counters)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this library runs on a single GPU; --gpus must be 1 "
              "(sharding over several GPUs is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1604_07486_amd import binding as thx
    from paper_1604_07486_amd import inputs

    dev = torch.device("cuda:0")
    N = 1 << args.log2n
    alpha = inputs.coeffs(N, 1.5, seed=20)
    a = torch.from_numpy(alpha).to(dev)
    b = torch.empty_like(a)

    if args.headline_only:
        prec = {"fp64": thx.FP64, "fp32": thx.FP32_BULK, "tail32": thx.FP64_TAIL32}[args.prec]
        if args.shapes:   # read by the library when the plan is created
            os.environ["THX_ROW_LEN"], os.environ["THX_P1_BLOCKS"] = (str(v) for v in args.shapes)
        plan = thx.Plan(thx.LEG2CHEB, N, 1e-7 if prec == thx.FP32_BULK else 1e-15, prec)
        tuned = not (args.no_autotune or args.shapes)
        if tuned:
            plan.autotune(1)
        ms, tim = time_plan(thx, torch, plan, a, b, args.steps, args.warmup, phase="row")
        parts = phase_breakdown(torch, plan, a, b, max(5, args.steps // 5))
        copy_gbs = copy_bandwidth(torch) if args.copy_calibration else None
        es = 8 if prec == thx.FP32_BULK else 16
        S = plan.rank - plan.tail_slots
        pb = {ph: phase_bytes(ph, es, S, N // 2 + 1, plan.fft_length, plan.partial_groups(1))
              for ph in ("col_fwd", "row", "col_inv")}
        print(json.dumps({"headline_only": True, "prec": args.prec, "log2n": args.log2n, "ms_per_step": ms,
                          "autotuned": tuned, "shapes": args.shapes,
                          "fft_geometry": list(plan.fft_geometry()) if plan.path == 2 else None,
                          "p1_blocks": plan.p1_blocks if plan.path == 2 else None,
                          "copy_gbs": copy_gbs, "K": plan.rank, "tail_slots": plan.tail_slots, "L": plan.fft_length,
                          "row_ms_avg": phase_avg(tim).get("row"),
                          "row_kernel": row_kernel_name(plan) if prec == thx.FP64 else None,
                          "row_bytes_per_launch": pb["row"], "phase_bytes": pb,
                          "phases_ms_avg": phase_avg(parts)}), flush=True)
        return

    import oracle

    if args.only:
        precs = ({"fp64": "fp64", "fp32": "fp32_bulk", "tail32": "fp64_tail32"}[args.prec],)
        if args.only == "batched":
            res = run_batched(thx, torch, inputs, oracle, dev, args.steps, precs=precs)
        elif args.only == "sweep":
            res = {"precision_sweep": run_sweep(thx, torch, inputs, oracle, dev, args.steps)}
        elif args.only == "config1":
            res = {"config1": run_config1(thx, torch, inputs, oracle, dev, args.steps)}
        elif args.only == "dense":
            prec = thx.FP64 if precs[0] == "fp64" else thx.FP32_BULK
            res = {"dense_alone": dense_alone(thx, torch, dev, prec, 1e-15 if prec == thx.FP64 else 1e-7, args.steps)}
            if args.copy_calibration:
                res["copy_gbs"] = copy_bandwidth(torch)
        else:
            kinds = (args.kind,) if args.kind else ("ultra", "jac2cheb")
            res = run_config5(thx, torch, inputs, oracle, dev, args.steps, kinds=kinds, precs=precs)
        print(json.dumps({"only": args.only, **res}), flush=True)
        return

    # ---- plan (Fig. 1 steps 1-2 + symbol FFT), timed cold ----
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = thx.Plan(thx.LEG2CHEB, N, 1e-15, thx.FP64)
    torch.cuda.synchronize()
    plan_ms = (time.perf_counter() - t0) * 1e3
    t0 = time.perf_counter()
    plan.autotune(1)
    torch.cuda.synchronize()
    tune_ms = (time.perf_counter() - t0) * 1e3

    # per-phase split first (untimed for the value), to name the dominant kernel
    for _ in range(args.warmup):
        plan.execute(a, b)
    parts = phase_breakdown(torch, plan, a, b, max(5, args.steps // 5))
    dname = max(parts.items(), key=lambda kv: kv[1][0])[0]
    ms, tim = time_plan(thx, torch, plan, a, b, args.steps, args.warmup, phase=dname)
    value = (N + 1) / (ms * 1e-3)
    rows = inputs.sample_rows(N, 256, seed=17)
    err64 = sampled_error(oracle, "leg2cheb", alpha, b.cpu().numpy(), rows)

    # ---- roofline of the dominant kernel (live HIP-event timings) ----
    S, L = plan.rank, plan.fft_length
    nc = N // 2 + 1
    es = 16
    dtot, dcount = tim[dname]
    davg_ms = dtot / dcount
    # partial-sum groups of the inverse column pass, as the tuned plan runs it
    Gc = plan.partial_groups(1)
    dbytes = phase_bytes(dname, es, S, nc, L, Gc)
    roof = None
    if dbytes is not None:
        achieved = dbytes / (davg_ms * 1e-3) / 1e9
        traffic = measured_traffic(dname, row_kernel_name(plan), dbytes)
        roof = {"kernel": dname, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "bytes_per_launch": dbytes, "avg_launch_ms": round(davg_ms, 5), "launches": dcount}
    # whole-step algorithmic bytes (all phases) over the step time
    step_bytes = sum(phase_bytes(p, es, S, nc, L, Gc) or 0 for p in ("col_fwd", "row", "col_inv")) \
        + 8 * 2 * (N + 1) + es * nc * (1 + Gc)

    # ---- FP32-bulk at the same N (Lambda, Cholesky, D1/D2 in FP64) ----
    plan32 = thx.Plan(thx.LEG2CHEB, N, 1e-7, thx.FP32_BULK)
    plan32.autotune(1)
    ms32, _ = time_plan(thx, torch, plan32, a, b, args.steps, args.warmup)
    tim32 = phase_breakdown(torch, plan32, a, b, max(5, args.steps // 5))
    err32 = sampled_error(oracle, "leg2cheb", alpha, b.cpu().numpy(), rows)
    K32 = plan32.rank
    del plan32

    # ---- FP64 with the small-pivot ranks in single precision (same tolerance) ----
    plant = thx.Plan(thx.LEG2CHEB, N, 1e-15, thx.FP64_TAIL32)
    plant.autotune(1)
    mst, _ = time_plan(thx, torch, plant, a, b, args.steps, args.warmup)
    timt = phase_breakdown(torch, plant, a, b, max(5, args.steps // 5))
    errt = sampled_error(oracle, "leg2cheb", alpha, b.cpu().numpy(), rows)
    tail32 = {"coeffs_per_s": round((N + 1) / (mst * 1e-3), 1), "ms_per_step": round(mst, 5),
              "K": plant.rank, "fp32_slots": plant.tail_slots, "max_err_over_l1": errt, "bar": 3e-15,
              "hankel_tol": 1e-15, "phases_ms_avg": phase_avg(timt)}
    del plant

    # ---- Chebyshev -> Legendre at the same N (Sec. 5.1) ----
    planc = thx.Plan(thx.CHEB2LEG, N, 1e-15, thx.FP64)
    planc.autotune(1)
    msc, _ = time_plan(thx, torch, planc, a, b, max(5, args.steps // 2), 2)
    errc = sampled_error(oracle, "cheb2leg", alpha, b.cpu().numpy(), rows)
    Kc = planc.rank
    del planc

    conf1 = run_config1(thx, torch, inputs, oracle, dev, args.steps)
    batch_res = run_batched(thx, torch, inputs, oracle, dev, args.steps)
    conf5 = run_config5(thx, torch, inputs, oracle, dev, args.steps)
    sweep = run_sweep(thx, torch, inputs, oracle, dev, args.steps)

    copy_gbs = copy_bandwidth(torch)

    # ---- CPU oracle on a bounded sample of output rows ----
    cpu = None
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        g = inputs.rng(99)
        done_rows, t_used = 0, 0.0
        chunk = 64
        while t_used < args.cpu_seconds:
            r = g.integers(0, N + 1, size=chunk)
            t0 = time.perf_counter()
            oracle.matvec("leg2cheb", alpha, rows=r, nthreads=threads)
            t_used += time.perf_counter() - t0
            done_rows += chunk
            chunk = min(chunk * 2, 4096)
        rows_per_s = done_rows / t_used
        cpu = {"value": round(rows_per_s, 2), "unit": "coeffs/s", "cores": threads, "kind": "oracle",
               "sample": f"{done_rows} uniformly random output rows of leg2cheb at N=2^20 "
                         f"(O(N) each, extended precision) in {t_used:.1f} s; a full conversion "
                         f"would take (N+1)/value = {(N + 1) / rows_per_s:.0f} s (extrapolated)"}
        cpu.update(oracle_extras(oracle, inputs, alpha, N, threads))

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "coeffs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "leg2cheb N=2^20 (1048577 coefficients), batch 1, FP64 end to end, "
                               "alpha_k ~ N(0,1)(k+1)^-1.5 seed 20, Hankel tol 1e-15, plan reused "
                               "(autotuned for one vector)",
                   "N": N, "batch": 1, "K": S, "L": L, "path": plan.path},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": {"fp64_max_err_over_l1": err64, "fp64_bar": 1e-13,
                     "rows_checked": int(len(rows))},
        "plan_ms": round(plan_ms, 2),
        "autotune_ms": round(tune_ms, 2),
        "fft_geometry": list(plan.fft_geometry()) if plan.path == 2 else None,
        "launch_shape": {"lds_blocks": plan.launch_shape()[0], "p3_blocks": plan.launch_shape()[1],
                         "p1_blocks": plan.p1_blocks, "partial_groups": Gc},
        "copy_gbs_measured": round(copy_gbs, 1),
        "step_hbm_gbs_algorithmic": round(step_bytes / (ms * 1e-3) / 1e9, 1),
        "phases_ms_avg": phase_avg(parts),
        "fp32_bulk": {"coeffs_per_s": round((N + 1) / (ms32 * 1e-3), 1), "ms_per_step": round(ms32, 5),
                      "K": K32, "max_err_over_l1": err32, "bar": 5e-6, "hankel_tol": 1e-7,
                      "phases_ms_avg": phase_avg(tim32)},
        "fp64_tail32": tail32,
        "config1": conf1,
        "batched": batch_res,
        "config5": conf5,
        "precision_sweep": sweep,
        "cheb2leg_fp64": {"coeffs_per_s": round((N + 1) / (msc * 1e-3), 1), "ms_per_step": round(msc, 5),
                          "K": Kc, "max_err_over_l1": errc, "hankel_tol": 1e-15},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
