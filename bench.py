#!/usr/bin/env python3
"""Benchmark of the loop-internalised contraction kernels on one MI355X.

Headline workload: the FP32 two-GEMM chain D = alpha*(A*B)*C + beta*D with
NI = NJ = NK = NL = 2048 (tmp kept in HBM), inputs uniform in [-1, 1) from
seed 2, alpha = 1.5, beta = 1.2.  One step is one li_mm2 call (two FP32
matrix-core GEMM launches).  W untimed warm-up steps, then K timed steps
between HIP events on the stream the kernels run on; inputs are resident in
HBM before timing starts.

Printed: one JSON line with the contract fields, plus
  roofline      the dominant kernel (the FP32 GEMM launch of the step) against
                the FP32 matrix peak: its flops over its own mean duration,
                K launches of each of the step's two products timed back to
                back between HIP events on their stream,
  step          the whole step's rate against the same peak (launch gaps
                included),
  rows          the other kernels of the path (mean / median / min of 30
                timed calls after 100 ms of untimed calls and one warm-up;
                cold-cache times for the HBM-sized ones),
  cpu_baseline  the FP64 oracle timed on the host cores,
  max_rel_err   every measured result against the FP64 oracle: normwise
                max|x - ref| / max|ref| (and, for the products, the
                componentwise error against |alpha||A||B| + |beta||C|),
                computed by the CPU-baseline leg from one clean call's
                output of each row.

Before the headline's W warm-up steps the same step runs untimed for
--settle-ms milliseconds (default 300): the GPU's clocks take tens of
milliseconds to leave idle, longer than a few warm-up steps last, and a
run that starts timing inside that ramp measures the clock, not the
kernels.  The other rows follow the headline (after the heavy 8192^3 rows
the clocks settle lower, so the headline is not measured after them); each
row's call first runs untimed for 100 ms for the same reason (the GPU
idles while the host builds the row's inputs).  Rows whose call updates
its output in place (beta != 0, mvt's +=) are checked on one clean call
after the timing, from reset outputs.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_MFMA = 157.3   # TFLOP/s, MI355X dense FP32 matrix
PEAK_BF16_MFMA = 2516.6  # TFLOP/s, MI355X dense bf16/fp16 matrix
PEAK_HBM = 8000.0        # GB/s

ROWS_DEFAULT = "gemm256,cov,corr,precision,grouped,forms,paper1024,rank,matvec,vendor"


def gemm_flops(M, N, K):
    """Algorithmic flops of C = alpha*A*B + beta*C."""
    return 2.0 * M * N * K + 3.0 * M * N


def syrk_flops(M, N):
    """Flops of the symmetric contraction of N samples x M features
    (upper triangle including the diagonal, N multiply-adds each)."""
    return float(N) * M * (M + 1)


def parse():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--main-only", action="store_true", help="skip the other kernels' rows")
    p.add_argument("--rows-only", action="store_true",
                   help="measure only the rows named by --rows (no headline line)")
    p.add_argument("--settle-ms", type=float, default=300.0,
                   help="untimed steps run for this long before the warm-up steps, so the "
                        "clocks have left idle")
    p.add_argument("--no-cpu-baseline", action="store_true",
                   help="skip the oracle leg (CPU baseline and error report)")
    p.add_argument("--timed-only", action="store_true",
                   help="skip the per-step and cold-cache timings of the headline (for kernel "
                        "traces whose mean duration is compared with the timed loop)")
    p.add_argument("--stats-profile", choices=["hot", "cold"], default=None,
                   help="only run 20 covariance and 20 correlation calls at 4096 x 2048, with "
                        "(cold) or without (hot) the caches flushed before each, for kernel traces")
    p.add_argument("--lp-profile", action="store_true",
                   help="only run 3 + 10 bf16 products at 8192^3 (the tuned 16-bit kernel with its "
                        "rounding pre-pass), then 3 + 10 vendor bf16 products of the rounded "
                        "operands, for kernel traces and counters")
    p.add_argument("--rows", default=ROWS_DEFAULT, help="comma list of extra rows to measure")
    return p.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every li_* call uses).

    Every measurement first runs the call untimed for settle_ms: between
    rows the host prepares the next inputs and the GPU idles, and its
    clocks take tens of milliseconds to come back up, longer than one
    warm-up call lasts."""

    def __init__(self, torch, settle_ms=100.0):
        self.torch = torch
        self.settle_ms = settle_ms

    def settle(self, fn):
        torch = self.torch
        t0 = time.perf_counter()
        while (time.perf_counter() - t0) * 1e3 < self.settle_ms:
            for _ in range(4):
                fn()
            torch.cuda.synchronize()

    def time(self, fn, reps, warmup):
        torch = self.torch
        self.settle(fn)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps  # ms per call

    def stats(self, fn, reps, warmup):
        """mean, median and min of per-call times (ms)."""
        t = sorted(self.time_each(fn, reps, warmup))
        return {"ms": round(sum(t) / len(t), 4), "ms_median": round(t[len(t) // 2], 4),
                "ms_min": round(t[0], 4)}

    def time_cold(self, fn, reps, flush):
        """mean ms per call with the 256 MB MALL and the L2s flushed before
        every call (a 512 MiB buffer is written first, outside the timed
        events)."""
        torch = self.torch
        self.settle(fn)
        total = 0.0
        for _ in range(reps):
            flush.fill_(1.0)
            s = torch.cuda.Event(enable_timing=True)
            e = torch.cuda.Event(enable_timing=True)
            s.record()
            fn()
            e.record()
            torch.cuda.synchronize()
            total += s.elapsed_time(e)
        return total / reps

    def time_each(self, fn, reps, warmup):
        """per-call times (ms) for mean / median / min."""
        torch = self.torch
        self.settle(fn)
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record()
        for i in range(reps):
            fn()
            ev[i + 1].record()
        torch.cuda.synchronize()
        return [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]


def calib_copy(torch):
    """A plain 256 MiB device copy: the reference kernel for scaling the
    FETCH_SIZE / WRITE_SIZE counters of a profiled run."""
    a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    del a, b


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the kernels run on a single MI355X and this "
              "build has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2312_13170_amd import li, synth

    torch.cuda.set_device(0)
    li.li_init()
    timer = Timer(torch)
    calib_copy(torch)

    if args.stats_profile:
        stats_profile(args.stats_profile, torch, li, synth)
        return
    if args.lp_profile:
        lp_profile(torch, li, synth)
        return

    checks = []  # (result name, fn(oracle) -> error dict), run by the oracle leg
    rows = None
    if args.rows_only:
        rows = measure_rows(args, torch, li, synth, timer, checks)
        out = {"rows": rows}
        if not args.no_cpu_baseline:
            out["max_rel_err"] = run_checks(checks)
        print(json.dumps(out), flush=True)
        return
    # ---------------------------------------------------------------- headline: 2mm 2048^4
    c = synth.workload("mm2_2048")
    NI, NJ, NK, NL = c["NI"], c["NJ"], c["NK"], c["NL"]
    alpha, beta = c["alpha"], c["beta"]
    dA, dB, dC = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
    dD0 = torch.from_numpy(c["D"]).cuda()
    dD = dD0.clone()
    tmp = torch.empty((NI, NJ), device="cuda")
    torch.cuda.synchronize()

    def step():
        li.li_mm2(NI, NJ, NK, NL, alpha, beta, dA, dB, tmp, dC, dD)

    settle_steps = 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < args.settle_ms:
        for _ in range(10):
            step()
        settle_steps += 10
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    t_start.record()
    for _ in range(args.steps):
        step()
    t_end.record()
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
    ms_step = ms_total / args.steps
    f1 = gemm_flops(NI, NJ, NK)
    f2 = gemm_flops(NI, NL, NJ)
    flops_step = f1 + f2
    value = flops_step / (ms_step * 1e-3) / 1e9

    # The dominant kernel on its own: each of the step's two GEMM launches
    # (li_gemm with li_mm2's arguments) repeated K times back to back between
    # two events recorded on the stream they run on; the mean launch
    # duration is what the committed kernel trace of this command reports
    # for the same launches.  (Events around every single launch add their
    # own gaps, about 4% here; they are reported as well.)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for i in range(args.steps):
        li.li_gemm(NI, NJ, NK, alpha, dA, dB, 0.0, tmp)
    e[1].record()
    for i in range(args.steps):
        li.li_gemm(NI, NL, NJ, 1.0, tmp, dC, beta, dD)
    e[2].record()
    torch.cuda.synchronize()
    d1 = e[0].elapsed_time(e[1]) / args.steps
    d2 = e[1].elapsed_time(e[2]) / args.steps
    launch_ms = (d1 + d2) / 2
    achieved = (f1 + f2) / 2 / (launch_ms * 1e-3) / 1e12
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2 * args.steps)]
    for i in range(args.steps):
        ev[2 * i].record()
        li.li_gemm(NI, NJ, NK, alpha, dA, dB, 0.0, tmp)
        ev[2 * i + 1].record()
    torch.cuda.synchronize()
    each_ms = sum(ev[2 * i].elapsed_time(ev[2 * i + 1]) for i in range(args.steps)) / args.steps

    per_step, ms_cold = None, None
    if not args.timed_only:
        per_step = sorted(timer.time_each(step, args.steps, 0))
        flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
        ms_cold = timer.time_cold(step, 10, flush)
        del flush

    # result of one clean step for the error report (D is updated in place)
    dD.copy_(dD0)
    step()
    torch.cuda.synchronize()
    tmp_gpu, D_gpu = tmp.cpu().numpy(), dD.cpu().numpy()

    out = {
        "metric": "GFLOP/s and % of MFMA/HBM roofline per kernel; max rel err vs FP64 oracle",
        "value": round(value, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2mm FP32 NI=NJ=NK=NL=2048, alpha=1.5, beta=1.2, tmp in HBM, seed 2",
                   "global_batch": 1, "parallelism": "single GPU",
                   "settle": "%d untimed steps (%.0f ms) before the %d warm-up steps" % (
                       settle_steps, args.settle_ms, args.warmup)},
        "roofline": {"bound": "mfma", "kernel": "gemm_f32_kernel 2048x2048x2048 (both launches of the step)",
                     "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": committed_traffic(),
                     "launch_us_mean": round(launch_ms * 1e3, 2),
                     "launch_us_first_product": round(d1 * 1e3, 2),
                     "launch_us_second_product": round(d2 * 1e3, 2),
                     "launch_us_first_product_events_each": round(each_ms * 1e3, 2)},
        "step": {"ms_mean": round(ms_step, 4),
                 "TFLOP/s": round(value / 1e3, 2),
                 "frac_fp32_mfma": round(value / 1e3 / PEAK_FP32_MFMA, 4)},
    }
    if per_step:
        out["step"].update({"ms_median": round(per_step[len(per_step) // 2], 4),
                            "ms_min": round(per_step[0], 4),
                            "ms_cold_cache_mean": round(ms_cold, 4)})
    if not args.main_only:
        rows = measure_rows(args, torch, li, synth, timer, checks)
    if rows is not None:
        out["rows"] = rows

    if not args.no_cpu_baseline:
        checks.insert(0, ("mm2_2048", lambda orc: mm2_errors(orc, c, tmp_gpu, D_gpu)))
        out["cpu_baseline"] = cpu_baseline(c, flops_step)
        out["max_rel_err"] = run_checks(checks)

    print(json.dumps(out), flush=True)


def committed_traffic():
    """HBM bytes per launch of the headline GEMM kernel from the committed
    counter summary, or None when the kernel sources (or the tuning table)
    changed since the counters were taken."""
    import re

    from paper_2312_13170_amd import profsum

    path = os.path.join(ROOT, "profiles", "gemm_f32_2mm_2048_hbm.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    t = re.search(r"traffic_bytes_per_launch: ([0-9.eE+]+)", text)
    if not t or not profsum.still_current(text):
        return None
    return float(t.group(1))


# ------------------------------------------------------------------ oracle leg
# Only the functions below import the oracle (the CPU baseline and the error
# report built from the rows' results).

def cpu_baseline(c, flops_step, min_seconds=8.0):
    """The FP64 oracle (plain loop nests) on the host cores, run on the whole
    2mm workload repeatedly for about min_seconds, plus the plain method on
    one core over sampled rows."""
    import oracle

    oracle._load()
    runs = 0
    t0 = time.perf_counter()
    while True:
        oracle.mm2(c["A"], c["B"], c["C"], c["D"], alpha=c["alpha"], beta=c["beta"])
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    base = {"value": round(runs * flops_step / dt / 1e9, 2), "unit": "GFLOP/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": "the full 2mm 2048^4 workload (34.4 GFLOP) run %d times, %.1f s" % (runs, dt)}
    # the plain method on one core: 256 sampled rows of the same workload
    # (the oracle computes rows independently), scaled to the whole step
    rows = np.arange(0, c["NI"], c["NI"] // 256)
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.mm2(c["A"], c["B"], c["C"], c["D"], alpha=c["alpha"], beta=c["beta"], rows=rows)
    dt1 = time.perf_counter() - t0
    oracle.set_num_threads(threads)
    base["single_thread"] = {"value": round(flops_step * len(rows) / c["NI"] / dt1 / 1e9, 2),
                             "unit": "GFLOP/s", "cores": 1,
                             "sample": "%d of %d rows of the 2mm workload, %.1f s" % (len(rows), c["NI"], dt1)}
    return base


def run_checks(checks):
    import oracle

    oracle._load()
    errs = {}
    t0 = time.perf_counter()
    for name, fn in checks:
        errs[name] = fn(oracle)
    errs["_oracle_seconds"] = round(time.perf_counter() - t0, 1)
    return errs


def nw(x, ref):
    """normwise error max|x - ref| / max|ref|"""
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.max(np.abs(ref))) if ref.size else 0.0
    num = float(np.max(np.abs(x - ref))) if ref.size else 0.0
    return float("%.3g" % (num / den if den > 0 else num))


def comp(x, ref, bound):
    """componentwise error max |x - ref| / bound (bound > 0 elementwise)"""
    d = np.abs(np.asarray(x, dtype=np.float64) - ref) / np.maximum(bound, 1e-300)
    return float("%.3g" % float(np.max(d)))


def mm2_errors(orc, c, tmp_gpu, D_gpu):
    rt, rD = orc.mm2(c["A"], c["B"], c["C"], c["D"], alpha=c["alpha"], beta=c["beta"])
    _, bD = orc.mm2(np.abs(c["A"]), np.abs(c["B"]), np.abs(c["C"]), np.abs(c["D"]),
                    alpha=abs(c["alpha"]), beta=abs(c["beta"]))
    return {"tmp": nw(tmp_gpu, rt), "D": nw(D_gpu, rD), "D_componentwise": comp(D_gpu, rD, bD),
            "sample": "every element"}


# ------------------------------------------------------------------ rows

def stats_profile(kind, torch, li, synth, settle_ms=300.0):
    """20 covariance and 20 correlation calls at 4096 x 2048 (after one of
    each), each preceded by a 512 MiB fill when kind == 'cold'.  Before
    them the covariance runs untimed for settle_ms (with the same fills), so
    the calls do not start at idle clocks; a kernel trace of this mode
    averages the settle calls too."""
    s = synth.workload("stats_4096x2048")
    X = torch.from_numpy(s["data"]).cuda()
    N, M = s["N"], s["M"]
    Y = torch.empty_like(X)
    mean = torch.empty(M, dtype=torch.float64, device="cuda")
    std = torch.empty(M, dtype=torch.float64, device="cuda")
    out = torch.empty((M, M), device="cuda")
    ws = torch.empty(li.li_stats_workspace_bytes(M, N) // 8 + 1, dtype=torch.float64, device="cuda")
    flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda") if kind == "cold" else None
    calls = [lambda: li.li_covariance(M, N, X, Y, mean, out, ws),
             lambda: li.li_correlation(M, N, 0.1, X, Y, mean, std, out, ws)]
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < settle_ms:
        for _ in range(10):
            if flush is not None:
                flush.fill_(1.0)
            calls[0]()
        torch.cuda.synchronize()
    for fn in calls:
        fn()
        for _ in range(20):
            if flush is not None:
                flush.fill_(1.0)
            fn()
        torch.cuda.synchronize()
    print(json.dumps({"stats_profile": kind, "calls": 42}), flush=True)


def lp_profile(torch, li, synth):
    """3 + 10 bf16 products of the 8192^3 precision workload through
    li_gemm_ex, then 3 + 10 vendor (torch.mm) bf16 products of the same
    operands rounded to bf16."""
    c = synth.workload("precision_8192")
    n = c["M"]
    A, B = torch.from_numpy(c["A"]).cuda(), torch.from_numpy(c["B"]).cuda()
    C = torch.empty((n, n), device="cuda")
    ws = torch.empty(li.li_gemm_ex_workspace_bytes(n, n, n, "bf16") // 4 + 1, device="cuda")
    for _ in range(13):
        li.li_gemm_ex(n, n, n, 1.0, A, B, 0.0, C, "bf16", ws)
    torch.cuda.synchronize()
    Ab, Bb = A.bfloat16(), B.bfloat16()
    for _ in range(13):
        torch.mm(Ab, Bb)
    torch.cuda.synchronize()
    print(json.dumps({"lp_profile": "bf16 8192^3", "calls": 13}), flush=True)


def measure_rows(args, torch, li, synth, timer, checks):
    rows = {}
    want = set(r for r in args.rows.split(",") if r)
    reps = 30

    if "gemm256" in want:
        c = synth.workload("gemm_256")
        A, B, C0 = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
        C = C0.clone()
        ms = timer.time(lambda: li.li_gemm(256, 256, 256, 1.5, A, B, 1.2, C), reps, 1)
        f = gemm_flops(256, 256, 256)
        rows["gemm_256"] = {"ms": round(ms, 5), "GFLOP/s": round(f / ms / 1e6, 1), "bound": "launch"}
        C.copy_(C0)
        li.li_gemm(256, 256, 256, 1.5, A, B, 1.2, C)
        out = C.cpu().numpy()

        def chk(orc, c=c, out=out):
            ref = orc.gemm(c["A"], c["B"], c["C"], alpha=1.5, beta=1.2)
            bnd = orc.gemm(np.abs(c["A"]), np.abs(c["B"]), np.abs(c["C"]), alpha=1.5, beta=1.2)
            return {"C": nw(out, ref), "C_componentwise": comp(out, ref, bnd), "sample": "every element"}
        checks.append(("gemm_256", chk))
        del A, B, C0, C

    if "cov" in want or "corr" in want:
        measure_stats(want, torch, li, synth, timer, reps, rows, checks)

    if "precision" in want:
        measure_precision(torch, li, synth, timer, rows, checks)

    if "grouped" in want:
        rows["grouped"] = measure_grouped(torch, li, synth, timer, checks)

    if "forms" in want:
        # the paper's polybench size (1024): the GEMM in each form the device
        # passes produce, then the production matrix-core kernel
        n = 1024
        c = synth.gemm_inputs(n, n, n, seed=1)
        A, B, C0 = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
        C = C0.clone()
        f = gemm_flops(n, n, n)
        res = {}
        outs = {}
        for form in ("naive", "reduced", "internalized"):
            ms = timer.time(lambda: li.li_gemm_form(form, n, n, n, 1.5, A, B, 1.2, C), 5, 1)
            res[form] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}
            C.copy_(C0)
            li.li_gemm_form(form, n, n, n, 1.5, A, B, 1.2, C)
            outs[form] = C.cpu().numpy()
        ms = timer.time(lambda: li.li_gemm(n, n, n, 1.5, A, B, 1.2, C), reps, 1)
        res["matrix_core"] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}
        C.copy_(C0)
        li.li_gemm(n, n, n, 1.5, A, B, 1.2, C)
        outs["matrix_core"] = C.cpu().numpy()
        base = res["naive"]["ms"]
        for k in res:
            res[k]["speedup_vs_naive"] = round(base / res[k]["ms"], 2)
        rows["gemm_1024_forms"] = res

        def chk(orc, c=c, outs=outs):
            ref = orc.gemm(c["A"], c["B"], c["C"], alpha=1.5, beta=1.2)
            d = {k: nw(v, ref) for k, v in outs.items()}
            d["sample"] = "every element"
            return d
        checks.append(("gemm_1024_forms", chk))
        del A, B, C0, C

    if "paper1024" in want:
        measure_paper1024(torch, li, synth, timer, reps, rows, checks)

    if "rank" in want:
        measure_rank(torch, li, synth, timer, reps, rows, checks)

    if "matvec" in want:
        rows.update(measure_matvec(torch, li, synth, timer, checks))

    if "vendor" in want:
        # context only: the vendor BLAS behind torch.mm (FP32, no TF32) on
        # the headline GEMM shape, and on a size between the searched powers
        # of two (its tile chosen for wave quantisation), next to li_gemm on
        # the same operands
        torch.backends.cuda.matmul.allow_tf32 = False
        for n in (2048, 3072):
            c = synth.gemm_inputs(n, n, n, seed=2)
            A, B = torch.from_numpy(c["A"]).cuda(), torch.from_numpy(c["B"]).cuda()
            C = torch.empty((n, n), device="cuda")
            # alternating rounds so both see the same clock state; medians
            tv, tl = [], []
            for _ in range(6):
                tv.append(timer.time(lambda: torch.mm(A, B, out=C), 10, 1))
                tl.append(timer.time(lambda: li.li_gemm(n, n, n, 1.0, A, B, 0.0, C), 10, 1))
            ms_v, ms_l = sorted(tv)[3], sorted(tl)[3]
            f = 2.0 * n ** 3
            rows["vendor_sgemm_%d" % n] = {"torch_mm_ms": round(ms_v, 4),
                                           "torch_mm_TFLOP/s": round(f / ms_v / 1e9, 1),
                                           "li_gemm_ms": round(ms_l, 4),
                                           "li_gemm_TFLOP/s": round(f / ms_l / 1e9, 1)}
            del A, B, C
    return rows


def measure_stats(want, torch, li, synth, timer, reps, rows, checks):
    """covariance / correlation at 4096 samples x 2048 features, unfused and
    fused; errors on the statistics and centred data in full and on 4096
    seeded entries of cov / corr (every diagonal entry among them)."""
    s = synth.workload("stats_4096x2048")
    Xh = s["data"]
    X = torch.from_numpy(Xh).cuda()
    N, M = s["N"], s["M"]
    Y = torch.empty_like(X)
    mean = torch.empty(M, dtype=torch.float64, device="cuda")
    std = torch.empty(M, dtype=torch.float64, device="cuda")
    out = torch.empty((M, M), device="cuda")
    ws = torch.empty(li.li_stats_workspace_bytes(M, N) // 8 + 1, dtype=torch.float64, device="cuda")
    f = syrk_flops(M, N)
    pa = synth.integer_matrix(3, "check_pa", (2048,), 0, M - 1).astype(np.int64)
    pb = synth.integer_matrix(3, "check_pb", (2048,), 0, M - 1).astype(np.int64)
    pa = np.concatenate([pa, np.arange(M)])
    pb = np.concatenate([pb, np.arange(M)])
    for kind in ("cov", "corr"):
        if kind not in want:
            continue
        if kind == "cov":
            fn = lambda: li.li_covariance(M, N, X, Y, mean, out, ws)
            fn_f = lambda: li.li_covariance_fused(M, N, X, mean, out, ws)
        else:
            fn = lambda: li.li_correlation(M, N, 0.1, X, Y, mean, std, out, ws)
            fn_f = lambda: li.li_correlation_fused(M, N, 0.1, X, mean, std, out, ws)
        st = timer.stats(fn, reps, 1)
        ms = st["ms"]
        flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
        ms_cold = timer.time_cold(fn, 10, flush)
        del flush
        rows[kind + "_4096x2048"] = dict(st, **{"GFLOP/s": round(f / ms / 1e6, 1),
                                               "frac_fp32_mfma": round(f / ms / 1e9 / PEAK_FP32_MFMA, 4),
                                               "ms_cold_cache": round(ms_cold, 4)})
        fn()
        torch.cuda.synchronize()
        res = {"Y": Y.cpu().numpy(), "mean": mean.cpu().numpy(), "out": out.cpu().numpy()[pa, pb]}
        if kind == "corr":
            res["std"] = std.cpu().numpy()
        # the same with the centring fused into the contraction's loads
        ms_f = timer.time(fn_f, reps, 1)
        rows[kind + "_fused_4096x2048"] = {"ms": round(ms_f, 4), "GFLOP/s": round(f / ms_f / 1e6, 1),
                                           "speedup_vs_unfused": round(ms / ms_f, 3)}
        fn_f()
        torch.cuda.synchronize()
        res["fused"] = out.cpu().numpy()[pa, pb]

        def chk(orc, kind=kind, res=res):
            corr = kind == "corr"
            rY, rmean, rstd = orc.centred_data(Xh, correlation=corr)
            ref = orc.correlation_entries(Xh, pa, pb) if corr else orc.covariance_entries(Xh, pa, pb)
            # normwise over the sampled entries, against the largest entry of
            # the result (its diagonal for covariance, 1 for correlation)
            scale = 1.0 if corr else float(np.max(np.abs(ref[-M:])))
            d = {"mean": nw(res["mean"], rmean), "data_out": nw(res["Y"], rY),
                 kind: float("%.3g" % (np.max(np.abs(res["out"] - ref)) / scale)),
                 kind + "_fused": float("%.3g" % (np.max(np.abs(res["fused"] - ref)) / scale)),
                 "sample": "%d entries of the %d x %d result (all diagonal ones); mean, stddev and "
                           "centred data in full" % (len(pa), M, M)}
            if corr:
                d["stddev"] = nw(res["std"], rstd)
            return d
        checks.append((kind + "_4096x2048", chk))
    del X, Y, out, ws


def measure_precision(torch, li, synth, timer, rows, checks):
    """GEMM 8192^3 in FP32, bf16, fp16 and split bf16; errors against the
    exact product of the FP32 inputs on 256 seeded rows."""
    p = synth.workload("precision_8192")
    M = N = K = 8192
    A, B = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
    C = torch.empty((M, N), device="cuda")
    ws = torch.empty(li.li_gemm_ex_workspace_bytes(M, N, K, "bf16x3") // 4 + 1, device="cuda")
    f = gemm_flops(M, N, K)
    sample = np.unique(synth.integer_matrix(4, "check_rows", (256,), 0, M - 1).astype(np.int64))
    outs = {}
    for prec in ("fp32", "bf16", "fp16", "bf16x3"):
        fn = lambda: li.li_gemm_ex(M, N, K, 1.0, A, B, 0.0, C, prec, ws)
        ms = timer.time(fn, 10, 1)
        peak = PEAK_FP32_MFMA if prec == "fp32" else PEAK_BF16_MFMA
        rows["gemm_8192_" + prec] = {"ms": round(ms, 3), "TFLOP/s": round(f / ms / 1e9, 1),
                                     "frac_peak": round(f / ms / 1e9 / peak, 4)}
        outs[prec] = C.cpu().numpy()[sample]

    def chk(orc):
        exact = orc.gemm_quantised(p["A"], p["B"], "exact", rows=sample)
        bound = orc.gemm(np.abs(p["A"]), np.abs(p["B"]), rows=sample)
        d = {}
        for prec, o in outs.items():
            d[prec] = nw(o, exact)
            d[prec + "_componentwise"] = comp(o, exact, bound)
        d["sample"] = "%d seeded rows of 8192, against the exact product of the FP32 inputs" % len(sample)
        return d
    checks.append(("gemm_8192", chk))
    del A, B, C, ws


def measure_paper1024(torch, li, synth, timer, reps, rows, checks):
    """the four kernels at the paper's problem size 1024"""
    n = 1024
    m = synth.mm2_inputs(n, n, n, n, seed=2)
    dA, dB, dC, dD0 = (torch.from_numpy(m[k]).cuda() for k in ("A", "B", "C", "D"))
    dD = dD0.clone()
    tmp = torch.empty((n, n), device="cuda")
    ms = timer.time(lambda: li.li_mm2(n, n, n, n, 1.5, 1.2, dA, dB, tmp, dC, dD), reps, 1)
    rows["mm2_1024"] = {"ms": round(ms, 4), "GFLOP/s": round(2 * gemm_flops(n, n, n) / ms / 1e6, 1)}
    dD.copy_(dD0)
    li.li_mm2(n, n, n, n, 1.5, 1.2, dA, dB, tmp, dC, dD)
    D_out = dD.cpu().numpy()
    s = synth.stats_inputs(n, n, seed=3)
    X = torch.from_numpy(s["data"]).cuda()
    Y = torch.empty_like(X)
    mean = torch.empty(n, dtype=torch.float64, device="cuda")
    std = torch.empty(n, dtype=torch.float64, device="cuda")
    out = torch.empty((n, n), device="cuda")
    ws = torch.empty(li.li_stats_workspace_bytes(n, n) // 8 + 1, dtype=torch.float64, device="cuda")
    f = syrk_flops(n, n)
    ms = timer.time(lambda: li.li_covariance(n, n, X, Y, mean, out, ws), reps, 1)
    rows["cov_1024"] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}
    cov_out = out.cpu().numpy()
    ms = timer.time(lambda: li.li_correlation(n, n, 0.1, X, Y, mean, std, out, ws), reps, 1)
    rows["corr_1024"] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}
    corr_out = out.cpu().numpy()

    def chk(orc):
        _, rD = orc.mm2(m["A"], m["B"], m["C"], m["D"], alpha=1.5, beta=1.2)
        _, _, rc = orc.covariance(s["data"], want_y=False)
        _, _, _, rr = orc.correlation(s["data"], want_y=False)
        return {"mm2_D": nw(D_out, rD), "cov": nw(cov_out, rc), "corr": nw(corr_out, rr),
                "sample": "every element"}
    checks.append(("paper_1024", chk))


def measure_rank(torch, li, synth, timer, reps, rows, checks):
    """3mm, syrk, syr2k at the paper's size (1024) and at 2048"""
    for n in (1024, 2048):
        m = synth.mm3_inputs(n, n, n, n, n, seed=6)
        dA, dB, dC, dD = (torch.from_numpy(m[k]).cuda() for k in ("A", "B", "C", "D"))
        E, F, G = (torch.empty((n, n), device="cuda") for _ in range(3))
        ms = timer.time(lambda: li.li_mm3(n, n, n, n, n, dA, dB, dC, dD, E, F, G), reps, 1)
        f = 3 * 2.0 * n ** 3
        rows["mm3_%d" % n] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1),
                              "frac_fp32_mfma": round(f / ms / 1e9 / PEAK_FP32_MFMA, 4)}
        sample = np.arange(0, n, 8)
        G_out = G.cpu().numpy()[sample]
        r = synth.rank_update_inputs(n, n, seed=7)
        A, B, C0 = (torch.from_numpy(r[k]).cuda() for k in ("A", "B", "C"))
        C = C0.clone()
        ws = torch.empty(li.li_syrk_workspace_bytes(n, n) // 4 + 1, device="cuda")
        # flops of the symmetric product counted once per unordered pair
        # (n (n + 1) / 2 dot products of length k; syr2k two of them),
        # plus the update of all n^2 elements
        f1 = float(n) * (n + 1) * n + 3.0 * n * n
        ms = timer.time(lambda: li.li_syrk(n, n, 1.5, A, 1.2, C, ws), reps, 1)
        rows["syrk_%d" % n] = {"ms": round(ms, 4), "GFLOP/s": round(f1 / ms / 1e6, 1),
                               "frac_fp32_mfma": round(f1 / ms / 1e9 / PEAK_FP32_MFMA, 4)}
        C.copy_(C0)
        li.li_syrk(n, n, 1.5, A, 1.2, C, ws)
        syrk_out = C.cpu().numpy()[sample]
        f2 = 2.0 * n * (n + 1) * n + 4.0 * n * n
        ms = timer.time(lambda: li.li_syr2k(n, n, 1.5, A, B, 1.2, C, ws), reps, 1)
        rows["syr2k_%d" % n] = {"ms": round(ms, 4), "GFLOP/s": round(f2 / ms / 1e6, 1),
                                "frac_fp32_mfma": round(f2 / ms / 1e9 / PEAK_FP32_MFMA, 4)}
        C.copy_(C0)
        li.li_syr2k(n, n, 1.5, A, B, 1.2, C, ws)
        syr2k_out = C.cpu().numpy()[sample]

        def chk(orc, m=m, r=r, sample=sample, G_out=G_out, syrk_out=syrk_out, syr2k_out=syr2k_out):
            _, _, rG = orc.mm3(m["A"], m["B"], m["C"], m["D"], rows=sample)
            rs = orc.syrk(r["A"], r["C"], alpha=1.5, beta=1.2, rows=sample)
            rs2 = orc.syr2k(r["A"], r["B"], r["C"], alpha=1.5, beta=1.2, rows=sample)
            return {"mm3_G": nw(G_out, rG), "syrk": nw(syrk_out, rs), "syr2k": nw(syr2k_out, rs2),
                    "sample": "every eighth row"}
        checks.append(("rank_%d" % n, chk))
        del dA, dB, dC, dD, E, F, G, A, B, C0, C, ws


def measure_matvec(torch, li, synth, timer, checks):
    """atax at 4096, bicg / mvt / gesummv at 16384 (the paper's sizes);
    HBM-bound: GB/s of algorithmic traffic (each matrix once, each vector
    read or written once) against the HBM peak."""
    out = {}
    c = synth.matvec_inputs(4096, 4096, seed=8)
    A = torch.from_numpy(c["A"]).cuda()
    x = torch.from_numpy(c["x"]).cuda()
    M = N = 4096
    ws = torch.empty(li.li_matvec_workspace_bytes(M, N) // 4 + 1, device="cuda")
    t, y = torch.empty(M, device="cuda"), torch.empty(N, device="cuda")
    fn = lambda: li.li_atax(M, N, A, x, t, y, ws)
    st = timer.stats(fn, 30, 1)
    ms = st["ms"]
    flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
    ms_cold = timer.time_cold(fn, 10, flush)
    del flush
    b = 4.0 * (M * N + 2 * N + M)
    out["atax_4096"] = dict(st, **{"GB/s": round(b / ms / 1e6, 1),
                                   "frac_hbm": round(b / ms / 1e6 / PEAK_HBM, 4),
                                   "ms_cold_cache": round(ms_cold, 4),
                                   "GB/s_cold_cache": round(b / ms_cold / 1e6, 1)})
    atax_out = (t.cpu().numpy(), y.cpu().numpy())

    def chk_atax(orc):
        rt, ry = orc.atax(c["A"], c["x"])
        return {"tmp": nw(atax_out[0], rt), "y": nw(atax_out[1], ry), "sample": "every element"}
    checks.append(("atax_4096", chk_atax))
    del A, ws
    M = N = 16384
    c2 = synth.matvec_inputs(M, N, seed=9, with_b=True)
    A, B = torch.from_numpy(c2["A"]).cuda(), torch.from_numpy(c2["B"]).cuda()
    v = {k: torch.from_numpy(c2[k]).cuda() for k in ("x", "p", "r", "y1", "y2", "x1", "x2")}
    ws = torch.empty(li.li_matvec_workspace_bytes(M, N) // 4 + 1, device="cuda")
    o1, o2 = torch.empty(M, device="cuda"), torch.empty(N, device="cuda")
    x1, x2 = v["x1"].clone(), v["x2"].clone()
    cases = {
        "bicg": (lambda: li.li_bicg(M, N, A, v["p"], v["r"], o1, o2, ws), 4.0 * (M * N + 2 * (M + N))),
        "mvt": (lambda: li.li_mvt(M, N, A, v["y1"], v["y2"], x1, x2, ws),
                4.0 * (M * N + 3 * (M + N))),
        "gesummv": (lambda: li.li_gesummv(M, N, 1.5, 1.2, A, B, v["x"], o1, o2, ws),
                    4.0 * (2 * M * N + N + 2 * M)),
    }
    res = {}
    for name, (fn, b) in cases.items():
        ms = timer.time(fn, 10, 1)
        out[name + "_16384"] = {"ms": round(ms, 4), "GB/s": round(b / ms / 1e6, 1),
                                "frac_hbm": round(b / ms / 1e6 / PEAK_HBM, 4)}
        if name == "mvt":
            x1.copy_(v["x1"])
            x2.copy_(v["x2"])
            fn()
            res[name] = (x1.cpu().numpy(), x2.cpu().numpy())
        else:
            fn()
            res[name] = (o1.cpu().numpy(), o2.cpu().numpy())

    def chk(orc):
        q, s = orc.bicg(c2["A"], c2["p"], c2["r"])
        a1, a2 = orc.mvt(c2["A"], c2["x1"], c2["x2"], c2["y1"], c2["y2"])
        gt, gy = orc.gesummv(c2["A"], c2["B"], c2["x"], alpha=1.5, beta=1.2)
        return {"bicg_q": nw(res["bicg"][0], q), "bicg_s": nw(res["bicg"][1], s),
                "mvt_x1": nw(res["mvt"][0], a1), "mvt_x2": nw(res["mvt"][1], a2),
                "gesummv_tmp": nw(res["gesummv"][0], gt), "gesummv_y": nw(res["gesummv"][1][:M], gy),
                "sample": "every element"}
    checks.append(("matvec_16384", chk))
    del A, B, ws
    return out


def measure_grouped(torch, li, synth, timer, checks):
    b = synth.workload("batch_512_512")
    keep = []
    probs = []
    gemm_bufs = []
    for d in b.gemm:
        A, B, C = (torch.from_numpy(d[k]).cuda() for k in ("A", "B", "C"))
        keep += [A, B, C]
        gemm_bufs.append(C)
        probs.append(li.make_problem(li.LI_PROBLEM_GEMM, d["M"], d["N"], d["K"], d["alpha"], d["beta"],
                                     A, B, C))
    cov_bufs = []
    for d in b.cov:
        X = torch.from_numpy(d["data"]).cuda()
        Y = torch.empty_like(X)
        mean = torch.empty(d["M"], dtype=torch.float64, device="cuda")
        cov = torch.empty((d["M"], d["M"]), device="cuda")
        keep += [X, Y, mean, cov]
        cov_bufs.append(cov)
        probs.append(li.make_problem(li.LI_PROBLEM_COVARIANCE, d["M"], d["N"], 0, 1.0, 0.0, X, None, cov,
                                     Y, mean))
    plan = li.li_group_plan_create(probs)
    f = plan.flops
    ms_g = timer.time(plan.launch, 30, 1)
    ms_l = timer.time(plan.launch_loop, 5, 1)
    # one clean graph launch (C of the GEMM instances reset) for the errors
    sample = list(range(0, len(b.gemm), 8))
    for i in sample:
        gemm_bufs[i].copy_(torch.from_numpy(b.gemm[i]["C"]))
    plan.launch()
    torch.cuda.synchronize()
    g_out = {i: gemm_bufs[i].cpu().numpy() for i in sample}
    c_out = {i: cov_bufs[i].cpu().numpy() for i in sample}
    plan.close()

    def chk(orc):
        eg = max(nw(g_out[i], orc.gemm(b.gemm[i]["A"], b.gemm[i]["B"], b.gemm[i]["C"], alpha=1.5, beta=1.2))
                 for i in sample)
        ec = max(nw(c_out[i], orc.covariance(b.cov[i]["data"], want_y=False)[2]) for i in sample)
        return {"gemm_max": eg, "cov_max": ec,
                "sample": "%d of 512 GEMM and %d of 512 covariance instances (every eighth)" %
                          (len(sample), len(sample))}
    checks.append(("batch_512_512", chk))
    return {"instances": len(probs), "GFLOP": round(f / 1e9, 3), "grouped_ms": round(ms_g, 4),
            "grouped_GFLOP/s": round(f / ms_g / 1e6, 1), "loop_ms": round(ms_l, 4),
            "loop_GFLOP/s": round(f / ms_l / 1e6, 1), "speedup": round(ms_l / ms_g, 2)}


if __name__ == "__main__":
    main()
