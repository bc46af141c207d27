#!/usr/bin/env python3
"""Benchmark of the loop-internalised contraction kernels on one MI355X.

Headline workload: the FP32 two-GEMM chain D = alpha*(A*B)*C + beta*D with
NI = NJ = NK = NL = 2048 (tmp kept in HBM), inputs uniform in [-1, 1) from
seed 2, alpha = 1.5, beta = 1.2.  One step is one li_mm2 call (two FP32
matrix-core GEMM launches).  W untimed warm-up steps, then K timed steps
between HIP events on the stream the kernels run on; inputs are resident in
HBM before timing starts.

Printed: one JSON line with the contract fields, plus
  roofline      dominant kernel (the FP32 GEMM) vs the FP32 matrix peak,
  cpu_baseline  the FP64 oracle timed on the host cores,
  rows          the other kernels of the path, measured the same way
                (mean of 30 timed runs after one warm-up).
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
    # enough untimed steps (about 15 ms) for the GPU to leave its idle
    # clocks before the timed region starts
    p.add_argument("--warmup", type=int, default=50)
    p.add_argument("--main-only", action="store_true", help="skip the other kernels' rows")
    p.add_argument("--rows-only", action="store_true",
                   help="measure only the rows named by --rows (no headline line)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--timed-only", action="store_true",
                   help="skip the per-step and cold-cache timings of the headline (for kernel "
                        "traces whose mean duration is compared with the timed loop)")
    p.add_argument("--rows", default="gemm256,cov,corr,precision,grouped,forms,paper1024,rank,matvec,vendor",
                   help="comma list of extra rows to measure")
    return p.parse_args()


class Timer:
    """HIP events on torch's current stream (the stream every li_* call uses)."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps, warmup):
        torch = self.torch
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
        fn()
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

    if args.rows_only:
        print(json.dumps({"rows": measure_rows(args, torch, li, synth, timer)}), flush=True)
        return

    # ---------------------------------------------------------------- headline: 2mm 2048^4
    c = synth.workload("mm2_2048")
    NI, NJ, NK, NL = c["NI"], c["NJ"], c["NK"], c["NL"]
    dA, dB, dC = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
    dD0 = torch.from_numpy(c["D"]).cuda()
    dD = dD0.clone()
    tmp = torch.empty((NI, NJ), device="cuda")
    torch.cuda.synchronize()

    def step():
        li.li_mm2(NI, NJ, NK, NL, c["alpha"], c["beta"], dA, dB, tmp, dC, dD)

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
    per_step, ms_cold = None, None
    if not args.timed_only:
        per_step = sorted(timer.time_each(step, args.steps, 0))
        flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
        ms_cold = timer.time_cold(step, 10, flush)
        del flush
    f1 = gemm_flops(NI, NJ, NK)
    f2 = gemm_flops(NI, NL, NJ)
    flops_step = f1 + f2
    value = flops_step / (ms_step * 1e-3) / 1e9
    # every kernel in the step is the FP32 GEMM (two launches of one shape)
    launch_ms = ms_total / (2 * args.steps)
    achieved = f1 / (launch_ms * 1e-3) / 1e12

    # result of one clean step for the error check (D is updated in place)
    dD.copy_(dD0)
    step()
    torch.cuda.synchronize()
    D_gpu = dD.cpu().numpy()

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
                   "global_batch": 1, "parallelism": "single GPU"},
        "roofline": {"bound": "mfma", "kernel": "gemm_f32_kernel (2048x2048x2048)",
                     "achieved": round(achieved, 2), "peak": PEAK_FP32_MFMA, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": committed_traffic()},
    }

    if per_step:
        out["step_ms_stats"] = {"median": round(per_step[len(per_step) // 2], 4),
                                "min": round(per_step[0], 4),
                                "cold_cache_mean": round(ms_cold, 4)}
    if not args.main_only:
        out["rows"] = measure_rows(args, torch, li, synth, timer)

    if not args.no_cpu_baseline:
        out["cpu_baseline"], out["max_rel_err"] = cpu_baseline(c, D_gpu, flops_step)

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


def cpu_baseline(c, D_gpu, flops_step, min_seconds=8.0):
    """The FP64 oracle (plain loop nests) on the host cores, run on the whole
    2mm workload repeatedly for about min_seconds; also gives the normwise
    error of the GPU result."""
    import oracle

    oracle._load()
    runs = 0
    t0 = time.perf_counter()
    while True:
        _, D = oracle.mm2(c["A"], c["B"], c["C"], c["D"], alpha=c["alpha"], beta=c["beta"])
        runs += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds:
            break
    err = oracle.normwise_error(D_gpu, D)
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
    return base, {"2mm_D": err}


def measure_rows(args, torch, li, synth, timer):
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
        del A, B, C0, C

    if "cov" in want or "corr" in want:
        s = synth.workload("stats_4096x2048")
        X = torch.from_numpy(s["data"]).cuda()
        N, M = s["N"], s["M"]
        Y = torch.empty_like(X)
        mean = torch.empty(M, dtype=torch.float64, device="cuda")
        std = torch.empty(M, dtype=torch.float64, device="cuda")
        out = torch.empty((M, M), device="cuda")
        ws = torch.empty(li.li_stats_workspace_bytes(M, N) // 8 + 1, dtype=torch.float64, device="cuda")
        f = syrk_flops(M, N)
        for kind in ("cov", "corr"):
            if kind not in want:
                continue
            if kind == "cov":
                fn = lambda: li.li_covariance(M, N, X, Y, mean, out, ws)
            else:
                fn = lambda: li.li_correlation(M, N, 0.1, X, Y, mean, std, out, ws)
            st = timer.stats(fn, reps, 1)
            ms = st["ms"]
            flush = torch.empty(128 << 20, dtype=torch.float32, device="cuda")
            ms_cold = timer.time_cold(fn, 10, flush)
            del flush
            rows[kind + "_4096x2048"] = dict(st, **{"GFLOP/s": round(f / ms / 1e6, 1),
                                                   "frac_fp32_mfma": round(f / ms / 1e9 / PEAK_FP32_MFMA, 4),
                                                   "ms_cold_cache": round(ms_cold, 4)})
            # the same with the centring fused into the contraction's loads
            if kind == "cov":
                fn = lambda: li.li_covariance_fused(M, N, X, mean, out, ws)
            else:
                fn = lambda: li.li_correlation_fused(M, N, 0.1, X, mean, std, out, ws)
            ms_f = timer.time(fn, reps, 1)
            rows[kind + "_fused_4096x2048"] = {"ms": round(ms_f, 4), "GFLOP/s": round(f / ms_f / 1e6, 1),
                                               "speedup_vs_unfused": round(ms / ms_f, 3)}
        del X, Y, out, ws

    if "precision" in want:
        p = synth.workload("precision_8192")
        M = N = K = 8192
        A, B = torch.from_numpy(p["A"]).cuda(), torch.from_numpy(p["B"]).cuda()
        C = torch.empty((M, N), device="cuda")
        ws = torch.empty(li.li_gemm_ex_workspace_bytes(M, N, K, "bf16x3") // 4 + 1, device="cuda")
        f = gemm_flops(M, N, K)
        for prec in ("fp32", "bf16", "fp16", "bf16x3"):
            fn = lambda: li.li_gemm_ex(M, N, K, 1.0, A, B, 0.0, C, prec, ws)
            ms = timer.time(fn, 10, 1)
            peak = PEAK_FP32_MFMA if prec == "fp32" else PEAK_BF16_MFMA
            rows["gemm_8192_" + prec] = {"ms": round(ms, 3), "TFLOP/s": round(f / ms / 1e9, 1),
                                         "frac_peak": round(f / ms / 1e9 / peak, 4)}
        del A, B, C, ws

    if "grouped" in want:
        rows["grouped"] = measure_grouped(torch, li, synth, timer)

    if "forms" in want:
        # the paper's polybench size (1024): the GEMM in each form the device
        # passes produce, then the production matrix-core kernel
        n = 1024
        c = synth.gemm_inputs(n, n, n, seed=1)
        A, B, C0 = (torch.from_numpy(c[k]).cuda() for k in ("A", "B", "C"))
        C = C0.clone()
        f = gemm_flops(n, n, n)
        res = {}
        for form in ("naive", "reduced", "internalized"):
            ms = timer.time(lambda: li.li_gemm_form(form, n, n, n, 1.5, A, B, 1.2, C), 5, 1)
            res[form] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}
        ms = timer.time(lambda: li.li_gemm(n, n, n, 1.5, A, B, 1.2, C), reps, 1)
        res["matrix_core"] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}
        base = res["naive"]["ms"]
        for k in res:
            res[k]["speedup_vs_naive"] = round(base / res[k]["ms"], 2)
        rows["gemm_1024_forms"] = res
        del A, B, C0, C

    if "paper1024" in want:
        # the four kernels at the paper's problem size 1024
        n = 1024
        m = synth.mm2_inputs(n, n, n, n, seed=2)
        dA, dB, dC, dD = (torch.from_numpy(m[k]).cuda() for k in ("A", "B", "C", "D"))
        tmp = torch.empty((n, n), device="cuda")
        ms = timer.time(lambda: li.li_mm2(n, n, n, n, 1.5, 1.2, dA, dB, tmp, dC, dD), reps, 1)
        rows["mm2_1024"] = {"ms": round(ms, 4), "GFLOP/s": round(2 * gemm_flops(n, n, n) / ms / 1e6, 1)}
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
        ms = timer.time(lambda: li.li_correlation(n, n, 0.1, X, Y, mean, std, out, ws), reps, 1)
        rows["corr_1024"] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1)}

    if "rank" in want:
        # 3mm, syrk, syr2k at the paper's size (1024) and at 2048
        for n in (1024, 2048):
            m = synth.mm3_inputs(n, n, n, n, n, seed=6)
            dA, dB, dC, dD = (torch.from_numpy(m[k]).cuda() for k in ("A", "B", "C", "D"))
            E, F, G = (torch.empty((n, n), device="cuda") for _ in range(3))
            ms = timer.time(lambda: li.li_mm3(n, n, n, n, n, dA, dB, dC, dD, E, F, G), reps, 1)
            f = 3 * 2.0 * n ** 3
            rows["mm3_%d" % n] = {"ms": round(ms, 4), "GFLOP/s": round(f / ms / 1e6, 1),
                                  "frac_fp32_mfma": round(f / ms / 1e9 / PEAK_FP32_MFMA, 4)}
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
            f2 = 2.0 * n * (n + 1) * n + 4.0 * n * n
            ms = timer.time(lambda: li.li_syr2k(n, n, 1.5, A, B, 1.2, C, ws), reps, 1)
            rows["syr2k_%d" % n] = {"ms": round(ms, 4), "GFLOP/s": round(f2 / ms / 1e6, 1),
                                    "frac_fp32_mfma": round(f2 / ms / 1e9 / PEAK_FP32_MFMA, 4)}
            del dA, dB, dC, dD, E, F, G, A, B, C0, C, ws

    if "matvec" in want:
        rows.update(measure_matvec(torch, li, synth, timer))

    if "vendor" in want:
        # context only: the vendor BLAS behind torch.mm (FP32, no TF32) on
        # the headline GEMM shape, next to li_gemm on the same operands
        n = 2048
        torch.backends.cuda.matmul.allow_tf32 = False
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
        rows["vendor_sgemm_2048"] = {"torch_mm_ms": round(ms_v, 4),
                                     "torch_mm_TFLOP/s": round(f / ms_v / 1e9, 1),
                                     "li_gemm_ms": round(ms_l, 4),
                                     "li_gemm_TFLOP/s": round(f / ms_l / 1e9, 1)}
        del A, B, C
    return rows


def measure_matvec(torch, li, synth, timer):
    """atax at 4096, bicg / mvt / gesummv at 16384 (the paper's sizes);
    HBM-bound: GB/s of algorithmic traffic (each matrix once, each vector
    read or written once) against the HBM peak."""
    out = {}
    c = synth.matvec_inputs(4096, 4096, seed=8)
    A = torch.from_numpy(c["A"]).cuda()
    vec = {k: torch.from_numpy(c[k]).cuda() for k in ("x",)}
    M = N = 4096
    ws = torch.empty(li.li_matvec_workspace_bytes(M, N) // 4 + 1, device="cuda")
    t, y = torch.empty(M, device="cuda"), torch.empty(N, device="cuda")
    fn = lambda: li.li_atax(M, N, A, vec["x"], t, y, ws)
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
    del A, ws
    M = N = 16384
    c = synth.matvec_inputs(M, N, seed=9, with_b=True)
    A, B = torch.from_numpy(c["A"]).cuda(), torch.from_numpy(c["B"]).cuda()
    v = {k: torch.from_numpy(c[k]).cuda() for k in ("x", "p", "r", "y1", "y2", "x1", "x2")}
    ws = torch.empty(li.li_matvec_workspace_bytes(M, N) // 4 + 1, device="cuda")
    o1, o2 = torch.empty(M, device="cuda"), torch.empty(N, device="cuda")
    cases = {
        "bicg": (lambda: li.li_bicg(M, N, A, v["p"], v["r"], o1, o2, ws), 4.0 * (M * N + 2 * (M + N))),
        "mvt": (lambda: li.li_mvt(M, N, A, v["y1"], v["y2"], v["x1"], v["x2"], ws),
                4.0 * (M * N + 3 * (M + N))),
        "gesummv": (lambda: li.li_gesummv(M, N, 1.5, 1.2, A, B, v["x"], o1, o2, ws),
                    4.0 * (2 * M * N + N + 2 * M)),
    }
    for name, (fn, b) in cases.items():
        ms = timer.time(fn, 10, 1)
        out[name + "_16384"] = {"ms": round(ms, 4), "GB/s": round(b / ms / 1e6, 1),
                                "frac_hbm": round(b / ms / 1e6 / PEAK_HBM, 4)}
    del A, B, ws
    return out


def measure_grouped(torch, li, synth, timer):
    b = synth.workload("batch_512_512")
    keep = []
    probs = []
    for d in b.gemm:
        A, B, C = (torch.from_numpy(d[k]).cuda() for k in ("A", "B", "C"))
        keep += [A, B, C]
        probs.append(li.make_problem(li.LI_PROBLEM_GEMM, d["M"], d["N"], d["K"], d["alpha"], d["beta"],
                                     A, B, C))
    for d in b.cov:
        X = torch.from_numpy(d["data"]).cuda()
        Y = torch.empty_like(X)
        mean = torch.empty(d["M"], dtype=torch.float64, device="cuda")
        cov = torch.empty((d["M"], d["M"]), device="cuda")
        keep += [X, Y, mean, cov]
        probs.append(li.make_problem(li.LI_PROBLEM_COVARIANCE, d["M"], d["N"], 0, 1.0, 0.0, X, None, cov,
                                     Y, mean))
    plan = li.li_group_plan_create(probs)
    f = plan.flops
    ms_g = timer.time(plan.launch, 30, 1)
    ms_l = timer.time(plan.launch_loop, 5, 1)
    plan.close()
    return {"instances": len(probs), "GFLOP": round(f / 1e9, 3), "grouped_ms": round(ms_g, 4),
            "grouped_GFLOP/s": round(f / ms_g / 1e6, 1), "loop_ms": round(ms_l, 4),
            "loop_GFLOP/s": round(f / ms_l / 1e6, 1), "speedup": round(ms_l / ms_g, 2)}


if __name__ == "__main__":
    main()
