#!/usr/bin/env python3
"""Tile-shape search for the kernel families of libli.so.

For each family and size bucket, every compiled candidate is forced in turn
(li_tune_force) and the ordinary entry point is timed with HIP events on
the current stream (1 warm-up, then the mean of `reps` calls); the fastest
candidate is written to the table (li_tune_set) and the table is saved as
text (li_tune_save), which li.py loads at import.

Representative problems per bucket (bucket = bit length of max(M, N, K)):
square GEMMs 256 .. 8192, the 2048^4 two-GEMM chain's shape, covariance of
N = 2 M samples for M = 256 .. 2048, square syrk of order 256 .. 4096 and
square reduced-precision GEMMs.

Usage: python -m paper_2312_13170_amd.autotune [--out PATH] [--quick]
"""
import argparse
import json
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
if os.path.dirname(HERE) not in sys.path:
    sys.path.insert(0, os.path.dirname(HERE))

from paper_2312_13170_amd import li, synth  # noqa: E402


def time_call(fn, reps):
    fn()
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / reps


def gemm_case(n):
    A = torch.from_numpy(synth.uniform_pm1(90, "A", (n, n))).cuda()
    B = torch.from_numpy(synth.uniform_pm1(90, "B", (n, n))).cuda()
    C = torch.from_numpy(synth.uniform_pm1(90, "C", (n, n))).cuda()
    return (n, n, n), lambda: li.li_gemm(n, n, n, 1.5, A, B, 1.2, C)


def syrk_case(m):
    n = 2 * m
    X = torch.from_numpy(synth.uniform_pm1(91, "X", (n, m))).cuda()
    Y = torch.empty_like(X)
    mean = torch.empty(m, dtype=torch.float64, device="cuda")
    cov = torch.empty((m, m), device="cuda")
    ws = torch.empty(li.li_stats_workspace_bytes(m, n) // 8 + 1, dtype=torch.float64, device="cuda")
    return (m, m, n), lambda: li.li_covariance(m, n, X, Y, mean, cov, ws)


def lp_case(n, prec):
    A = torch.from_numpy(synth.uniform_pm1(92, "A", (n, n))).cuda()
    B = torch.from_numpy(synth.uniform_pm1(92, "B", (n, n))).cuda()
    C = torch.empty((n, n), device="cuda")
    ws = torch.empty(li.li_gemm_ex_workspace_bytes(n, n, n, prec) // 4 + 1, device="cuda")
    return (n, n, n), lambda: li.li_gemm_ex(n, n, n, 1.0, A, B, 0.0, C, prec, ws)


def rank_case(n):
    A = torch.from_numpy(synth.uniform_pm1(93, "A", (n, n))).cuda()
    C = torch.from_numpy(synth.uniform_pm1(93, "C", (n, n))).cuda()
    ws = torch.empty(li.li_syrk_workspace_bytes(n, n) // 4 + 1, device="cuda")
    return (n, n, n), lambda: li.li_syrk(n, n, 1.5, A, 1.2, C, ws)


def warm_up(fn, seconds=0.5):
    """Run until the GPU has left its idle clocks, so the first candidates
    are not timed at a lower clock than the last."""
    import time
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            fn()
        torch.cuda.synchronize()


def search(kernel, cases, reps, log, passes=2):
    for label, (shape, fn) in cases:
        bucket = li.li_tune_bucket(*shape)
        n = li.li_tune_num_candidates(kernel)
        warm_up(fn)
        # every candidate timed in `passes` sweeps, the best sweep kept, so
        # clock drift during a sweep does not decide the winner
        times = {}
        for p in range(passes):
            order = range(n) if p % 2 == 0 else range(n - 1, -1, -1)
            for idx in order:
                li.li_tune_force(kernel, idx)
                t = time_call(fn, reps)
                times[idx] = min(times.get(idx, t), t)
        li.li_tune_force(kernel, -1)
        best = min(times, key=times.get)
        li.li_tune_set(kernel, bucket, best)
        rec = {"kernel": kernel, "case": label, "bucket": bucket, "best": best,
               "candidate": li.li_tune_candidate(kernel, best),
               "ms": {str(k): round(v, 4) for k, v in times.items()}}
        log.append(rec)
        print(json.dumps(rec), flush=True)


def main():
    p = argparse.ArgumentParser()
    p.add_argument("--out", default=os.path.join(HERE, "tune_gfx950.txt"))
    p.add_argument("--log", default=None, help="also write the timings as JSON lines")
    p.add_argument("--quick", action="store_true", help="fewer sizes and repetitions")
    a = p.parse_args()
    torch.cuda.set_device(0)
    li.li_init()
    reps = 3 if a.quick else 10
    log = []
    gsizes = [512, 2048] if a.quick else [256, 512, 1024, 2048, 4096, 8192]
    search(li.LI_KERNEL_GEMM_F32, [("gemm %d" % n, gemm_case(n)) for n in gsizes], reps, log)
    ssizes = [512, 2048] if a.quick else [256, 512, 1024, 2048]
    search(li.LI_KERNEL_SYRK_F32, [("cov M=%d" % m, syrk_case(m)) for m in ssizes], reps, log)
    rsizes = [1024, 2048] if a.quick else [256, 512, 1024, 2048, 4096]
    search(li.LI_KERNEL_SYRK_ROWS, [("syrk %d" % n, rank_case(n)) for n in rsizes], reps, log)
    lsizes = [2048, 8192] if a.quick else [1024, 2048, 4096, 8192]
    search(li.LI_KERNEL_GEMM_LP, [("bf16x3 %d" % n, lp_case(n, "bf16x3")) for n in lsizes], reps, log)
    li.li_tune_save(a.out)
    if a.log:
        with open(a.log, "w") as f:
            for r in log:
                f.write(json.dumps(r) + "\n")
    print("table written to", a.out, flush=True)


if __name__ == "__main__":
    main()
