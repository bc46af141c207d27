#!/usr/bin/env python3
"""Summaries of rocprofv3 results (SQLite output) for profiles/.

  profsum.py trace DB OUT.md --cmd "..."
      per-kernel dispatch count and mean / min / max duration
  profsum.py hbm FETCH_DB WRITE_DB OUT.md --kernel SUBSTR --copy-bytes B --cmd "..."
      HBM traffic per dispatch of the kernels matching SUBSTR from the
      FETCH_SIZE and WRITE_SIZE counters (KiB per dispatch), each scaled by
      what the same counter reads for the plain device copy of B bytes that
      the profiled program runs (the largest copy kernel dispatch)
  profsum.py pmc DB[,DB2] OUT.md --kernel SUBSTR [--kernel SUBSTR2] --cmd "..."
      mean of every collected counter per dispatch for each kernel (after
      --skip dispatches), plus matrix-core utilisation when
      SQ_VALU_MFMA_BUSY_CYCLES and GRBM_GUI_ACTIVE are present; several
      counter runs' databases and commands (joined by " ;; ") may be given

Every summary records the command that produced the database and a hash of
the kernel sources, so a reader can tell whether the numbers still describe
the current kernels.
"""
import argparse
import collections
import hashlib
import os
import sqlite3

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ["csrc/f32_tile.h", "csrc/gemm_f32.hip", "csrc/tiles.h", "csrc/stats.hip",
                  "csrc/stats_dev.h", "csrc/gemm_lp.hip", "csrc/grouped.hip", "csrc/symm_kernels.h",
                  "csrc/symm_rows.hip", "csrc/matvec.hip", "csrc/cov_fused.hip", "tune_gfx950.txt"]


def source_hash(files=KERNEL_SOURCES):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(PKG, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hash_line(files):
    """'Kernel sources hash: `H` (files: a, b)' for the given package files."""
    return "Kernel sources hash: `%s` (files: %s)" % (source_hash(files), ", ".join(files))


def parse_hash_line(text):
    """(hash, files) from a summary's hash line, or (None, None)."""
    import re
    m = re.search(r"Kernel sources hash: `([0-9a-f]+)`(?: \(files: ([^)]*)\))?", text)
    if not m:
        return None, None
    files = [f.strip() for f in m.group(2).split(",")] if m.group(2) else list(KERNEL_SOURCES)
    return m.group(1), files


def still_current(text):
    """True when the kernel sources named in a summary are unchanged."""
    h, files = parse_hash_line(text)
    if h is None:
        return False
    try:
        return h == source_hash(files)
    except OSError:
        return False


def short(name, n=150):
    return name if len(name) <= n else name[: n - 3] + "..."


def trace(args):
    con = sqlite3.connect(args.db)
    rows = con.execute("select name, duration from kernels order by start").fetchall()
    agg = collections.OrderedDict()
    for n, d in rows:
        agg.setdefault(n, []).append(d / 1e3)
    total = sum(sum(v) for v in agg.values())
    lines = ["# Kernel trace: %s" % args.title, "",
             "Command: `%s`" % args.cmd, "",
             hash_line(args.sources), "",
             "| kernel | calls | mean us | min us | max us | share of GPU time |",
             "|---|---|---|---|---|---|"]
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| `%s` | %d | %.2f | %.2f | %.2f | %.1f%% |" % (
            short(n), len(v), sum(v) / len(v), min(v), max(v), 100.0 * sum(v) / total))
    if args.timed_kernel:
        # the launches after the warm-up ones: those of the timed loop (and
        # whatever the program runs after it), to compare with its clock
        for n, v in agg.items():
            if args.timed_kernel in n and len(v) > args.skip:
                t = v[args.skip:]
                lines += ["", "Launches %d onwards of `%s` (after the %d warm-up launches, whose "
                          "clocks are still rising): %d launches, mean %.2f us, median %.2f us." % (
                              args.skip + 1, short(n)[:80], args.skip, len(t), sum(t) / len(t),
                              sorted(t)[len(t) // 2])]
                lines.append("timed_mean_us: %.3f" % (sum(t) / len(t)))
    open(args.out, "w").write("\n".join(lines) + "\n")


def _counter(db, name):
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, dispatch_id, value from counters_collection "
                       "where counter_name=? order by dispatch_id", (name,)).fetchall()
    return rows


def hbm(args):
    fetch = _counter(args.fetch_db, "FETCH_SIZE")
    write = _counter(args.write_db, "WRITE_SIZE")
    copy_kib = args.copy_bytes / 1024.0
    cf = max(v for n, d, v in fetch if "copyBuffer" in n)
    cw = max(v for n, d, v in write if "copyBuffer" in n)
    f_scale = copy_kib / cf
    w_scale = copy_kib / cw
    fk = [v for n, d, v in fetch if args.kernel in n]
    wk = [v for n, d, v in write if args.kernel in n]
    kname = next(n for n, d, v in fetch if args.kernel in n)
    fb = sum(fk) / len(fk) * f_scale * 1024
    wb = sum(wk) / len(wk) * w_scale * 1024
    lines = ["# HBM traffic: %s" % args.title, "",
             "Commands (one counter per run):", "",
             "    %s" % args.cmd.replace("COUNTER", "FETCH_SIZE"),
             "    %s" % args.cmd.replace("COUNTER", "WRITE_SIZE"), "",
             hash_line(args.sources), "",
             "Kernel: `%s` (%d dispatches)" % (short(kname, 140), len(fk)), "",
             "Calibration: the program copies %d bytes device-to-device once; the copy "
             "dispatch reads FETCH_SIZE = %.1f KiB and WRITE_SIZE = %.1f KiB, so the "
             "scale factors are %.4f (fetch) and %.4f (write)." % (args.copy_bytes, cf, cw, f_scale, w_scale), "",
             "| per dispatch | raw KiB | scaled bytes |", "|---|---|---|",
             "| FETCH_SIZE | %.1f | %.4g |" % (sum(fk) / len(fk), fb),
             "| WRITE_SIZE | %.1f | %.4g |" % (sum(wk) / len(wk), wb), "",
             "traffic_bytes_per_launch: %.6g" % (fb + wb)]
    if args.algorithmic:
        lines.append("")
        lines.append("Algorithmic bytes per launch: %.4g; measured / algorithmic = %.2f" % (
            args.algorithmic, (fb + wb) / args.algorithmic))
    open(args.out, "w").write("\n".join(lines) + "\n")


def pmc(args):
    """Counters per dispatch of each --kernel (the last --skip-first... none:
    every matching dispatch after --skip of them is averaged)."""
    lines = ["# Counters: %s" % args.title, "", "Commands (one run per counter set):", ""]
    lines += ["    %s" % c for c in args.cmd.split(" ;; ")]
    lines += ["", hash_line(args.sources)]
    for db in args.db.split(","):
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, dispatch_id, counter_name, value from counters_collection "
                           "order by dispatch_id").fetchall()
        for want in args.kernel:
            agg = collections.OrderedDict()
            kname = None
            for n, d, c, v in rows:
                if want in n:
                    kname = n
                    agg.setdefault(c, []).append(v)
            agg = {c: v[args.skip:] if len(v) > args.skip else v for c, v in agg.items()}
            mean = {c: sum(v) / len(v) for c, v in agg.items()}
            lines += ["", "Kernel: `%s` (%d dispatches averaged)" % (
                short(kname or "?", 140), len(next(iter(agg.values()))) if agg else 0), "",
                "| counter | mean per dispatch |", "|---|---|"]
            for c, v in mean.items():
                lines.append("| %s | %.6g |" % (c, v))
            if "SQ_VALU_MFMA_BUSY_CYCLES" in mean and "GRBM_GUI_ACTIVE" in mean:
                simds = args.cus * 4
                cycles = mean["GRBM_GUI_ACTIVE"] / args.xcds
                util = mean["SQ_VALU_MFMA_BUSY_CYCLES"] / simds / cycles
                lines += ["", "Matrix-core busy fraction = SQ_VALU_MFMA_BUSY_CYCLES / (%d SIMDs x "
                          "GRBM_GUI_ACTIVE / %d XCDs) = %.3f" % (simds, args.xcds, util)]
    open(args.out, "w").write("\n".join(lines) + "\n")


def main():
    p = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = p.add_subparsers(dest="mode", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("out")
    t.add_argument("--timed-kernel", default=None,
                   help="also report this kernel's mean over the launches after --skip")
    t.add_argument("--skip", type=int, default=0, help="warm-up launches of --timed-kernel")
    h = sub.add_parser("hbm")
    h.add_argument("fetch_db")
    h.add_argument("write_db")
    h.add_argument("out")
    h.add_argument("--kernel", required=True)
    h.add_argument("--copy-bytes", type=float, default=256 * 2 ** 20)
    h.add_argument("--algorithmic", type=float, default=None)
    c = sub.add_parser("pmc")
    c.add_argument("db", help="one database, or several joined by commas (one per counter set)")
    c.add_argument("out")
    c.add_argument("--kernel", required=True, action="append",
                   help="kernel name substring (repeat for several kernels)")
    c.add_argument("--skip", type=int, default=0, help="leading dispatches of each kernel left out")
    c.add_argument("--cus", type=int, default=256)
    c.add_argument("--xcds", type=int, default=8)
    for q in (t, h, c):
        q.add_argument("--cmd", required=True)
        q.add_argument("--title", default="")
        q.add_argument("--sources", nargs="+", default=list(KERNEL_SOURCES),
                       help="package files whose hash the summary records")
    a = p.parse_args()
    {"trace": trace, "hbm": hbm, "pmc": pmc}[a.mode](a)


if __name__ == "__main__":
    main()
