"""Summaries of rocprofv3 CSV output for the profiles/ folder.

kernels   per-kernel time table from a --kernel-trace CSV, plus the mean
          duration of the launches of one kernel family that did their full
          work (launches that returned at once because the solve had already
          converged are left out: they last about a microsecond);
counters  mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the same
          kernel family from two --pmc runs, each scaled by what that counter
          reads for a plain device copy of known size, giving HBM bytes per
          Chebyshev step (a kernel that fuses two steps counts twice; the
          "per launch" keys mean per step of the polynomial).

The summary records a digest of the kernel sources, so a reader (bench.py)
can tell whether the counters still describe the kernels that are built.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re
import statistics

HERE = os.path.dirname(os.path.abspath(__file__))
DIGEST_FILES = ("csrc/kernels.hpp", "csrc/op.hpp", "csrc/dfn.hpp", "csrc/common.hpp", "csrc/dia_plan.hpp",
                "csrc/stencil2.hpp", "csrc/lowrank.hpp", "csrc/ltile.hpp", "csrc/reorder.hpp", "csrc/persistent.hpp",
                "csrc/sym_eig.hpp", "csrc/pp_lib.hip", "csrc/batch.hpp", "csrc/batch_persist.hpp", "csrc/pp_batch.hip",
                "build.py")


def _code_only(text: str) -> str:
    """Source text without // comments and blank lines (comment edits keep the digest)."""
    out = []
    for line in text.splitlines():
        if not line.lstrip().startswith("#"):  # keep preprocessor lines and Python comments whole
            line = re.sub(r"//.*$", "", line)
        line = line.rstrip()
        if line:
            out.append(line)
    return "\n".join(out)


def source_digest(root: str = HERE) -> str:
    """Digest of the code (not the comments) of the solver and batch kernel sources."""
    h = hashlib.sha256()
    for rel in DIGEST_FILES:
        with open(os.path.join(root, rel), encoding="utf-8") as f:
            text = f.read()
        if not rel.endswith(".py"):
            text = _code_only(text)
        h.update(rel.encode() + b"\0" + text.encode())
    return h.hexdigest()[:16]


def _full(values, frac=0.25):
    """Indices of the launches that did their full work (>= frac of the family's median)."""
    if not values:
        return []
    med = statistics.median(values)
    return [i for i, v in enumerate(values) if v >= frac * med]


def _steps(name, pair_rx):
    """Chebyshev steps one launch performs (2 for the fused-pair kernel)."""
    return 2 if pair_rx is not None and pair_rx.search(name) else 1


def kernels(trace_csv, match, top=15, pair_match=None):
    rows = list(csv.DictReader(open(trace_csv)))
    by = collections.defaultdict(list)
    for r in rows:
        by[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1000.0)
    total = sum(sum(v) for v in by.values())
    lines = ["%-10s %8s %12s %10s  %s" % ("share", "calls", "total_ms", "avg_us", "kernel")]
    for nm, v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append("%9.2f%% %8d %12.3f %10.2f  %s" % (100 * sum(v) / total, len(v), sum(v) / 1e3,
                                                        sum(v) / len(v), nm[:150]))
    rx = re.compile(match)
    prx = re.compile(pair_match) if pair_match else None
    fam = [(d, _steps(nm, prx)) for nm, v in by.items() if rx.search(nm) for d in v]
    # full launches per kernel name (a pair lasts about twice a single step)
    keep = []
    for nm, v in by.items():
        if rx.search(nm):
            keep += [(v[i], _steps(nm, prx)) for i in _full(v)]
    steps = sum(st for _, st in keep)
    return lines, dict(launches=len(fam), full_launches=len(keep), steps=steps,
                       mean_full_us=sum(d for d, _ in keep) / max(1, steps))


def stats_table(stats_csv, top=16):
    """Per-kernel table from a rocprofv3 --stats kernel_stats CSV (when the trace is too large to keep)."""
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["%-10s %8s %12s %10s  %s" % ("share", "calls", "total_ms", "avg_us", "kernel")]
    for r in rows[:top]:
        lines.append("%9.2f%% %8d %12.3f %10.2f  %s" % (float(r["Percentage"]), int(r["Calls"]),
                                                        float(r["TotalDurationNs"]) / 1e6,
                                                        float(r["AverageNs"]) / 1e3, r["Name"][:150]))
    return lines


def _counter(path, name):
    out = []
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name", name) == name:
            out.append((r["Kernel_Name"], float(r["Counter_Value"])))
    return out


def counters(fetch_csv, write_csv, match, calib_match, calib_bytes, pair_match=None):
    """Mean FETCH / WRITE (KiB) per Chebyshev step of the matched kernels (a fused
    pair counts as two steps), each counter scaled by the calibration copy."""
    rx, cx = re.compile(match), re.compile(calib_match)
    prx = re.compile(pair_match) if pair_match else None
    f, w = _counter(fetch_csv, "FETCH_SIZE"), _counter(write_csv, "WRITE_SIZE")
    cal_f = max((v for nm, v in f if cx.search(nm)), default=0.0)
    cal_w = max((v for nm, v in w if cx.search(nm)), default=0.0)
    if cal_f <= 0 or cal_w <= 0:
        raise SystemExit("calibration copy not found in the counter output")
    kf = calib_bytes / (cal_f * 1024.0)
    kw = calib_bytes / (cal_w * 1024.0)

    def per_step(vals):
        # launches classified per kernel name by their own counter (the FETCH
        # and WRITE runs are separate processes)
        by = collections.defaultdict(list)
        for nm, v in vals:
            if rx.search(nm):
                by[nm].append(v)
        tot, steps, n = 0.0, 0, 0
        for nm, v in by.items():
            for i in _full(v):
                tot += v[i]
                steps += _steps(nm, prx)
                n += 1
        return tot / max(1, steps), n, steps

    fetch_kib, nf, sf = per_step(f)
    write_kib, _, _ = per_step(w)
    nall = sum(1 for nm, _ in f if rx.search(nm))
    return dict(calib_fetch_kib=cal_f, calib_write_kib=cal_w, fetch_factor=kf, write_factor=kw,
                launches=nall, full_launches=nf, steps=sf, fetch_kib=fetch_kib, write_kib=write_kib,
                traffic_bytes_per_launch=fetch_kib * 1024.0 * kf + write_kib * 1024.0 * kw)


def read_summary(path):
    """key: value lines of a summary written by this module (others ignored)."""
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        m = re.match(r"^([a-z_]+):\s*(.*)$", line.strip())
        if m:
            out[m.group(1)] = m.group(2)
    return out


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("--trace", required=True)
    k.add_argument("--match", required=True)
    k.add_argument("--title", required=True)
    k.add_argument("--command", required=True)
    k.add_argument("--out", required=True)
    k.add_argument("--field", action="append", default=[], help="extra KEY=VALUE line")
    k.add_argument("--pair-match", default=None, help="kernels that perform two steps per launch")
    t = sub.add_parser("stats")
    t.add_argument("--stats", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--field", action="append", default=[], help="extra KEY=VALUE line")
    c = sub.add_parser("counters")
    c.add_argument("--fetch", required=True)
    c.add_argument("--write", required=True)
    c.add_argument("--match", required=True)
    c.add_argument("--calib-match", required=True)
    c.add_argument("--calib-bytes", type=float, required=True)
    c.add_argument("--algorithmic-bytes", type=float, required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--field", action="append", default=[], help="extra KEY=VALUE line")
    c.add_argument("--pair-match", default=None, help="kernels that perform two steps per launch")
    a = ap.parse_args()
    extra = "".join("%s: %s\n" % tuple(f.split("=", 1)) for f in a.field)
    if a.cmd == "stats":
        with open(a.out, "w") as fo:
            fo.write("# %s\n\ncommand: %s\nsource_digest: %s\n" % (a.title, a.command, source_digest()))
            fo.write(extra + "\n")
            fo.write("\n".join(stats_table(a.stats)) + "\n")
    elif a.cmd == "kernels":
        lines, fam = kernels(a.trace, a.match, pair_match=a.pair_match)
        with open(a.out, "w") as fo:
            fo.write("# %s\n\ncommand: %s\nsource_digest: %s\nmatch: %s\n" % (a.title, a.command,
                                                                              source_digest(), a.match))
            if a.pair_match:
                fo.write("pair_match: %s\n" % a.pair_match)
            fo.write(extra)
            fo.write("launches: %d\nfull_launches: %d\nsteps: %d\nmean_full_us: %.2f\n\n" %
                     (fam["launches"], fam["full_launches"], fam["steps"], fam["mean_full_us"]))
            fo.write("\n".join(lines) + "\n")
    else:
        r = counters(a.fetch, a.write, a.match, a.calib_match, a.calib_bytes, a.pair_match)
        with open(a.out, "w") as fo:
            fo.write("# %s\n\ncommand: %s\nsource_digest: %s\nmatch: %s\n" % (a.title, a.command,
                                                                              source_digest(), a.match))
            if a.pair_match:
                fo.write("pair_match: %s\n" % a.pair_match)
            fo.write(extra)
            fo.write("calibration: plain device copy of %d bytes read %.1f KiB FETCH_SIZE and %.1f KiB "
                     "WRITE_SIZE\n" % (a.calib_bytes, r["calib_fetch_kib"], r["calib_write_kib"]))
            fo.write("fetch_factor: %.4f\nwrite_factor: %.4f\n" % (r["fetch_factor"], r["write_factor"]))
            fo.write("launches: %d\nfull_launches: %d\nsteps: %d\n" % (r["launches"], r["full_launches"],
                                                                        r["steps"]))
            fo.write("fetch_kib_per_step: %.1f\nwrite_kib_per_step: %.1f\n" % (r["fetch_kib"], r["write_kib"]))
            fo.write("traffic_bytes_per_launch: %.0f\nalgorithmic_bytes_per_launch: %.0f\n"
                     % (r["traffic_bytes_per_launch"], a.algorithmic_bytes))
            fo.write("traffic_over_algorithmic: %.4f\n" % (r["traffic_bytes_per_launch"] / a.algorithmic_bytes))


if __name__ == "__main__":
    main()
