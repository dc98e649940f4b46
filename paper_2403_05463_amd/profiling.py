"""Summaries of rocprofv3 output for the kernels of this library.

``python -m paper_2403_05463_amd.profiling stats <kernel_stats.csv> [--trace <kernel_trace.csv>] --cmd "<command>"``
    per-kernel call count and mean duration from ``--kernel-trace --stats``,
    and with the trace the mean over the dispatches that ran alone;
``python -m paper_2403_05463_amd.profiling traffic <fetch.csv> <write.csv> --copy-bytes B --cmd "<command>"``
    HBM bytes per dispatch from two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
    runs, each scaled by what the same counter reads for the plain copy kernel
    of known size (copy bytes / counter reading);
``python -m paper_2403_05463_amd.profiling timeline <kernel_trace.csv> --kernel <name> [--kernel <name>] --cmd "<command>"``
    start, end, duration and idle gap of the named kernels' dispatches;
``python -m paper_2403_05463_amd.profiling flops <f64.csv> <f32.csv> --cmd64 "<command>" --cmd32 "<command>"``
    floating-point operations per dispatch from ``--pmc SQ_INSTS_VALU_ADD_F64
    SQ_INSTS_VALU_MUL_F64 SQ_INSTS_VALU_FMA_F64 SQ_INSTS_VALU_TRANS_F64`` (and
    the F32 counters): the counters count wave instructions, so FLOPs =
    64 (ADD + MUL + TRANS + 2 FMA), an upper bound that counts every lane of
    a wave, active or not.

The traffic summary records a hash of the kernel sources; ``traffic_for``
returns its figure only while the sources are unchanged.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f) for f in ("hdg_kernels.hip", "hdg_internal.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    m = re.search(r"(k_[a-z_]+)(<[^>]*>)?", name)
    return (m.group(1) + (m.group(2) or "")) if m else name[:48]


def isolated_dispatches(trace_csv: str) -> dict:
    """Per kernel: durations (ns) of the dispatches that overlapped no other
    dispatch in time, i.e. that had the device to themselves (a kernel timed
    with the library's per-launch events runs alone; graph replays overlap
    independent branches)."""
    rows = [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
            for r in csv.DictReader(open(trace_csv))]
    rows.sort()
    out = collections.defaultdict(list)
    reach = -1          # latest end among earlier dispatches
    for i, (s0, e0, k) in enumerate(rows):
        alone = s0 >= reach and (i + 1 == len(rows) or rows[i + 1][0] >= e0)
        reach = max(reach, e0)
        if alone:
            out[k].append(e0 - s0)
    return out


def timer_windows(trace_csv: str, kernel: str, count: int, max_gap_ns: int = 50000) -> list:
    """Mean durations (ns) of `kernel` in each serial window of the trace that
    holds exactly `count` of its dispatches: a window is a run of dispatches
    that each overlapped no other and follow one another within max_gap_ns,
    as the library's kernel timer launches them (one stream, one at a time)."""
    rows = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]))
                  for r in csv.DictReader(open(trace_csv)))
    want = kernel.replace(" ", "")
    out, cur, reach, prev_end = [], [], -1, None
    for i, (s0, e0, k) in enumerate(rows):
        alone = s0 >= reach and (i + 1 == len(rows) or rows[i + 1][0] >= e0)
        reach = max(reach, e0)
        if not alone or (prev_end is not None and s0 - prev_end > max_gap_ns):
            if len(cur) == count:
                out.append(sum(cur) / len(cur))
            cur = []
        if alone:
            if k.replace(" ", "") == want:
                cur.append(e0 - s0)
            prev_end = e0
        else:
            prev_end = None
    if len(cur) == count:
        out.append(sum(cur) / len(cur))
    return out


def stats_summary(path: str, cmd: str, trace_csv: str = None, timer: str = None) -> str:
    rows = list(csv.DictReader(open(path)))
    iso = isolated_dispatches(trace_csv) if trace_csv else {}
    lines = [f"# rocprofv3 kernel statistics", f"command: {cmd}", f"kernel source hash: {kernel_source_hash()}",
             "alone: dispatches that overlapped no other dispatch, and their mean duration" if trace_csv else "", "",
             f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'share':>7s}"
             + (f" {'alone':>6s} {'alone_avg_us':>12s}" if trace_csv else "")]
    for r in rows:
        name = short_name(r["Name"])
        line = (f"{name.replace(' ', ''):40s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}%")
        if trace_csv:
            d = iso.get(name, [])
            line += f" {len(d):6d} {(sum(d) / len(d) / 1e3 if d else float('nan')):12.2f}"
        lines.append(line)
    if trace_csv and timer:
        name, count = timer.rsplit(":", 1)
        means = timer_windows(trace_csv, name, int(count))
        lines += ["", f"kernel timer windows of {name.replace(' ', '')} ({count} dispatches each, one stream, "
                      f"one at a time): mean " + ", ".join(f"{m / 1e3:.2f}" for m in means) + " us"]
    return "\n".join(lines) + "\n"


def timeline_summary(trace_csv: str, kernels: list, cmd: str, first: int = 0, count: int = 30) -> str:
    """Start, end and duration (µs, relative to the first listed dispatch) of
    the dispatches of the named kernels, in start order, from a
    ``--kernel-trace`` run: which launches overlap, and the idle gap between
    dependent ones.  ``first`` skips that many of the matching dispatches."""
    rows = sorted((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), short_name(r["Kernel_Name"]),
                   r.get("Queue_Id", "")) for r in csv.DictReader(open(trace_csv)))
    want = [k.replace(" ", "") for k in kernels]
    rows = [r for r in rows if r[2].replace(" ", "") in want][first:first + count]
    lines = ["# kernel dispatch timeline (rocprofv3 --kernel-trace)", f"command: {cmd}",
             f"kernel source hash: {kernel_source_hash()}", "",
             f"{'start_us':>10s} {'end_us':>10s} {'dur_us':>8s} {'gap_us':>8s} {'queue':>5s}  kernel"]
    if not rows:
        return "\n".join(lines) + "\n"
    t0, reach = rows[0][0], None
    for s0, e0, k, q in rows:
        # gap: idle time since every earlier dispatch ended (negative: overlap)
        gap = "" if reach is None else f"{(s0 - reach) / 1e3:8.1f}"
        lines.append(f"{(s0 - t0) / 1e3:10.1f} {(e0 - t0) / 1e3:10.1f} {(e0 - s0) / 1e3:8.1f} {gap:>8s} {q:>5s}  {k}")
        reach = e0 if reach is None else max(reach, e0)
    return "\n".join(lines) + "\n"


def _per_kernel(path: str, counter: str, counts: dict = None) -> dict:
    """Mean counter value per dispatch of each kernel (a dispatch's rows,
    one per XCD or instance, summed); ``counts`` receives the dispatch count."""
    acc = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[(short_name(r["Kernel_Name"]), r.get("Dispatch_Id", ""))] += float(r["Counter_Value"])
    per = collections.defaultdict(list)
    for (k, _), v in acc.items():
        per[k].append(v)
    if counts is not None:
        counts.update({k: len(v) for k, v in per.items()})
    return {k: sum(v) / len(v) for k, v in per.items()}


def traffic_summary(fetch_csv: str, write_csv: str, copy_bytes: int, cmd_fetch: str, cmd_write: str) -> str:
    counts = {}
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE", counts)
    write = _per_kernel(write_csv, "WRITE_SIZE")
    copy = next(k for k in fetch if k.startswith("k_copy"))
    f_fetch = copy_bytes / (fetch[copy] * 1024.0)
    f_write = copy_bytes / (write[copy] * 1024.0)
    lines = ["# HBM traffic per dispatch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch)",
             f"command (fetch): {cmd_fetch}", f"command (write): {cmd_write}",
             f"kernel source hash: {kernel_source_hash()}",
             f"calibration: plain copy of {copy_bytes} bytes reads FETCH_SIZE {fetch[copy]:.1f} KiB "
             f"and WRITE_SIZE {write[copy]:.1f} KiB; factors fetch {f_fetch:.4f}, write {f_write:.4f}", "",
             f"{'kernel':40s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'traffic_bytes':>16s} {'dispatches':>10s}"]
    for k in sorted(fetch):
        if k not in write:
            continue
        t = fetch[k] * 1024.0 * f_fetch + write[k] * 1024.0 * f_write
        lines.append(f"{k.replace(' ', ''):40s} {fetch[k]:12.1f} {write[k]:12.1f} {t:16.0f} {counts[k]:10d}")
    return "\n".join(lines) + "\n"


def traffic_for(summary_path: str, kernel_prefix: str):
    """Traffic bytes per dispatch of the first kernel starting with ``kernel_prefix``,
    or None if the summary is missing or the kernel sources changed since."""
    if not os.path.exists(summary_path):
        return None
    text = open(summary_path).read()
    m = re.search(r"kernel source hash: (\w+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    want = kernel_prefix.replace(" ", "")
    for line in text.splitlines():
        parts = line.split()
        if len(parts) in (4, 5) and parts[0].startswith(want):
            try:
                return float(parts[3])
            except ValueError:
                return None
    return None


FLOP_COUNTERS = {64: ["SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64", "SQ_INSTS_VALU_FMA_F64",
                      "SQ_INSTS_VALU_TRANS_F64"],
                 32: ["SQ_INSTS_VALU_ADD_F32", "SQ_INSTS_VALU_MUL_F32", "SQ_INSTS_VALU_FMA_F32",
                      "SQ_INSTS_VALU_TRANS_F32"]}
# MI355X peak vector rates (TFLOP/s)
PEAK_TFLOPS = {64: 78.6, 32: 157.3}


def flops_summary(csv64: str, csv32: str, cmd64: str, cmd32: str) -> str:
    lines = ["# floating-point operations per dispatch from VALU instruction counters",
             f"command (FP64 counters): {cmd64}", f"command (FP32 counters): {cmd32}",
             f"kernel source hash: {kernel_source_hash()}",
             "FLOPs = 64 (ADD + MUL + TRANS + 2 FMA) per precision (wave instructions x 64 lanes)", "",
             f"{'kernel':40s} {'flops_f64':>14s} {'flops_f32':>14s}"]
    per = {}
    for bits, path in ((64, csv64), (32, csv32)):
        add, mul, fma, trans = (_per_kernel(path, c) for c in FLOP_COUNTERS[bits])
        for k in fma:
            per.setdefault(k, {})[bits] = 64.0 * (add.get(k, 0) + mul.get(k, 0) + trans.get(k, 0) + 2 * fma[k])
    for k in sorted(per):
        lines.append(f"{k.replace(' ', ''):40s} {per[k].get(64, 0.0):14.4e} {per[k].get(32, 0.0):14.4e}")
    return "\n".join(lines) + "\n"


def flops_for(summary_path: str, kernel_prefix: str, avg_launch_s: float):
    """FLOP count per dispatch of the first kernel starting with ``kernel_prefix``
    and its rate over ``avg_launch_s`` against the peak of the kernel's
    arithmetic type, or None if the summary is missing or the kernel sources
    changed since it was taken."""
    if not os.path.exists(summary_path):
        return None
    text = open(summary_path).read()
    m = re.search(r"kernel source hash: (\w+)", text)
    if not m or m.group(1) != kernel_source_hash():
        return None
    want = kernel_prefix.replace(" ", "")
    bits = 32 if want.startswith("k_residual<float") or want.startswith("k_viscous<float") else 64
    for line in text.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[0].startswith(want):
            f64, f32 = float(parts[1]), float(parts[2])
            main = f64 if bits == 64 else f32
            tf = main / avg_launch_s / 1e12
            return {"flops_per_launch": main, "other_precision_flops": f32 if bits == 64 else f64,
                    "achieved_tflops": tf, "peak_tflops": PEAK_TFLOPS[bits], "frac": tf / PEAK_TFLOPS[bits],
                    "unit": "TFLOP/s", "arith": f"f{bits}"}
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--trace", help="kernel_trace.csv of the same run: adds the dispatches that ran alone")
    s.add_argument("--cmd", required=True)
    s.add_argument("--timer", help="KERNEL:COUNT: mean duration in each serial window of COUNT dispatches")
    s.add_argument("--out")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out")
    tl = sub.add_parser("timeline")
    tl.add_argument("trace_csv")
    tl.add_argument("--kernel", action="append", required=True, help="kernel name as in the stats (repeatable)")
    tl.add_argument("--first", type=int, default=0)
    tl.add_argument("--count", type=int, default=30)
    tl.add_argument("--cmd", required=True)
    tl.add_argument("--out")
    f = sub.add_parser("flops")
    f.add_argument("csv64")
    f.add_argument("csv32")
    f.add_argument("--cmd64", required=True)
    f.add_argument("--cmd32", required=True)
    f.add_argument("--out")
    a = ap.parse_args(argv)
    if a.what == "stats":
        text = stats_summary(a.csv, a.cmd, a.trace, a.timer)
    elif a.what == "timeline":
        text = timeline_summary(a.trace_csv, a.kernel, a.cmd, a.first, a.count)
    elif a.what == "flops":
        text = flops_summary(a.csv64, a.csv32, a.cmd64, a.cmd32)
    else:
        text = traffic_summary(a.fetch_csv, a.write_csv, a.copy_bytes, a.cmd_fetch, a.cmd_write)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
