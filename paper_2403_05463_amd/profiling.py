"""Summaries of rocprofv3 output for the kernels of this library.

``python -m paper_2403_05463_amd.profiling stats <kernel_stats.csv> --cmd "<command>"``
    per-kernel call count and mean duration from ``--kernel-trace --stats``;
``python -m paper_2403_05463_amd.profiling traffic <fetch.csv> <write.csv> --copy-bytes B --cmd "<command>"``
    HBM bytes per dispatch from two ``--pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE``
    runs, each scaled by what the same counter reads for the plain copy kernel
    of known size (copy bytes / counter reading).

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


def stats_summary(path: str, cmd: str) -> str:
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 kernel statistics", f"command: {cmd}", f"kernel source hash: {kernel_source_hash()}", "",
             f"{'kernel':40s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'share':>7s}"]
    for r in rows:
        lines.append(f"{short_name(r['Name']):40s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:10.2f} "
                     f"{float(r['MinNs']) / 1e3:10.2f} {float(r['MaxNs']) / 1e3:10.2f} {float(r['Percentage']):6.2f}%")
    return "\n".join(lines) + "\n"


def _per_kernel(path: str, counter: str) -> dict:
    acc = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            acc[short_name(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic_summary(fetch_csv: str, write_csv: str, copy_bytes: int, cmd_fetch: str, cmd_write: str) -> str:
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    copy = next(k for k in fetch if k.startswith("k_copy"))
    f_fetch = copy_bytes / (fetch[copy] * 1024.0)
    f_write = copy_bytes / (write[copy] * 1024.0)
    lines = ["# HBM traffic per dispatch from FETCH_SIZE and WRITE_SIZE (KiB per dispatch)",
             f"command (fetch): {cmd_fetch}", f"command (write): {cmd_write}",
             f"kernel source hash: {kernel_source_hash()}",
             f"calibration: plain copy of {copy_bytes} bytes reads FETCH_SIZE {fetch[copy]:.1f} KiB "
             f"and WRITE_SIZE {write[copy]:.1f} KiB; factors fetch {f_fetch:.4f}, write {f_write:.4f}", "",
             f"{'kernel':40s} {'FETCH_KiB':>12s} {'WRITE_KiB':>12s} {'traffic_bytes':>16s}"]
    for k in sorted(fetch):
        if k not in write:
            continue
        t = fetch[k] * 1024.0 * f_fetch + write[k] * 1024.0 * f_write
        lines.append(f"{k.replace(' ', ''):40s} {fetch[k]:12.1f} {write[k]:12.1f} {t:16.0f}")
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
        if len(parts) == 4 and parts[0].startswith(want):
            try:
                return float(parts[3])
            except ValueError:
                return None
    return None


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="what", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", required=True)
    s.add_argument("--out")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-bytes", type=int, required=True)
    t.add_argument("--cmd-fetch", required=True)
    t.add_argument("--cmd-write", required=True)
    t.add_argument("--out")
    a = ap.parse_args(argv)
    if a.what == "stats":
        text = stats_summary(a.csv, a.cmd)
    else:
        text = traffic_summary(a.fetch_csv, a.write_csv, a.copy_bytes, a.cmd_fetch, a.cmd_write)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)
    print(text)


if __name__ == "__main__":
    main()
