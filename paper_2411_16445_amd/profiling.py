"""Summaries of rocprofv3 output for the fused epoch kernel.

Two uses:

* ``python -m paper_2411_16445_amd.profiling counters FETCH_DIR WRITE_DIR
  --kernel k_epoch --copy-mib 256 --steps-per-dispatch N --workload W
  [--last L] --command "..." > profiles/<name>.md``
  turns two ``rocprofv3 --pmc FETCH_SIZE`` / ``--pmc WRITE_SIZE`` runs of
  ``bench.py --copy-probe-mib 256`` into the HBM traffic per launch of the
  kernel.  Both counters are in KiB per dispatch; each is scaled by what it
  reads for the plain device copy of known size that the same run performs
  (the copy moves exactly ``copy-mib`` MiB each way), so the figure is in
  true bytes.
* ``python -m paper_2411_16445_amd.profiling trace STATS_CSV --command "..."
  [--kernel K --last L]`` formats a ``--kernel-trace --stats``
  kernel_stats.csv as a table, with the mean duration of the kernel's last L
  dispatches (a bench run's timed launches) from the kernel_trace.csv beside
  it.

``traffic_for_bench`` reads a counters summary back for ``bench.py``; it
returns None when the kernel sources changed since the counters were taken
(the summary records a fingerprint of them).
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import os
import re
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/kernels_fused.hip", "csrc/device_common.hpp", "csrc/sim.hpp")


def source_fingerprint() -> str:
    """sha256 over the sources the fused kernel is compiled from."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(_HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _rows(d: str):
    path = d if d.endswith(".csv") else None
    if path is None:
        for root, _, files in os.walk(d):
            for fn in files:
                if fn.endswith("counter_collection.csv"):
                    path = os.path.join(root, fn)
    if path is None:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    with open(path) as f:
        return list(csv.DictReader(f))


def _per_dispatch(rows, counter, pick):
    """Counter value per dispatch of the kernels selected by pick(row), in
    dispatch order."""
    out = {}
    for r in rows:
        if r["Counter_Name"] != counter or not pick(r):
            continue
        key = int(r["Dispatch_Id"])
        out[key] = out.get(key, 0.0) + float(r["Counter_Value"])
    return [out[k] for k in sorted(out)]


def counters_summary(fetch_dir, write_dir, kernel, copy_mib, command, steps_per_dispatch, workload, last=0):
    """last > 0: only the kernel's last `last` dispatches count (a bench
    run's timed launches come after its plan trials, settling and warm-up),
    and steps_per_dispatch is their mean step count."""
    copy_bytes = copy_mib * 1024 * 1024
    lines = []
    res = {}
    for name, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = _rows(d)
        kern = _per_dispatch(rows, name, lambda r: kernel in r["Kernel_Name"])
        if last > 0:
            kern = kern[-last:]
        # the copy probe: the largest device-to-device copies after the
        # kernel's last dispatch (earlier copies of the same grid size, such
        # as the network's upload, move other amounts)
        last_k = max((int(r["Dispatch_Id"]) for r in rows if kernel in r["Kernel_Name"]), default=-1)
        copies = [r for r in rows if r["Counter_Name"] == name and "copyBuffer" in r["Kernel_Name"]
                  and int(r["Dispatch_Id"]) > last_k]
        if not kern or not copies:
            raise SystemExit(f"{name}: no dispatches of {kernel} or of the copy probe after them in {d}")
        big = max(int(r["Grid_Size"]) for r in copies)
        cp = [float(r["Counter_Value"]) for r in copies if int(r["Grid_Size"]) == big]
        cp_kib = sum(cp) / len(cp)
        factor = copy_bytes / (cp_kib * 1024.0)
        k_kib = sum(kern) / len(kern)
        res[name] = dict(kib=k_kib, n=len(kern), copy_kib=cp_kib, factor=factor,
                         bytes=k_kib * 1024.0 * factor)
    fp = source_fingerprint()
    lines.append(f"# HBM traffic of `{kernel}` per launch (rocprofv3 counters)")
    lines.append("")
    lines.append("Commands (repository root on the MI355X box, one counter per run):")
    lines.append("")
    for c in command:
        lines.append(f"    {c}")
    lines.append("")
    lines.append(f"The same run then copies {copy_mib} MiB device to device (a plain copy kernel); the")
    lines.append("factor scales each counter so that it reads that copy's true size.")
    lines.append("")
    lines.append("| counter | dispatches | KiB per dispatch | copy probe KiB | scale factor | bytes per launch |")
    lines.append("|---|---|---|---|---|---|")
    for name in ("FETCH_SIZE", "WRITE_SIZE"):
        r = res[name]
        lines.append(f"| {name} | {r['n']} | {r['kib']:.1f} | {r['copy_kib']:.1f} | {r['factor']:.3f} | "
                     f"{r['bytes']:.0f} |")
    total = res["FETCH_SIZE"]["bytes"] + res["WRITE_SIZE"]["bytes"]
    lines.append("")
    if last > 0:
        lines.append(f"Only the kernel's last {last} dispatches (the timed launches) count; they advance "
                     f"{steps_per_dispatch} steps each on average.")
    else:
        lines.append(f"Each dispatch advances {steps_per_dispatch} steps.")
    lines.append("")
    lines.append(f"traffic_bytes_per_launch: {total:.0f}")
    lines.append(f"traffic_bytes_per_step: {total / steps_per_dispatch:.1f}")
    lines.append(f"kernel: {kernel}")
    lines.append(f"workload: {workload}")
    lines.append(f"source_sha256: {fp}")
    return "\n".join(lines) + "\n"


def timed_launches(trace_csv, kernel, last):
    """Durations (us) of the last `last` dispatches of the kernel whose name
    contains `kernel`, from a --kernel-trace kernel_trace.csv."""
    with open(trace_csv) as f:
        rows = [r for r in csv.DictReader(f) if kernel in r["Kernel_Name"]]
    rows.sort(key=lambda r: int(r["Dispatch_Id"]))
    return [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in rows[-last:]]


def trace_summary(stats_csv, command, title, kernel=None, last=0):
    with open(stats_csv) as f:
        rows = list(csv.DictReader(f))
    lines = [f"# Kernel trace: {title}", "", "Command (repository root on the MI355X box):", ""]
    for c in command:
        lines.append(f"    {c}")
    lines += ["", "Durations in microseconds (rocprofv3 kernel_stats.csv).", "",
              "| kernel | calls | total us | average us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows:
        name = r.get("Name", "")
        calls = int(r.get("Calls", 0))
        tot = float(r.get("TotalDurationNs", 0)) / 1e3
        avg = float(r.get("AverageNs", 0)) / 1e3
        mn = float(r.get("MinNs", 0)) / 1e3
        mx = float(r.get("MaxNs", 0)) / 1e3
        pct = float(r.get("Percentage", 0))
        lines.append(f"| {name} | {calls} | {tot:.1f} | {avg:.3f} | {mn:.3f} | {mx:.3f} | {pct:.2f} |")
    if kernel and last > 0:
        trace_csv = os.path.join(os.path.dirname(stats_csv), os.path.basename(stats_csv).replace(
            "kernel_stats", "kernel_trace"))
        dur = timed_launches(trace_csv, kernel, last)
        lines += ["", f"Timed launches (the last {len(dur)} dispatches of `{kernel}`): "
                      + ", ".join(f"{x:.1f}" for x in dur) + f" us; mean {sum(dur) / len(dur):.1f} us.",
                  "", f"timed_launch_mean_us: {sum(dur) / len(dur):.3f}"]
    return "\n".join(lines) + "\n"


def traffic_for_bench(profiles_dir, kernel, workload):
    """(HBM bytes per step, summary file) from a counters summary of this
    kernel and workload whose source fingerprint equals the present
    sources, else (None, reason)."""
    if not os.path.isdir(profiles_dir):
        return None, "no profiles directory"
    fp = source_fingerprint()
    stale = None
    for fn in sorted(os.listdir(profiles_dir)):
        if not fn.startswith("counters_") or not fn.endswith(".md"):
            continue
        with open(os.path.join(profiles_dir, fn)) as f:
            text = f.read()
        m_k = re.search(r"^kernel: (.+)$", text, re.M)
        m_t = re.search(r"^traffic_bytes_per_step: ([0-9.]+)$", text, re.M)
        m_s = re.search(r"^source_sha256: ([0-9a-f]+)$", text, re.M)
        m_w = re.search(r"^workload: (.+)$", text, re.M)
        if not (m_k and m_t and m_s and m_w) or m_k.group(1).strip() not in kernel:
            continue
        if m_w.group(1).strip() != workload:
            continue
        if m_s.group(1) != fp:
            stale = fn
            continue
        return float(m_t.group(1)), fn
    return None, (f"{stale}: kernel sources changed since the counters were taken" if stale
                  else "no counters summary for this kernel")


def main(argv=None):
    ap = argparse.ArgumentParser(prog="python -m paper_2411_16445_amd.profiling")
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--kernel", default="k_epoch")
    c.add_argument("--copy-mib", type=int, default=256)
    c.add_argument("--steps-per-dispatch", type=float, required=True)
    c.add_argument("--workload", required=True)
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--last", type=int, default=0, help="count only the kernel's last N dispatches")
    t = sub.add_parser("trace")
    t.add_argument("stats_csv")
    t.add_argument("--title", default="")
    t.add_argument("--command", action="append", default=[])
    t.add_argument("--kernel", default=None)
    t.add_argument("--last", type=int, default=0, help="report the mean of the kernel's last N dispatches")
    sub.add_parser("fingerprint")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        sys.stdout.write(counters_summary(a.fetch_dir, a.write_dir, a.kernel, a.copy_mib, a.command,
                                          a.steps_per_dispatch, a.workload, a.last))
    elif a.cmd == "trace":
        sys.stdout.write(trace_summary(a.stats_csv, a.command, a.title, a.kernel, a.last))
    else:
        print(source_fingerprint())


if __name__ == "__main__":
    main()
