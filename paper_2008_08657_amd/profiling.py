"""Summaries of rocprofv3 output for the benchmark's kernels.

``summarize``: a Markdown table of the kernel-trace statistics
(``*_kernel_stats.csv``) with the command that produced them; with
``--dispatches`` and ``--last N``, also the mean duration of the last N
launches of each named kernel (the launches of ``bench.py``'s timed region,
after the prepare, warm-up and checked runs), read from the per-dispatch
trace (``*_kernel_trace.csv``).

``traffic``: HBM bytes per launch of one kernel from two counter runs
(``FETCH_SIZE`` and ``WRITE_SIZE``, KiB per dispatch), each scaled by what the
same counter reads for a plain device copy of known size.  The record names
the kernel and a digest of its generated source and launch grid;
``bench.py`` reports the bytes only while the kernel it measures has that
same source and grid.

``counters``: per-dispatch means of SQ counters of one kernel (instruction
mix, waves, waits) as a Markdown table.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import sys


def source_digest(text: str) -> str:
    return hashlib.sha1(text.encode()).hexdigest()[:16]


def builtin_source() -> str:
    """The text of the library's built-in kernels (a traffic record of a
    built-in kernel is valid while this text is unchanged)."""
    import os
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "csrc", "kernels.hip")) as f:
        return f.read()


def step_digest(source: str, step: str, grid: int) -> str:
    """Digest of a built-in kernel's step as bench.py computes it."""
    return source_digest(source + f"\n// step {step}" + f"\n// grid {grid}")


def _counter_rows(path, counter):
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter:
                yield row["Kernel_Name"], float(row["Counter_Value"])


def mean_counter(path, counter, kernel, skip=0):
    vals = [v for k, v in _counter_rows(path, counter) if k == kernel][skip:]
    if not vals:
        raise SystemExit(f"{path}: no {counter} rows for kernel {kernel}")
    return sum(vals) / len(vals), len(vals)


def copy_counter(path, counter):
    """The counter of the largest copy dispatch (the 1 GiB calibration copy)."""
    vals = [v for k, v in _counter_rows(path, counter) if "copyBuffer" in k]
    if not vals:
        raise SystemExit(f"{path}: no copy dispatch")
    return max(vals)


def traffic(a):
    f_kib, nf = mean_counter(a.fetch, "FETCH_SIZE", a.kernel, a.skip)
    w_kib, nw = mean_counter(a.write, "WRITE_SIZE", a.kernel, a.skip)
    cf = copy_counter(a.copy_fetch, "FETCH_SIZE")
    cw = copy_counter(a.copy_write, "WRITE_SIZE")
    f_scale = a.copy_bytes / (cf * 1024.0)
    w_scale = a.copy_bytes / (cw * 1024.0)
    rec = {"workload": a.workload, "kernel": a.kernel, "step": a.step, "source_digest": a.source_digest,
           "fetch_kib": f_kib, "write_kib": w_kib, "dispatches": [nf, nw], "skipped_first": a.skip,
           "copy_bytes": a.copy_bytes, "copy_fetch_kib": cf, "copy_write_kib": cw,
           "fetch_scale": f_scale, "write_scale": w_scale,
           "bytes_read": f_kib * 1024.0 * f_scale, "bytes_written": w_kib * 1024.0 * w_scale,
           "commands": a.command}
    rec["bytes"] = rec["bytes_read"] + rec["bytes_written"]
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def counters(a):
    sums, n = {}, {}
    with open(a.csv, newline="") as f:
        for row in csv.DictReader(f):
            if row["Kernel_Name"] != a.kernel:
                continue
            k = row["Counter_Name"]
            sums[k] = sums.get(k, 0.0) + float(row["Counter_Value"])
            n[k] = n.get(k, 0) + 1
    lines = [f"# {a.title}", "", "Command:", "", "```", *a.command, "```", "",
             "| counter | mean per dispatch |", "|---|---:|"]
    for k in sorted(sums):
        lines.append(f"| {k} | {sums[k] / n[k]:.0f} |")
    if a.note:
        lines += ["", *a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def summarize(a):
    rows = []
    with open(a.trace, newline="") as f:
        for r in csv.DictReader(f):
            rows.append(r)
    lines = [f"# {a.title}", "", "Command:", "", "```", *a.command, "```", "",
             "| kernel | calls | total ms | average us | % |", "|---|---:|---:|---:|---:|"]
    for r in rows[:a.top]:
        name = r["Name"] if len(r["Name"]) < 90 else r["Name"][:87] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    if a.dispatches and a.last > 0 and a.kernel:
        lines += ["", f"Last {a.last} launches of each kernel below (the timed steps), from the per-dispatch trace:",
                  "", "| kernel | launches | average us | min us | max us |", "|---|---:|---:|---:|---:|"]
        for k in a.kernel:
            d = last_launches(a.dispatches, k, a.last)
            if d:
                lines.append(f"| `{k}` | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")
    if a.note:
        lines += ["", *a.note]
    with open(a.out, "w") as f:
        f.write("\n".join(lines) + "\n")


def last_launches(path, kernel, n):
    """Durations (us) of the last n launches of the kernel whose name starts
    with ``kernel``, in dispatch order."""
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            if r["Kernel_Name"].startswith(kernel):
                rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    rows.sort()
    return [(e - s) / 1e3 for s, e in rows[-n:]]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "out", "workload", "step"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--source-digest", required=True)
    t.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    # dispatches left out at the start (a first run into a table that is
    # regrown afterwards has a different size from the timed runs')
    t.add_argument("--skip", type=int, default=0)
    t.add_argument("--command", action="append", default=[])
    s = sub.add_parser("summarize")
    s.add_argument("--trace", required=True)
    s.add_argument("--out", required=True)
    s.add_argument("--title", required=True)
    s.add_argument("--top", type=int, default=25)
    s.add_argument("--dispatches", default=None)
    s.add_argument("--last", type=int, default=0)
    s.add_argument("--kernel", action="append", default=[])
    s.add_argument("--command", action="append", default=[])
    s.add_argument("--note", action="append", default=[])
    c = sub.add_parser("counters")
    c.add_argument("--csv", required=True)
    c.add_argument("--kernel", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--title", required=True)
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--note", action="append", default=[])
    a = ap.parse_args(argv)
    {"traffic": traffic, "summarize": summarize, "counters": counters}[a.cmd](a)
    return 0


if __name__ == "__main__":
    sys.exit(main())
