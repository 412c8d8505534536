"""Summaries of rocprofv3 output for the step's kernels (text for profiles/).

    python -m paper_1005_2594_amd.rocprof_summary trace <kernel_trace.csv> <out.md> <title>
    python -m paper_1005_2594_amd.rocprof_summary traffic <fetch_counter.csv> <write_counter.csv> <out.txt> <title>
    python -m paper_1005_2594_amd.rocprof_summary sizes <rdreq_counter.csv> <out.md> <title>

trace: per kernel, calls and the average, minimum, maximum and median
duration of its dispatches.
traffic: per kernel, the median FETCH_SIZE and WRITE_SIZE per dispatch and
the dispatches per step (dispatches relative to the LB kernel's, one per
step; kernels of the set-up only round to none and are left out); the counters (KiB of traffic between L2 and the fabric) are turned
into bytes with the factor a plain device copy of 2^31 bytes gives in the
same run (the largest copy dispatches); the per-step sums over all kernels,
and the hash of the library's HIP sources they belong to.
sizes: per kernel, the read requests split by size (32, 64, 128 bytes) and
the exact read bytes they make.
"""
from __future__ import annotations

import csv
import hashlib
import os
import statistics
import sys
from collections import defaultdict

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
COPY_BYTES = 1 << 31


def csrc_sha256() -> str:
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            h.update(open(os.path.join(CSRC, name), "rb").read())
    return h.hexdigest()


def short(name: str) -> str:
    return name if len(name) <= 70 else name[:67] + "..."


def trace(path, out, title):
    dur = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            dur[row["Kernel_Name"]].append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in dur.values())
    lines = [f"# {title}", "", "| kernel | calls | average us | min us | max us | median us | % of GPU time |",
             "|---|---|---|---|---|---|---|"]
    for k, v in sorted(dur.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{short(k)}` | {len(v)} | {statistics.mean(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                     f"{statistics.median(v):.1f} | {100 * sum(v) / total:.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")


def _counters(path, counter):
    per = defaultdict(list)
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Counter_Name"] == counter:
                per[row["Kernel_Name"]].append(float(row["Counter_Value"]))
    return per


def traffic(fetch_csv, write_csv, out, title):
    fe = _counters(fetch_csv, "FETCH_SIZE")
    wr = _counters(write_csv, "WRITE_SIZE")
    copies = [k for k in fe if "copyBuffer" in k]
    cf = sorted(v for k in copies for v in fe[k])[-4:]
    cw = sorted(v for k in copies for v in wr.get(k, []))[-4:]
    f_scale = COPY_BYTES / (statistics.median(cf) * 1024.0)
    w_scale = COPY_BYTES / (statistics.median(cw) * 1024.0)
    lb = [k for k in fe if "lb_kernel" in k]
    if len(lb) != 1:
        # per-step figures assume one workload: one LB variant, one launch a step
        sys.exit(f"expected one LB kernel in the counter run, found {len(lb)}: {lb}")
    steps = len(fe[lb[0]])
    lines = [f"# {title}", "#",
             "# kernel | dispatches | per step | median fetch KiB | median write KiB | fetch MB per step | write MB per step"]
    tf = tw = 0.0
    for k in sorted(fe, key=lambda k: -statistics.median(fe[k]) * len(fe[k])):
        if "copyBuffer" in k or "FillFunc" in k or "fillBuffer" in k:
            continue
        n = len(fe[k])
        per_step = round(n / steps)  # set-up kernels (a few dispatches in all) round to 0
        if per_step == 0:
            continue
        mf = statistics.median(fe[k])
        mw = statistics.median(wr.get(k, [0.0]))
        bf, bw = per_step * mf * 1024.0 * f_scale, per_step * mw * 1024.0 * w_scale
        tf += bf
        tw += bw
        lines.append(f"# {short(k)} | {n} | {per_step} | {mf:.0f} | {mw:.0f} | {bf / 1e6:.1f} | {bw / 1e6:.1f}")
    k = lb[0]  # the fused LB kernel alone, per launch (the roofline's kernel)
    lines += [f"lb_kernel: {k}",
              f"lb_fetch_bytes_per_launch: {statistics.median(fe[k]) * 1024.0 * f_scale:.0f}",
              f"lb_write_bytes_per_launch: {statistics.median(wr[k]) * 1024.0 * w_scale:.0f}"]
    lines += ["#", f"copy_bytes: {COPY_BYTES}",
              f"copy_fetch_kib_per_launch: {statistics.median(cf):.0f}",
              f"copy_write_kib_per_launch: {statistics.median(cw):.0f}",
              f"fetch_scale_bytes_per_counted_byte: {f_scale:.3f}",
              f"write_scale_bytes_per_counted_byte: {w_scale:.3f}",
              f"steps_counted: {steps}",
              f"step_fetch_bytes: {tf:.0f}", f"step_write_bytes: {tw:.0f}",
              f"csrc_sha256: {csrc_sha256()}"]
    open(out, "w").write("\n".join(lines) + "\n")


def sizes(csv_path, out, title):
    """Read bytes per kernel from the request-size counters (TCC_EA0_RDREQ
    split into 32-, 64- and 128-byte requests): exact bytes with no scaling,
    a check of the copy-scaled FETCH_SIZE (which counts a 128-byte request
    as 64 bytes on this device)."""
    per = defaultdict(lambda: defaultdict(list))
    with open(csv_path) as f:
        for row in csv.DictReader(f):
            per[row["Kernel_Name"]][row["Counter_Name"]].append(float(row["Counter_Value"]))
    names = ("TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum")
    lines = [f"# {title}", "",
             "| kernel | dispatches | median requests | 128 B | 64 B | 32 B | read MB (exact) | share of 128 B requests |",
             "|---|---|---|---|---|---|---|---|"]
    rows = []
    for k, c in per.items():
        if not all(n in c for n in names):
            continue
        if "copyBuffer" in k:  # the calibration copies only (the largest dispatches)
            idx = sorted(range(len(c[names[0]])), key=lambda i: c[names[0]][i])[-4:]
            med = {n: statistics.median(c[n][i] for i in idx) for n in names}
        else:
            med = {n: statistics.median(c[n]) for n in names}
        byts = 32 * med[names[1]] + 64 * med[names[2]] + 128 * med[names[3]]
        rows.append((byts, k, len(c[names[0]]), med))
    for byts, k, n, med in sorted(rows, reverse=True)[:16]:
        tot = max(med[names[0]], 1.0)
        lines.append(f"| `{short(k)}` | {n} | {med[names[0]]:.0f} | {med[names[3]]:.0f} | {med[names[2]]:.0f} | "
                     f"{med[names[1]]:.0f} | {byts / 1e6:.1f} | {med[names[3]] / tot:.4f} |")
    open(out, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "trace":
        trace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5])
    elif sys.argv[1] == "sizes":
        sizes(sys.argv[2], sys.argv[3], sys.argv[4])
    else:
        raise SystemExit(__doc__)
