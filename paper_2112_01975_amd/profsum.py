"""Summaries of rocprofv3 output for the committed profile records.

  python -m paper_2112_01975_amd.profsum stats <kernel_stats.csv> <command...>
  python -m paper_2112_01975_amd.profsum traffic <fetch_counter_collection.csv> <write_counter_collection.csv> \
         <kernel-substring> <copy-bytes> <command...>
  python -m paper_2112_01975_amd.profsum counters <kernel-substring> <compute-units> <xcds> <csv>... -- <command...>
  python -m paper_2112_01975_amd.profsum stepfetch <fetch_counter_collection.csv> <kernel-substring> <copy-bytes> \
         <steps> <algorithmic-read-bytes-per-step> <label>

`stats` turns a --kernel-trace --stats summary into a short text table. `traffic`
reads two --pmc runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch), scales each
counter by what it reads for the plain device copy of known size in the same run
(the bench's copy probe, lbm_copy_probe), and prints HBM bytes per launch of the named kernel,
together with a fingerprint of the kernel sources so that a later run can tell
whether the counters still describe the current kernel.
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# the translation unit of k_fused3, the kernel the traffic counters describe
KERNEL_SOURCES = ["csrc/fused_kernels.hip", "csrc/step_common.hpp", "csrc/lattice.hpp", "csrc/kernels.hpp",
                  "csrc/fused.hpp"]


def source_fingerprint() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def short_name(name: str) -> str:
    m = re.search(r"(k_\w+|copyBuffer\w*|\w+Kernel\w*)", name)
    base = m.group(1) if m else name[:40]
    t = re.search(r"<([^()]*)>", name)
    return f"{base}<{t.group(1)}>" if t and base.startswith("k_") else base


def stats(path: str, command: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = [f"# rocprofv3 --kernel-trace --stats", f"# command: {command}", "",
           f"{'kernel':60s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'total_%':>8s}"]
    for r in rows:
        name = short_name(r["Name"])
        calls = int(r["Calls"])
        avg = float(r["AverageNs"]) / 1e3
        mn = float(r["MinNs"]) / 1e3
        mx = float(r["MaxNs"]) / 1e3
        pct = float(r["Percentage"])
        out.append(f"{name:60s} {calls:6d} {avg:10.2f} {mn:10.2f} {mx:10.2f} {pct:8.2f}")
    return "\n".join(out) + "\n"


def _per_kernel(path: str):
    acc = {}
    for r in csv.DictReader(open(path)):
        acc.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return acc


def traffic(fetch_csv: str, write_csv: str, kernel: str, copy_bytes: int, command: str) -> str:
    f = _per_kernel(fetch_csv)
    w = _per_kernel(write_csv)

    def pick(d, key):
        vals = [v for name, vs in d.items() if key in name for v in vs]
        if not vals:
            raise SystemExit(f"no dispatch matching {key!r}")
        return vals

    # copy probe (lbm_copy_probe's k_copy): its dispatches move copy_bytes each way
    cf = max(pick(f, "k_copy")) * 1024.0
    cw = max(pick(w, "k_copy")) * 1024.0
    fetch_scale = copy_bytes / cf
    write_scale = copy_bytes / cw
    kf = pick(f, kernel)
    kw = pick(w, kernel)
    fb = sum(kf) / len(kf) * 1024.0 * fetch_scale
    wb = sum(kw) / len(kw) * 1024.0 * write_scale
    lines = [
        "# HBM traffic per launch from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE)",
        f"# command: {command}",
        f"kernel: {kernel}",
    ]
    if "k_fused3" in kernel:   # the fingerprint describes k_fused3's sources only
        lines.append(f"source_fingerprint: {source_fingerprint()}")
    lines += [
        f"dispatches_fetch: {len(kf)}",
        f"dispatches_write: {len(kw)}",
        f"copy_probe_bytes: {copy_bytes}",
        f"fetch_scale: {fetch_scale:.4f}",
        f"write_scale: {write_scale:.4f}",
        f"fetch_bytes_per_launch: {fb:.0f}",
        f"write_bytes_per_launch: {wb:.0f}",
        f"traffic_bytes_per_launch: {fb + wb:.0f}",
    ]
    return "\n".join(lines) + "\n"


def counters(kernel: str, cus: int, xccs: int, paths: list, command: str) -> str:
    """Mean per dispatch of every counter in the --pmc runs' counter_collection.csv files for
    the named kernel, and busy fractions: a sum over CUs (`_sum`, SQ_ACTIVE_INST_VALU,
    SQ_BUSY_CU_CYCLES) divided by the CU count, or an average over instances (`_avr`), over
    the active cycles of one XCD (GRBM_GUI_ACTIVE, which each pass collects, summed over the
    `xccs` XCDs in the output)."""
    lines = ["# rocprofv3 --pmc counters per dispatch (mean over the kernel's dispatches)",
             f"# command: {command}", f"kernel: {kernel}", f"compute_units: {cus}", f"xcds: {xccs}"]
    for path in paths:
        acc = {}
        for r in csv.DictReader(open(path)):
            if kernel in r["Kernel_Name"]:
                acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        if not acc:
            raise SystemExit(f"no dispatch of {kernel!r} in {path}")
        mean = {k: sum(v) / len(v) for k, v in acc.items()}
        gui = mean.get("GRBM_GUI_ACTIVE")
        if gui:
            gui /= xccs   # active cycles of one XCD
        lines.append(f"## pass {os.path.basename(os.path.dirname(path)) or path} ({len(next(iter(acc.values())))} dispatches)")
        for k in sorted(mean):
            lines.append(f"{k}: {mean[k]:.6g}")
            if gui and k != "GRBM_GUI_ACTIVE":
                per_cu = k.endswith("_sum") or k in ("SQ_ACTIVE_INST_VALU", "SQ_BUSY_CU_CYCLES")
                frac = mean[k] / (cus * gui) if per_cu else (mean[k] / gui if k.endswith("_avr") else None)
                if frac is not None:
                    lines.append(f"{k}_frac_of_active_cycles: {frac:.4f}")
    return "\n".join(lines) + "\n"


def step_fetch(path: str, kernel: str, copy_bytes: int, steps: int, algorithmic: float, label: str) -> str:
    """One FETCH_SIZE run of a size leg: the named kernel's fetched bytes summed over its
    dispatches and divided by the steps the run took (a step may be several launches), scaled
    by the copy probe's reading in the same run, against the algorithmic read bytes per step."""
    rows = list(csv.DictReader(open(path)))
    kern = [float(r["Counter_Value"]) for r in rows if kernel in r["Kernel_Name"]]
    copy = [float(r["Counter_Value"]) for r in rows if "k_copy" in r["Kernel_Name"]]
    if not kern or not copy:
        raise SystemExit(f"no dispatches of {kernel!r} or of the copy probe in {path}")
    scale = copy_bytes / (max(copy) * 1024.0)
    per_step = sum(kern) * 1024.0 * scale / steps
    return (f"{label:14s} {len(kern) / steps:13.1f} {per_step:21.0f} {per_step / algorithmic:18.3f}\n")


def read_traffic(path: str) -> dict:
    d = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":", 1)
            d[k.strip()] = v.strip()
    return d


if __name__ == "__main__":
    if len(sys.argv) < 2:
        raise SystemExit(__doc__)
    if sys.argv[1] == "stats":
        sys.stdout.write(stats(sys.argv[2], " ".join(sys.argv[3:])))
    elif sys.argv[1] == "counters":
        # counters <kernel-substring> <compute-units> <xcds> <csv> [<csv> ...] -- <command...>
        i = sys.argv.index("--")
        sys.stdout.write(counters(sys.argv[2], int(sys.argv[3]), int(sys.argv[4]), sys.argv[5:i],
                                  " ".join(sys.argv[i + 1:])))
    elif sys.argv[1] == "stepfetch":
        # stepfetch <counter_collection.csv> <kernel-substring> <copy-bytes> <steps> <algorithmic-bytes> <label>
        sys.stdout.write(step_fetch(sys.argv[2], sys.argv[3], int(sys.argv[4]), int(sys.argv[5]), float(sys.argv[6]),
                                    sys.argv[7]))
    elif sys.argv[1] == "traffic":
        sys.stdout.write(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5]), " ".join(sys.argv[6:])))
    else:
        raise SystemExit(__doc__)
