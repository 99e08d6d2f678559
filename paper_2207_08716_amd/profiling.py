"""Summaries of rocprofv3 output for the profiles/ folder.

  python -m paper_2207_08716_amd.profiling trace <kernel_stats.csv> <out.md> <command...>
  python -m paper_2207_08716_amd.profiling traffic <fetch_counter_collection.csv>
        <write_counter_collection.csv> <n> <out.json> <out.md> <command...>
  python -m paper_2207_08716_amd.profiling traffic-waves <fetch_counter_collection.csv>
        <write_counter_collection.csv> <nx> <ny> <nz> <out.json> <out.md> <command...>

The first form covers the two-phase thesis sweep on an n^3 grid (A_eff =
25 N 8 bytes), the second the reactive porosity-wave sweep on nx x ny x nz
cells (4 iterated fields read and written and 3 old-step fields read:
11 N 8 bytes).

FETCH_SIZE and WRITE_SIZE are read in KiB per dispatch and calibrated with the
streaming copy kernel of known size that the benchmark runs in the same
process: factor = copied bytes / counter bytes for that kernel.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2207_08716_amd", "csrc", "iter_kernel.hip")
DOMINANT = "k_sweep<double, 0, false"   # thesis sweep without norms
COPY = "k_copy"


def short(name: str) -> str:
    n = name.replace("ptk::(anonymous namespace)::", "").replace("void ", "")
    return n.split("(")[0]


def trace_summary(stats_csv: str, out_md: str, command: str) -> None:
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# rocprofv3 kernel trace summary", "", f"Command: `{command}`", "",
             "| kernel | calls | average (us) | min (us) | max (us) | share (%) |",
             "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(path):
    acc = defaultdict(list)
    for r in csv.DictReader(open(path)):
        acc[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def traffic_summary(fetch_csv, write_csv, n, out_json, out_md, command, copy_elems=None,
                    dominant=DOMINANT, a_eff=None, kernel_src=KERNEL_SRC, grid=None):
    fetch = _per_kernel(fetch_csv)
    write = _per_kernel(write_csv)
    copy_key = next(k for k in fetch if COPY in k)
    dom_key = next(k for k in fetch if dominant in k)
    # the benchmark copies one padded field box: (n+1)^2 * pitch doubles
    pitch = ((n + 1 + 31) // 32) * 32
    copy_bytes = (copy_elems or (n + 1) * (n + 1) * pitch) * 8
    f_fac = copy_bytes / (fetch[copy_key] * 1024.0)
    w_fac = copy_bytes / (write[copy_key] * 1024.0)
    fb = fetch[dom_key] * 1024.0 * f_fac
    wb = write[dom_key] * 1024.0 * w_fac
    a_eff = 25.0 * n ** 3 * 8 if a_eff is None else float(a_eff)
    sha = hashlib.sha256(open(kernel_src, "rb").read()).hexdigest()[:16]
    rec = {"n": n, "grid": grid or f"{n}^3", "kernel": dom_key, "kernel_source_sha": sha,
           "fetch_bytes": fb, "write_bytes": wb, "bytes_per_launch": fb + wb,
           "fetch_factor": f_fac, "write_factor": w_fac, "a_eff_bytes": a_eff,
           "command": command}
    json.dump(rec, open(out_json, "w"), indent=1)
    lines = ["# HBM traffic from rocprofv3 counters", "", f"Command: `{command}`", "",
             f"Calibration: the streaming copy of {copy_bytes / 1e9:.3f} GB reads FETCH_SIZE = "
             f"{fetch[copy_key]:.0f} KiB and WRITE_SIZE = {write[copy_key]:.0f} KiB per dispatch; "
             f"factors {f_fac:.4f} (fetch) and {w_fac:.4f} (write).", "",
             "| kernel | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) | calibrated read (GB) | calibrated write (GB) |",
             "|---|---|---|---|---|"]
    for k in sorted(fetch, key=lambda x: -fetch[x]):
        if k in write:
            lines.append(f"| {k} | {fetch[k]:.0f} | {write[k]:.0f} | {fetch[k] * 1024 * f_fac / 1e9:.3f} | "
                         f"{write[k] * 1024 * w_fac / 1e9:.3f} |")
    lines += ["", f"Dominant kernel {dom_key}: {(fb + wb) / 1e9:.3f} GB per launch against "
              f"{a_eff / 1e9:.3f} GB of algorithmic bytes (ratio {(fb + wb) / a_eff:.3f}); "
              f"kernel source sha {sha}."]
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "trace":
        trace_summary(sys.argv[2], sys.argv[3], " ".join(sys.argv[4:]))
    elif what == "traffic":
        traffic_summary(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6],
                        " ".join(sys.argv[7:]))
    elif what == "traffic-waves":
        nx, ny, nz = (int(v) for v in sys.argv[4:7])
        pitch = ((nx + 1 + 31) // 32) * 32
        traffic_summary(sys.argv[2], sys.argv[3], nx, sys.argv[7], sys.argv[8], " ".join(sys.argv[9:]),
                        copy_elems=(nz + 1) * (ny + 1) * pitch, dominant="k_waves_sweep<false>",
                        a_eff=11 * nx * ny * nz * 8, grid=f"{nx}x{ny}x{nz}",
                        kernel_src=os.path.join(ROOT, "paper_2207_08716_amd", "csrc", "waves.hip"))
    else:
        raise SystemExit(__doc__)
