"""Summaries of rocprofv3 output for profiles/ (text) and bench.py (traffic).

    python -m paper_2401_04189_amd.profsum ktrace  <run_kernel_stats.csv> <out.md> "<command>"
    python -m paper_2401_04189_amd.profsum traffic <fetch.csv> <write.csv> <out.md> "<fetch cmd>" "<write cmd>"

`traffic` scales the per-dispatch FETCH_SIZE / WRITE_SIZE counters (KiB) by
what the same counters read for bench.py's calibration kernel (an
elementwise dst = 2*src over 512 MiB: 512 MiB read, 512 MiB written), and
records the per-launch HBM bytes of each exchange kernel in
profiles/traffic_core.json together with the hash of the kernel source they
were taken from (bench.py reports them only while the source is unchanged).
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
KERNEL_SRC = os.path.join(ROOT, "paper_2401_04189_amd", "csrc", "txe_kernels.hip")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_core.json")
CAL_BYTES = 512 << 20


def short(name):
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)
    return name.replace("txe::", "").replace("void ", "") or "(torch / runtime kernel)"


def ktrace(stats_csv, out_md, cmd):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ["# Kernel trace: 64^3 exchange apply (2080 unique pairs, r = 40, K = 40)", "",
             "Command (from the repository root, on the machine with the GPU):", "", "```", cmd, "```", "",
             "| Kernel | Calls | Average (ms) | Min (ms) | Max (ms) | Share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.2f}% |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return agg


def traffic(fetch_csv, write_csv, out_md, cmd_f, cmd_w):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    # calibration kernel: the elementwise kernel with the largest fetch
    cal_f = max((max(v) for k, v in fetch.items() if "elementwise" in k), default=None)
    cal_w = max((max(v) for k, v in write.items() if "elementwise" in k), default=None)
    sf = CAL_BYTES / cal_f if cal_f else None
    sw = CAL_BYTES / cal_w if cal_w else None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    lines = ["# HBM traffic per launch: 64^3 exchange apply, FP32 MFMA form", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two separate rocprofv3 runs, scaled",
             "by the counters of a calibration kernel of known size (elementwise dst = 2*src over",
             f"512 MiB): fetch scale {sf:.4f}, write scale {sw:.4f}.", "",
             f"Kernel source hash: `{sha}`", "", "Commands:", "", "```", cmd_f, cmd_w, "```", "",
             "| Kernel | Fetch (MB) | Write (MB) |", "|---|---|---|"]
    rec = {}
    for k in fetch:
        if "txe::" not in k:
            continue
        f = sum(fetch[k]) / len(fetch[k]) * (sf or 1.0)
        w = sum(write.get(k, [0.0])) / max(len(write.get(k, [1])), 1) * (sw or 1.0)
        lines.append(f"| `{short(k)}` | {f / 1e6:.1f} | {w / 1e6:.1f} |")
        m = re.search(r"k_core<(float|double)", k)
        if m:
            rec[f"cfg2/{'f32' if m.group(1) == 'float' else 'f64'}"] = {
                "kernel_source_sha": sha, "bytes_per_launch": round(f + w), "fetch_bytes": round(f),
                "write_bytes": round(w), "fetch_scale": sf, "write_scale": sw}
    open(out_md, "w").write("\n".join(lines) + "\n")
    old = {}
    if os.path.exists(TRAFFIC_JSON):
        old = json.load(open(TRAFFIC_JSON))
    old.update(rec)
    json.dump(old, open(TRAFFIC_JSON, "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "ktrace":
        ktrace(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "traffic":
        traffic(sys.argv[2], sys.argv[3], sys.argv[4], sys.argv[5], sys.argv[6])
    else:
        raise SystemExit(__doc__)
