"""Summaries of rocprofv3 output for profiles/ (text) and bench.py (traffic).

    python -m paper_2401_04189_amd.profsum ktrace  <run_kernel_stats.csv> <out.md> "<title>" "<command>"
    python -m paper_2401_04189_amd.profsum traffic <fetch.csv> <write.csv> <out.md> "<title>" <key> \
        "<fetch cmd>" "<write cmd>" [<algorithmic core bytes per launch>]
    python -m paper_2401_04189_amd.profsum sq <counter_collection.csv> <out.md> "<title>" "<command>" \
        [<FP32 core flops per launch> [<FP64 core flops per launch>]]

`traffic` scales the per-dispatch FETCH_SIZE / WRITE_SIZE counters (KiB) by
what the same counters read for bench.py's calibration kernel (torch.mul of
a 512 MiB FP64 tensor by 2: 512 MiB read, 512 MiB written; the first
AUnaryFunctor dispatch of the run), and records the per-launch HBM bytes of
the core kernel in profiles/traffic_core.json under <key> (e.g. "cfg4/f32")
together with the hash of the kernel source they were taken from (bench.py
reports them only while that source is unchanged).

`sq` summarises one pass of SQ / GRBM counters per kernel: cycles =
GRBM_GUI_ACTIVE / 8 (the counter sums the eight XCDs), MFMA busy =
SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles), executed MFMA flops =
SQ_INSTS_VALU_MFMA_MOPS_* x 512, waits = SQ_WAIT_ANY / SQ_WAVE_CYCLES, LDS
conflict share = SQ_LDS_BANK_CONFLICT / (256 CUs x cycles).
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
CSRC = os.path.join(ROOT, "paper_2401_04189_amd", "csrc")
# the sources the core kernel is compiled from (the traffic counters are tied to them)
KERNEL_SRC = [os.path.join(CSRC, f) for f in ("txe_core.h", "txe_dev.h")]
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic_core.json")
CAL_BYTES = 512 << 20


def source_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRC:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def short(name):
    name = name.replace("(anonymous namespace)::", "")
    name = re.sub(r"\(.*", "", name)
    name = name.replace("txe::", "").replace("void ", "")
    if name.startswith("Cijk_"):
        return "rocBLAS GEMM (input generation)"
    if name.startswith("at::native::"):
        return "torch elementwise (input generation)"
    return name or "(torch / runtime kernel)"


def ktrace(stats_csv, out_md, title, cmd):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# Kernel trace: {title}", "",
             "Command (from the repository root, on the machine with the GPU):", "", "```", cmd, "```", "",
             "| Kernel | Calls | Average (ms) | Min (ms) | Max (ms) | Share |", "|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e6:.4f} | "
                     f"{float(r['MinNs']) / 1e6:.4f} | {float(r['MaxNs']) / 1e6:.4f} | {float(r['Percentage']):.2f}% |")
    open(out_md, "w").write("\n".join(lines) + "\n")


def _per_kernel(path, counter):
    agg = collections.defaultdict(list)
    first = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter:
            agg[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
            d = int(r["Dispatch_Id"])
            if "AUnaryFunctor" in r["Kernel_Name"] and ("cal" not in first or d < first["cal"][0]):
                first["cal"] = (d, float(r["Counter_Value"]) * 1024.0)
    return agg, first.get("cal", (None, None))[1]


def traffic(fetch_csv, write_csv, out_md, title, key, cmd_f, cmd_w, alg_bytes=None):
    fetch, cal_f = _per_kernel(fetch_csv, "FETCH_SIZE")
    write, cal_w = _per_kernel(write_csv, "WRITE_SIZE")
    sf = CAL_BYTES / cal_f if cal_f else None
    sw = CAL_BYTES / cal_w if cal_w else None
    sha = source_sha()
    lines = [f"# HBM traffic per launch: {title}", "",
             "FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two separate rocprofv3 runs, scaled",
             "by the counters of a calibration kernel of known size (torch.mul of 512 MiB of FP64 by 2:",
             f"512 MiB read, 512 MiB written): fetch scale {sf:.4f}, write scale {sw:.4f}.", "",
             f"Core kernel source hash (txe_core.h, txe_dev.h): `{sha}`", "", "Commands:", "", "```", cmd_f, cmd_w,
             "```", "", "| Kernel | Launches | Fetch (GB) | Write (GB) |", "|---|---|---|---|"]
    rec = {}
    for k in fetch:
        if "txe::" not in k:
            continue
        f = sum(fetch[k]) / len(fetch[k]) * (sf or 1.0)
        w = sum(write.get(k, [0.0])) / max(len(write.get(k, [1])), 1) * (sw or 1.0)
        lines.append(f"| `{short(k)}` | {len(fetch[k])} | {f / 1e9:.2f} | {w / 1e9:.2f} |")
        want = "double" if key.endswith("f64") else "float"
        if re.search(r"k_core<" + want, k):
            rec[key] = {"kernel_source_sha": sha, "kernel": short(k), "bytes_per_launch": round(f + w),
                        "fetch_bytes": round(f), "write_bytes": round(w), "fetch_scale": sf, "write_scale": sw}
            if alg_bytes:
                rec[key]["algorithmic_bytes"] = float(alg_bytes)
                lines_alg = (f"Core kernel: {(f + w) / 1e9:.1f} GB moved per launch against "
                             f"{float(alg_bytes) / 1e9:.1f} GB algorithmic ({(f + w) / float(alg_bytes):.1f}x).")
    if alg_bytes and key in rec:
        lines += ["", lines_alg]
    open(out_md, "w").write("\n".join(lines) + "\n")
    old = {}
    if os.path.exists(TRAFFIC_JSON):
        old = json.load(open(TRAFFIC_JSON))
    old.update(rec)
    json.dump(old, open(TRAFFIC_JSON, "w"), indent=1)


def sq(csv_path, out_md, title, cmd, f32_core_flops=None, f64_core_flops=None, clock_ghz=2.4):
    per = collections.defaultdict(lambda: collections.defaultdict(dict))
    for r in csv.DictReader(open(csv_path)):
        per[r["Kernel_Name"]][int(r["Dispatch_Id"])][r["Counter_Name"]] = float(r["Counter_Value"])
    lines = [f"# Core-kernel counters: {title}", "", "Command (from the repository root, on the machine with the GPU):",
             "", "```", cmd, "```", "",
             "Derived per dispatch (averages over the dispatches of each kernel): cycles = GRBM_GUI_ACTIVE / 8;",
             "MFMA busy = SQ_VALU_MFMA_BUSY_CYCLES / (1024 SIMDs x cycles); executed MFMA flops =",
             "SQ_INSTS_VALU_MFMA_MOPS_* x 512 (a 16x16x4 MFMA counts 4); executed / algorithmic is the work the",
             "tiling adds; waits = SQ_WAIT_ANY / SQ_WAVE_CYCLES; LDS conflict share = SQ_LDS_BANK_CONFLICT /",
             "(256 CUs x cycles).", "",
             "| Kernel | Dispatches | ms (cycles / clock) | MFMA busy | Executed TFLOP/s | Executed / algorithmic | Waits | LDS conflict share |",
             "|---|---|---|---|---|---|---|---|"]
    for k, ds in per.items():
        if "txe::" not in k:
            continue
        def avg(name):
            v = [d.get(name, 0.0) for d in ds.values()]
            return sum(v) / len(v)
        cyc = avg("GRBM_GUI_ACTIVE") / 8.0
        if cyc <= 0:
            continue
        ms = cyc / (clock_ghz * 1e6)
        busy = avg("SQ_VALU_MFMA_BUSY_CYCLES") / (1024.0 * cyc)
        flops = (avg("SQ_INSTS_VALU_MFMA_MOPS_F32") + avg("SQ_INSTS_VALU_MFMA_MOPS_F64")) * 512.0
        tf = flops / (ms * 1e-3) / 1e12
        alg = f32_core_flops if re.search(r"k_core<float", k) else f64_core_flops if re.search(r"k_core<double", k) else None
        ratio = f"{flops / float(alg):.2f}" if alg else "—"
        waits = avg("SQ_WAIT_ANY") / max(avg("SQ_WAVE_CYCLES"), 1.0)
        lds = avg("SQ_LDS_BANK_CONFLICT") / (256.0 * cyc)
        lines.append(f"| `{short(k)}` | {len(ds)} | {ms:.1f} | {busy:.2f} | {tf:.1f} | {ratio} | {waits:.2f} | {lds:.2f} |")
    open(out_md, "w").write("\n".join(lines) + "\n")


if __name__ == "__main__":
    if sys.argv[1] == "ktrace":
        ktrace(*sys.argv[2:6])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:10])
    elif sys.argv[1] == "sq":
        sq(*sys.argv[2:6], *[float(x) for x in sys.argv[6:8]])
    else:
        raise SystemExit(__doc__)
