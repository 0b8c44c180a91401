#!/usr/bin/env python3
"""Throughput of the Tucker-tensor Fock-exchange hot path on one MI355X.

Default workload: the 128^3 block (1,842 orbitals from Gaussians on 310
rutile sites, r = 80, K = 50).  One step = one exchange apply (pair
densities, projection onto the shared Tucker bases, core-space Gaussian
kernel sum, back-projection, product with psi_j and sum over sources, pair
energies, E_x) for the next batch of 4 targets of the 128-target block
against all 1,842 sources (7,368 pairs), inputs resident in HBM.  The metric
is pair convolutions per second of the FP32-MFMA form, counted only when its
batch energies are within 1e-5 Ha of the FP64 form's, which is timed beside
it together with the split-bf16 forms.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config cfg4]

`--config cfg2` / `cfg3` time the symmetric 64^3 / 80^3 workloads (all unique
pairs per step); `--config cfg5` times 24 uneven systems as one captured
graph replay against 24 separate applies, FP32 MFMA, with every system's E_x
checked against its FP64 form.

Prints one JSON line.  Per-kernel durations come from HIP events the library
records on its own stream around every launch (txe_profile_*).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair convolutions/s for Vx psi, MFMA-FP32 vs FP64 at dE_x<=1e-5 Ha; % roofline"
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3, "bf16": 2516.0}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_core.json")
TUNE_CACHE = os.path.join(ROOT, "paper_2401_04189_amd", "tuned_shapes.json")


def flops_per_pair(n, r, K):
    """Algorithmic flops of one pair convolution (2 flops per multiply-add).

    projection and back-projection: n0 n1 n2 r2 + n0 n1 r1 r2 + n0 r0 r1 r2 each;
    core-space kernel sum: K r0 r1 r2 (r0 + r1 + r2); pair energy: r0 r1 r2."""
    n0, n1, n2 = n
    r0, r1, r2 = r
    proj = n0 * n1 * n2 * r2 + n0 * n1 * r1 * r2 + n0 * r0 * r1 * r2
    core = K * r0 * r1 * r2 * (r0 + r1 + r2)
    return 2.0 * (2 * proj + core + r0 * r1 * r2)


def core_kernel_flops_per_pair(n, r, K):
    """Algorithmic flops of the core kernel alone: the kernel sum, the pair
    energy dot and the first (mode-0) back-projection stage fused into it."""
    r0, r1, r2 = r
    return 2.0 * (K * r0 * r1 * r2 * (r0 + r1 + r2) + r0 * r1 * r2 + n[0] * r0 * r1 * r2)


def load_traffic(compute, cfg):
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    ent = t.get(f"{cfg}/{compute}")
    from paper_2401_04189_amd.profsum import source_sha

    if not ent or ent.get("kernel_source_sha") != source_sha():
        return None
    return ent.get("bytes_per_launch")


def time_leg(txe, torch, ctx, sysm, psi, vx, compute, steps, warmup, symmetric, i0, Ni):
    for _ in range(warmup):
        txe.apply(ctx, sysm, psi, compute=compute, symmetric=symmetric, i0=i0, Ni=Ni, vx_out=vx)
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        _, ex, _ = txe.apply(ctx, sysm, psi, compute=compute, symmetric=symmetric, i0=i0, Ni=Ni, vx_out=vx)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = ctx.kernel_times()
    ctx.profile(False)
    return wall, float(ex.item()), kt


def shapes(args, txe, ctx, sysm, psi, compute, symmetric=True, i0=0, Ni=None):
    """Launch shapes for one leg: the committed tuning cache, else a live
    search before the timed region (saved with --retune), else (--no-tune, or
    the block workload without --retune) the defaults."""
    if args.no_tune:
        return "defaults"
    kn, tuned = txe.plan(ctx, sysm, psi, compute, symmetric, i0, Ni)
    if tuned and not args.retune:
        return {"source": "cache", **kn}
    if not symmetric and not args.retune:
        return {"source": "defaults", **kn}
    ms, kn = txe.tune(ctx, sysm, psi, compute, symmetric, i0, Ni, reps=1 if not symmetric else 2)
    return {"source": "tuned live", **kn}


def load_cache(args, txe, ctx):
    # with --retune the file's other entries are kept (merged) and rewritten
    if not args.no_tune and os.path.exists(TUNE_CACHE):
        txe.tune_load(ctx, TUNE_CACHE)


def copy_calibration(torch):
    """One elementwise kernel of known traffic (reads 512 MiB, writes 512 MiB):
    the reference for scaling the HBM byte counters of a profile."""
    src = torch.empty(64 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    torch.mul(src, 2.0, out=dst)
    torch.cuda.synchronize()
    print(f"copy calibration: {src.numel() * 8} bytes read and written", file=sys.stderr, flush=True)
    del src, dst


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def block_cpu_baseline(s, seconds, single_seconds):
    """The CPU FP64 oracle, as it stands, on target 0 of the 128^3 block against
    its sources in order, until `seconds` of work are done (all host cores as
    BLAS threads), then a single-thread rate on the next sources."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import txe_oracle as O

    t0 = time.perf_counter()
    st = O.Setup(s.grid.x, s.grid.q, s.U, s.w, s.alpha)
    setup_s = time.perf_counter() - t0
    pi = s.psi[0].double().cpu().numpy()

    def run(j0, budget):
        done = 0
        t = time.perf_counter()
        while time.perf_counter() - t < budget and j0 + done < s.N:
            O.pair(pi, s.psi[j0 + done].double().cpu().numpy(), st)
            done += 1
        return done, time.perf_counter() - t

    done, el = run(0, seconds)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    with threadpool_limits(limits=1):
        done1, el1 = run(done, single_seconds)
    return {"value": round(done / el, 3), "unit": "pair-convolutions/s", "cores": int(threads), "kind": "oracle",
            "single_thread_value": round(done1 / el1, 3), "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"target 0 of the 128^3 block against its first {done} sources (numpy FP64, {el:.1f} s, "
                      f"{threads} BLAS threads), then sources {done}..{done + done1 - 1} on one thread "
                      f"({el1:.1f} s); setup tables {setup_s:.1f} s, not timed"}


def bench_block(args, txe, torch, W):
    """The 128^3 block (default): batches of `--batch` targets of the 128-target
    block against all 1,842 sources, r = 80, K = 50.  One step = one batch
    (the next one each step).  FP32 MFMA (the value) is timed for exactly
    --steps steps after --warmup batches; FP64, bf16 x3 and bf16 x6 are timed
    beside it on the first --side-steps batches.  Every reduced form is
    compared with FP64 on the batches both timed (|dE_batch|) and on batch 0
    (Vx psi per orbital in the W-norm, exchange-matrix diagonal from the
    library)."""
    if args.copy_calibration:
        copy_calibration(torch)
    t0 = time.perf_counter()
    s = W.build_config("cfg4", device="cuda")
    torch.cuda.empty_cache()
    print(f"generated the 128^3 block workload in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    load_cache(args, txe, ctx)
    psi = s.psi
    N, B = s.N, args.batch
    nbatch = 128 // B
    npairs = B * N
    w3 = s.grid.weights3d(device="cuda")
    vx = torch.empty((B,) + tuple(psi.shape[1:]), dtype=psi.dtype, device="cuda")
    n, r, K = s.grid.n, s.r, s.K
    legs, ref_batch0 = {}, {}
    for comp in args.legs.split(","):
        main = comp == "f32"
        steps = args.steps if main else max(1, min(args.steps, args.side_steps))
        warm = args.warmup if main else 1
        tuned = shapes(args, txe, ctx, sysm, psi, comp, symmetric=False, i0=0, Ni=B)
        for w in range(warm):
            txe.apply(ctx, sysm, psi, compute=comp, symmetric=False, i0=(w % nbatch) * B, Ni=B, vx_out=vx)
        torch.cuda.synchronize()
        print(f"{comp}: {warm} warm-up batches done", file=sys.stderr, flush=True)
        ctx.profile(True)
        exs = []
        t = time.perf_counter()
        for k in range(steps):
            exs.append(txe.apply(ctx, sysm, psi, compute=comp, symmetric=False, i0=(k % nbatch) * B, Ni=B,
                                 vx_out=vx)[1])
            if k % 5 == 4 or k == steps - 1:
                print(f"{comp}: step {k + 1}/{steps} enqueued", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t) / steps
        kt = ctx.kernel_times()
        ctx.profile(False)
        # batch 0 once more, untimed, for the per-orbital comparisons
        v0, e0, _, d0 = txe.apply(ctx, sysm, psi, compute=comp, symmetric=False, i0=0, Ni=B, want_orb=True)
        torch.cuda.synchronize()
        ref_batch0[comp] = (v0, float(e0), d0)
        legs[comp] = dict(sec=sec, steps=steps, warmup=warm, ex=[float(e) for e in exs], kt=kt, shapes=tuned)
        print(f"{comp}: {1e3 * sec:.1f} ms per batch", file=sys.stderr, flush=True)
    peak = {"f64": PEAK_TFLOPS["f64"], "f32": PEAK_TFLOPS["f32"], "bf16x3": PEAK_TFLOPS["bf16"] / 3,
            "bf16x6": PEAK_TFLOPS["bf16"] / 6}
    core_fl = core_kernel_flops_per_pair(n, r, K)
    out_legs = {}
    for comp, L in legs.items():
        core_ms, core_n = L["kt"]["core"]
        launches = max(core_n, 1)
        launch_ms = core_ms / launches
        achieved = core_fl * npairs * L["steps"] / (core_ms * 1e-3) / 1e12
        e = {"value": round(npairs / L["sec"], 1), "ms_per_step": round(1e3 * L["sec"], 3), "steps": L["steps"],
             "warmup": L["warmup"], "E_batch0": L["ex"][0],
             "kernel_ms_per_launch": {k: round(v[0] / max(v[1], 1), 4) for k, v in L["kt"].items()},
             "launches_per_step": {k: v[1] // L["steps"] for k, v in L["kt"].items()},
             "core_tflops": round(achieved, 3), "core_peak_tflops": round(peak[comp], 1),
             "core_frac": round(achieved / peak[comp], 4), "core_launch_ms": round(launch_ms, 3),
             "launch_shapes": L["shapes"]}
        if comp != "f64" and "f64" in legs:
            both = min(len(L["ex"]), len(legs["f64"]["ex"]))
            v0, e0, d0 = ref_batch0[comp]
            v64, e64, d64 = ref_batch0["f64"]
            num = ((v0 - v64) ** 2 * w3).sum(dim=(1, 2, 3))
            den = (v64 ** 2 * w3).sum(dim=(1, 2, 3))
            e["dE_batch_Ha_max"] = max(abs(a - b) for a, b in zip(L["ex"][:both], legs["f64"]["ex"][:both]))
            e["batches_compared"] = both
            e["vx_rel_wnorm_max"] = float(torch.sqrt(num / den).max())
            e["diag_abs_max_Ha"] = float((d0 - d64).abs().max())
            e["within_1e-5_Ha"] = e["dE_batch_Ha_max"] <= 1e-5
            e["over_fp64"] = round(legs["f64"]["sec"] / L["sec"], 3)
        out_legs[comp] = e
    # the FP32 leg is the value when its energies pass the gate against FP64
    # (or, when FP64 is not timed in this run, ungated: say so in the line)
    gated = "f64" in out_legs
    use = "f32" if "f32" in out_legs and (not gated or out_legs["f32"].get("within_1e-5_Ha")) else "f64"
    U = out_legs[use]
    roof = {"bound": "mfma", "kernel": "core", "achieved": U["core_tflops"], "peak": PEAK_TFLOPS[use],
            "unit": "TFLOP/s", "frac": round(U["core_tflops"] / PEAK_TFLOPS[use], 4),
            "traffic": load_traffic(use, "cfg4"), "launch_ms": U["core_launch_ms"],
            "flops_per_launch": core_fl * npairs / max(U["launches_per_step"]["core"], 1)}
    measured = ctx.ceiling(use)
    roof["measured_peak"] = round(measured, 1)
    roof["frac_of_measured"] = round(U["core_tflops"] / measured, 4)
    out = {
        "metric": METRIC, "value": U["value"], "unit": "pair-convolutions/s",
        "n_gpus": 1, "steps": legs[use]["steps"], "warmup": legs[use]["warmup"],
        "ms_per_step": U["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": use, "data": "synthetic",
        "config": {"workload": W.WORKLOAD_NAMES["cfg4"] + f"; one step = the next {B}-target batch of the block "
                   f"against all {N} sources ({npairs} pairs)", "grid": list(n), "orbitals": N, "rank": list(r),
                   "terms": K, "batch_targets": B, "pairs_per_step": npairs, "mode": "block (targets x all sources)"},
        "legs": out_legs,
        "energy_gate_evaluated": gated,
        "fp32_over_fp64": out_legs.get("f32", {}).get("over_fp64"),
        "whole_path_tflops": round(flops_per_pair(n, r, K) * npairs / (U["ms_per_step"] * 1e-3) / 1e12, 3),
        "roofline": roof,
        "measured_ceilings": {"f64_mfma_tflops": round(ctx.ceiling("f64"), 1),
                              "f32_mfma_tflops": round(ctx.ceiling("f32"), 1),
                              "bf16_mfma_tflops": round(ctx.ceiling("bf16"), 1),
                              "hbm_stream_gbs": round(ctx.ceiling("hbm"), 1)},
    }
    if args.retune:
        txe.tune_save(ctx, TUNE_CACHE)
    sysm.close()
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = block_cpu_baseline(s, args.cpu_seconds, args.cpu_single_seconds)
    print(json.dumps(out), flush=True)


def bench_batched(args, txe, torch, W):
    """cfg5: one graph replay of all systems against separate applies."""
    t0 = time.perf_counter()
    systems = W.build_cfg5(device="cuda")
    print(f"generated {len(systems)} systems in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    ctx = txe.Context(0)
    handles = [txe.System.from_workload(ctx, s) for s in systems]
    items = [(h, s.psi.contiguous()) for h, s in zip(handles, systems)]
    npairs = sum(s.N * (s.N + 1) // 2 for s in systems)
    ex64 = []
    for k, (h, p) in enumerate(items):
        ex64.append(float(txe.apply(ctx, h, p, compute="f64", want_vx=False)[1]))
        print(f"FP64 energy of system {k}: {ex64[-1]:.10f}", file=sys.stderr, flush=True)
    load_cache(args, txe, ctx)
    tuned = []
    for k, (h, p) in enumerate(items):
        tuned.append(shapes(args, txe, ctx, h, p, "f32"))
        print(f"launch shape of system {k}: {tuned[-1]}", file=sys.stderr, flush=True)
    if args.retune:
        txe.tune_save(ctx, TUNE_CACHE)
    print(f"launch shapes: {sum(isinstance(t, dict) and t['source'] == 'cache' for t in tuned)} from the cache, "
          f"{sum(isinstance(t, dict) and t['source'] != 'cache' for t in tuned)} tuned live", file=sys.stderr, flush=True)
    vxs = [torch.empty_like(p) for _, p in items]

    def separate():
        return [txe.apply(ctx, h, p, compute="f32", vx_out=v)[1] for (h, p), v in zip(items, vxs)]

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t) / args.steps

    sep_s = timed(separate)
    ctx.profile(True)
    separate()
    torch.cuda.synchronize()
    kt = ctx.kernel_times()
    ctx.profile(False)
    # each system's core time on its own (where the batch's time goes)
    per_system = []
    for (h, p), v, s in zip(items, vxs, systems):
        ctx.profile(True)
        txe.apply(ctx, h, p, compute="f32", vx_out=v)
        torch.cuda.synchronize()
        ks = ctx.kernel_times()
        ctx.profile(False)
        np_ = s.N * (s.N + 1) // 2
        per_system.append({"n": s.grid.n[0], "N": s.N, "r": s.r[0], "pairs": np_,
                           "core_ms": round(ks["core"][0], 3),
                           "core_tflops": round(core_kernel_flops_per_pair(s.grid.n, s.r, s.K) * np_
                                                / (ks["core"][0] * 1e-3) / 1e12, 1)})
    # concurrency of the batch: the lane count with the fastest eager batch
    lane_ms = {}
    for ln in (1, 2, 4):
        lane_ms[ln] = 1e3 * timed(lambda: txe.apply_batched(ctx, items, compute="f32", lanes=ln))
    lanes = min(lane_ms, key=lane_ms.get)
    bat_s = lane_ms[lanes] / 1e3
    g = txe.Graph(ctx, items, compute="f32", lanes=lanes)
    graph_s = timed(g.launch)
    ex32 = [float(o[1]) for o in g.outputs]
    g.close()
    dE = [abs(a - b) for a, b in zip(ex32, ex64)]
    core_ms = kt["core"][0]
    core_flops = sum(core_kernel_flops_per_pair(s.grid.n, s.r, s.K) * s.N * (s.N + 1) // 2 for s in systems)
    achieved = core_flops / (core_ms * 1e-3) / 1e12
    # the same with every rank rounded up to the 16-row MFMA tiles it occupies
    # (the kernels' M and N dimensions run over the padded rows)
    pad = lambda r: [16 * ((v + 15) // 16) for v in r]  # noqa: E731
    padded_flops = sum(core_kernel_flops_per_pair(s.grid.n, pad(s.r), s.K) * s.N * (s.N + 1) // 2 for s in systems)
    out = {
        "metric": METRIC,
        "value": round(npairs / graph_s, 1),
        "unit": "pair-convolutions/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * graph_s, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": W.WORKLOAD_NAMES["cfg5"], "systems": len(systems), "pairs": npairs,
                   "mode": "one captured graph, symmetric unique pairs per system", "lanes": lanes},
        "separate_launches": {"value": round(npairs / sep_s, 1), "ms_per_step": round(1e3 * sep_s, 4)},
        "batched_eager": {"value": round(npairs / bat_s, 1), "ms_per_step": round(1e3 * bat_s, 4),
                          "ms_by_lanes": {str(k): round(v, 3) for k, v in lane_ms.items()}},
        "graph_over_separate": round(sep_s / graph_s, 3),
        "per_system_core": per_system,
        "max_dE_x_fp32_vs_fp64_Ha": max(dE),
        "all_within_1e-5_Ha": max(dE) <= 1e-5,
        "launch_shapes": "defaults" if args.no_tune else
        {"from_cache": sum(t["source"] == "cache" for t in tuned), "tuned_live": sum(t["source"] != "cache" for t in tuned)},
        "roofline": {"bound": "mfma", "kernel": "core", "achieved": round(achieved, 3), "peak": PEAK_TFLOPS["f32"],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f32"], 4), "traffic": None,
                     "launch_ms": round(core_ms / max(kt["core"][1], 1), 4),
                     "frac_on_padded_ranks": round(padded_flops / (core_ms * 1e-3) / 1e12 / PEAK_TFLOPS["f32"], 4)},
    }
    for h in handles:
        h.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def colloc_flops_per_pair(n, r, K):
    """Algorithmic flops of the collocation reconstruction of one pair:
    per term G x0 A0 (n0 r0 r1 r2), x1 A1 (n0 n1 r1 r2), x2 A2 (n0 n1 n2 r2)."""
    n0, n1, n2 = n
    r0, r1, r2 = r
    return 2.0 * K * (n0 * r0 * r1 * r2 + n0 * n1 * r1 * r2 + n0 * n1 * n2 * r2)


def bench_fe(args, txe, torch, W):
    """Order-5 Lagrange elements on adaptively refined meshes: the core-space
    form in FP32 and FP64 and the collocation form (FP64) on one system."""
    p, L, r, K, N = 5, 10.0, 40, 40, 64
    atoms = W._atoms(("fcc", 13))
    edges = [W.adaptive_edges(L=L, bms=5.0, msna=1.5, centres=sorted(set(np.round(atoms[:, d], 9))), ball=1.0, p=p)
             for d in range(3)]
    xq = [txe.fe_mesh_1d(e, p) for e in edges]
    g = W.grid_from_nodes([v[0] for v in xq], [v[1] for v in xq])
    psi_h, _ = W.make_orbitals(g, N, 6, (0.3, 3.0), seed=2, atoms=atoms)
    U = W.hosvd_bases(psi_h, g, (r, r, r))
    w, alpha = W.exp_sum(K)
    C = [txe.fe_conv_matrices(e, p, alpha) for e in edges]
    ctx = txe.Context(0)
    sysm = txe.System(ctx, [v[0] for v in xq], [v[1] for v in xq], U, w, alpha, C=C)
    psi = psi_h.cuda()
    vx = torch.empty_like(psi)
    n = g.n
    npairs = N * (N + 1) // 2
    legs = {}
    load_cache(args, txe, ctx)
    side = max(1, min(args.steps, args.side_steps))
    for name, compute, form, pb, steps in (("f32", "f32", "core", False, args.steps),
                                           ("f64", "f64", "core", False, side),
                                           ("f64_collocation", "f64", "collocation", False, side),
                                           ("f64_pair_bases", "f64", "core", True, side)):
        for _ in range(1 if name != "f32" else args.warmup):
            txe.apply(ctx, sysm, psi, compute=compute, vx_out=vx, form=form, pair_bases=pb)
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            _, ex, _ = txe.apply(ctx, sysm, psi, compute=compute, vx_out=vx, form=form, pair_bases=pb)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / steps
        kt = ctx.kernel_times()
        ctx.profile(False)
        legs[name] = {"value": round(npairs / wall, 1), "ms_per_step": round(1e3 * wall, 4), "steps": steps,
                      "E_x": float(ex.item()),
                      "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kt.items()},
                      "launches": {k: v[1] for k, v in kt.items()}}
        print(f"{name}: {1e3 * wall:.1f} ms per apply", file=sys.stderr, flush=True)
    f32, f64, col = legs["f32"], legs["f64"], legs["f64_collocation"]
    core_ms = f32["kernel_ms"]["core"]
    achieved = core_kernel_flops_per_pair(n, (r, r, r), K) * npairs / (core_ms * 1e-3) / 1e12
    # the reconstruction's mode products run as 3 K launches per apply; their summed time per apply
    rec_ms = col["kernel_ms"]["core"] * col["launches"]["core"] / col["steps"]
    col_tf = colloc_flops_per_pair(n, (r, r, r), K) * npairs / (rec_ms * 1e-3) / 1e12
    col["reconstruction"] = {"bound": "mfma", "achieved": round(col_tf, 3), "peak": PEAK_TFLOPS["f64"],
                             "unit": "TFLOP/s", "frac": round(col_tf / PEAK_TFLOPS["f64"], 4),
                             "ms_per_apply": round(rec_ms, 3), "measured_peak": round(ctx.ceiling("f64"), 1)}
    col["dE_x_vs_core_form_Ha"] = abs(col["E_x"] - f64["E_x"])
    ppb = legs["f64_pair_bases"]
    ppb["dE_x_vs_shared_bases_Ha"] = abs(ppb["E_x"] - f64["E_x"])
    ppb["note"] = ("kernel_ms: proj12 = the per-pair decompositions (two Gram/Jacobi stages and the truncation "
                   "per mode), proj3 = the per-pair core matrices, core = the shared core kernel on them, "
                   "back = the back-projection in the pair's bases")
    out = {
        "metric": METRIC, "value": f32["value"], "unit": "pair-convolutions/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": f32["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "exchange apply on order-5 Lagrange elements at GLL nodes, adaptively refined "
                               "1-D meshes on [-10,10] (base cell 5, cells near atoms <= 1.5), 64^3 nodes, "
                               "64 orbitals on a 13-atom fcc cluster, r=40, K=40, 2080 unique pairs",
                   "grid": list(n), "order": p, "cells": [len(e) - 1 for e in edges], "orbitals": N,
                   "pairs": npairs, "rank": [r, r, r], "terms": K},
        "legs": legs,
        "dE_x_fp32_vs_fp64_Ha": abs(f32["E_x"] - f64["E_x"]),
        "fp32_over_fp64": round(f64["ms_per_step"] / f32["ms_per_step"], 3),
        "roofline": {"bound": "mfma", "kernel": "core", "achieved": round(achieved, 3),
                     "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS["f32"], 4),
                     "traffic": None, "launch_ms": core_ms, "measured_peak": round(ctx.ceiling("f32"), 1)},
    }
    sysm.close()
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_ace(txe, torch, ctx, sysm, psi, vx, args):
    """Adaptively compressed exchange from the FP32 exchange action already
    in vx: build time (Gram matrix, Cholesky factor and inverse, projection
    vectors) and the time of one V_ACE apply to N trial functions, with the
    FP64 flops of the two grid contractions of each."""
    txe.apply(ctx, sysm, psi, compute="f32", vx_out=vx)
    xi, info = txe.ace_build(ctx, sysm, psi, vx)
    out = txe.ace_apply(ctx, sysm, xi, psi)
    torch.cuda.synchronize()
    exact = float((out - vx).abs().max() / vx.abs().max())
    steps = max(args.steps, 3)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(steps):
        txe.ace_build(ctx, sysm, psi, vx)
    ev[1].record()
    for _ in range(steps):
        txe.ace_apply(ctx, sysm, xi, psi)
    ev[2].record()
    torch.cuda.synchronize()
    b_ms, a_ms = ev[0].elapsed_time(ev[1]) / steps, ev[1].elapsed_time(ev[2]) / steps
    N, ng = psi.shape[0], psi[0].numel()
    # build: M (N^2 ng MACs) and xi = L^-1 W (lower triangle: N(N+1)/2 ng); apply: 2 N^2 ng
    b_fl, a_fl = 2.0 * (N * N + N * (N + 1) / 2) * ng, 2.0 * 2 * N * N * ng
    return {"info": int(info), "exact_rel": exact, "build_ms": round(b_ms, 4), "apply_ms": round(a_ms, 4),
            "build_tflops_f64": round(b_fl / (b_ms * 1e-3) / 1e12, 2),
            "apply_tflops_f64": round(a_fl / (a_ms * 1e-3) / 1e12, 2), "peak_f64": PEAK_TFLOPS["f64"]}


def cpu_baseline(s, seconds):
    """The CPU FP64 oracle, as it stands, on the first unique pairs of the same
    workload until `seconds` of work are done."""
    from threadpoolctl import threadpool_info

    from oracle import txe_oracle as O

    st = O.Setup.from_system(s)
    psi = s.psi.numpy()
    N = psi.shape[0]
    pairs = [(i, j) for i in range(N) for j in range(i, N)]
    done = 0
    t0 = time.perf_counter()
    for (i, j) in pairs:
        O.pair(psi[i], psi[j], st)
        done += 1
        if time.perf_counter() - t0 >= seconds:
            break
    el = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    return {"value": done / el, "unit": "pair-convolutions/s", "cores": int(threads), "kind": "oracle",
            "sample": f"first {done} of {len(pairs)} unique pairs of the same workload (numpy FP64, "
                      f"{el:.1f} s, {threads} BLAS threads, host has {os.cpu_count()} CPUs)"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="cfg4", choices=["cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "fe5"],
                    help="workload: cfg4 = the 128^3 block (default), cfg2 = 64^3 symmetric, cfg3 = 80^3 "
                         "symmetric, cfg5 = 24 uneven systems in one graph, fe5 = order-5 elements on adaptive "
                         "meshes, core-space and collocation forms")
    ap.add_argument("--batch", type=int, default=4, choices=[1, 2, 4, 8, 16],
                    help="cfg4: targets per step (batch of the 128-target block, all 1,842 sources)")
    ap.add_argument("--side-steps", type=int, default=3,
                    help="cfg4: timed batches of the FP64 and split-bf16 legs (the FP32 leg times --steps)")
    ap.add_argument("--no-tune", action="store_true", help="use the default launch shapes")
    ap.add_argument("--retune", action="store_true",
                    help="search launch shapes live (before the timed region) and write them to the cache file")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-single-seconds", type=float, default=8.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one elementwise kernel that reads and writes 512 MiB (reference for "
                         "the HBM byte counters)")
    ap.add_argument("--legs", default="f32,f64,bf16x3,bf16x6", help="compute forms to time (comma separated)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}, "
              f"WORLD_SIZE {world}", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2401_04189_amd import txe, workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    if args.config == "cfg5":
        bench_batched(args, txe, torch, W)
        return
    if args.config == "cfg4":
        bench_block(args, txe, torch, W)
        return
    if args.config == "fe5":
        bench_fe(args, txe, torch, W)
        return
    s = W.build_config(args.config)
    n, r, K, N = s.grid.n, s.r, s.K, s.N
    symmetric = True
    npairs = N * (N + 1) // 2
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    vx = torch.empty_like(psi)

    if args.copy_calibration:
        copy_calibration(torch)

    legs = {}
    tuned = {}
    load_cache(args, txe, ctx)
    for compute in args.legs.split(","):
        tuned[compute] = shapes(args, txe, ctx, sysm, psi, compute)
        wall, ex, kt = time_leg(txe, torch, ctx, sysm, psi, vx, compute, args.steps, args.warmup, symmetric, 0, N)
        legs[compute] = {"wall": wall, "ex": ex, "kt": kt}
    if "f32" not in legs or "f64" not in legs:
        print(json.dumps({k: {"ms_per_step": 1e3 * v["wall"] / args.steps, "E_x": v["ex"]} for k, v in legs.items()}))
        return
    dex = abs(legs["f32"]["ex"] - legs["f64"]["ex"])
    use = "f32" if dex <= 1e-5 else "f64"
    L = legs[use]
    ms = 1e3 * L["wall"] / args.steps
    value = npairs / (ms / 1e3)
    fp64_ms = 1e3 * legs["f64"]["wall"] / args.steps
    fp32_ms = 1e3 * legs["f32"]["wall"] / args.steps

    core_ms, core_n = L["kt"]["core"]
    per_launch_ms = core_ms / max(core_n, 1)
    achieved = core_kernel_flops_per_pair(n, r, K) * npairs / (per_launch_ms * 1e-3) / 1e12
    peak = PEAK_TFLOPS[use]
    measured = ctx.ceiling(use)  # this device's MFMA rate for the same dtype (microbenchmark)
    roof = {"bound": "mfma", "kernel": "core", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": load_traffic(use, args.config),
            "launch_ms": round(per_launch_ms, 4), "measured_peak": round(measured, 1),
            "frac_of_measured": round(achieved / measured, 4)}

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "pair-convolutions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": use,
        "data": "synthetic",
        "config": {"workload": W.WORKLOAD_NAMES[args.config], "grid": list(n), "orbitals": N, "pairs": npairs,
                   "rank": list(r), "terms": K, "mode": "symmetric unique pairs"},
        "fp64": {"value": round(npairs / (fp64_ms / 1e3), 1), "ms_per_step": round(fp64_ms, 4),
                 "E_x": legs["f64"]["ex"],
                 "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in legs["f64"]["kt"].items()}},
        "fp32": {"value": round(npairs / (fp32_ms / 1e3), 1), "ms_per_step": round(fp32_ms, 4),
                 "E_x": legs["f32"]["ex"],
                 "kernel_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in legs["f32"]["kt"].items()}},
        "fp32_over_fp64": round(fp64_ms / fp32_ms, 3),
        "split_bf16": {c: {"value": round(npairs / (1e3 * legs[c]["wall"] / args.steps / 1e3), 1),
                           "ms_per_step": round(1e3 * legs[c]["wall"] / args.steps, 4),
                           "over_fp64": round(fp64_ms / (1e3 * legs[c]["wall"] / args.steps), 3),
                           "dE_x_vs_fp64_Ha": abs(legs[c]["ex"] - legs["f64"]["ex"]),
                           "within_1e-5_Ha": abs(legs[c]["ex"] - legs["f64"]["ex"]) <= 1e-5,
                           "core_ms": round(legs[c]["kt"]["core"][0] / max(legs[c]["kt"]["core"][1], 1), 4)}
                       for c in legs if c.startswith("bf16")},
        "dE_x_fp32_vs_fp64_Ha": dex,
        "whole_path_tflops": round(flops_per_pair(n, r, K) * npairs / (ms / 1e3) / 1e12, 3),
        "roofline": roof,
        "launch_shapes": tuned,
        "measured_ceilings": {"f64_mfma_tflops": round(ctx.ceiling("f64"), 1),
                              "f32_mfma_tflops": round(ctx.ceiling("f32"), 1),
                              "bf16_mfma_tflops": round(ctx.ceiling("bf16"), 1),
                              "hbm_stream_gbs": round(ctx.ceiling("hbm"), 1)},
    }
    out["ace"] = bench_ace(txe, torch, ctx, sysm, psi, vx, args)
    if args.retune:
        txe.tune_save(ctx, TUNE_CACHE)
    sysm.close()
    ctx.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(s, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
