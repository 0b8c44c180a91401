"""Batched applies, graph replays and the launch-shape tuner.

Six uneven systems (grids 16^3..40^3, 3..17 orbitals, ranks 8..32):
  * txe_apply_batched over 1 and 3 lanes is bitwise identical to separate
    txe_apply calls (FP64 and FP32), and one system is checked against the
    CPU oracle;
  * a captured graph, replayed three times with unrelated eager work and
    in-place changes of the orbitals between replays, matches eager
    batched applies of the same inputs bitwise at every replay;
  * the tuner keeps a valid shape, its cache survives save / load into a
    new context, every launch shape gives the default's results, and bad
    batches and caches are refused on the host.
"""
import json

import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

SPECS = [  # n, L, N, r, K
    (16, 5.0, 3, 8, 12),
    (24, 6.0, 7, 12, 16),
    (32, 8.0, 12, 16, 20),
    (20, 6.0, 5, 10, 8),
    (40, 9.0, 17, 32, 24),
    (28, 7.0, 9, 20, 16),
]


@pytest.fixture(scope="module")
def env():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ctx = txe.Context(0)
    systems = []
    for k, (n, L, N, r, K) in enumerate(SPECS):
        s = W.make_system(f"batch{k}", n, L, N, 4, (0.4, 2.5), r, K, seed=700 + k, box=0.4 * L)
        systems.append((s, txe.System.from_workload(ctx, s), s.psi.cuda()))
    yield ctx, systems
    for _, sysm, _ in systems:
        sysm.close()
    ctx.close()


def items_of(systems, dtype=torch.float64):
    return [(sysm, psi.to(dtype)) for _, sysm, psi in systems]


def separate(ctx, items, compute):
    return [txe.apply(ctx, sysm, psi, compute=compute, want_pairs=True) for sysm, psi in items]


def assert_same(got, ref):
    for k, ((v, e, p), (v0, e0, p0)) in enumerate(zip(got, ref)):
        assert torch.equal(v, v0), f"system {k}: Vx psi differs"
        assert torch.equal(e, e0), f"system {k}: E_x differs"
        assert torch.equal(p, p0), f"system {k}: pair energies differ"


@pytest.mark.parametrize("compute", ["f64", "f32"])
@pytest.mark.parametrize("lanes", [1, 3])
def test_batched_equals_separate(env, compute, lanes):
    ctx, systems = env
    items = items_of(systems, torch.float64 if compute == "f64" else torch.float32)
    print(f"batched {compute}, {len(items)} systems, {lanes} lanes", flush=True)
    ref = separate(ctx, items, compute)
    got = txe.apply_batched(ctx, items, compute=compute, lanes=lanes, want_pairs=True)
    torch.cuda.synchronize()
    assert_same(got, ref)


def test_batched_system_against_oracle(env):
    ctx, systems = env
    s, _, _ = systems[2]
    got = txe.apply_batched(ctx, items_of(systems), compute="f64", lanes=3)
    vx, ex, _ = got[2]
    st = O.Setup.from_system(s)
    ref_vx, ref_e = O.apply(s.psi.numpy(), st)
    e = float(ex)
    print(f"system 2: E_x gpu {e:.15e} oracle {ref_e:.15e}", flush=True)
    assert abs(e - ref_e) <= 1e-9 * abs(ref_e)
    w3 = O.weights3d(st.q)
    d = vx.cpu().numpy() - ref_vx
    rel = np.sqrt((d * d * w3).sum(axis=(1, 2, 3)) / (ref_vx * ref_vx * w3).sum(axis=(1, 2, 3))).max()
    assert rel <= 1e-9


@pytest.mark.parametrize("compute", ["f64", "f32"])
def test_graph_replays_match_eager(env, compute):
    ctx, systems = env
    dt = torch.float64 if compute == "f64" else torch.float32
    psis = [psi.to(dt).clone() for _, _, psi in systems]
    items = [(sysm, p) for (_, sysm, _), p in zip(systems, psis)]
    print(f"graph {compute}: capture", flush=True)
    g = txe.Graph(ctx, items, compute=compute, lanes=3, want_pairs=True)
    try:
        for rep in range(3):
            if rep > 0:  # change the inputs in place; the graph reads them at replay
                for p in psis:
                    p.mul_(1.0 + 0.25 * rep)
            # unrelated eager work on the same stream and context before the replay
            txe.apply(ctx, systems[0][1], systems[0][2].to(dt), compute=compute)
            junk = torch.randn(1 << 20, device="cuda").sum()
            g.launch()
            torch.cuda.synchronize()
            got = [tuple(t.clone() for t in o) for o in g.outputs]
            ref = txe.apply_batched(ctx, items, compute=compute, lanes=1, want_pairs=True)
            torch.cuda.synchronize()
            print(f"replay {rep}: E_x of system 4 = {float(got[4][1]):.12f} ({float(junk):.3f})", flush=True)
            assert_same(got, ref)
    finally:
        g.close()


def test_tuner_cache_roundtrip_and_shapes(env, tmp_path):
    ctx, systems = env
    _, sysm, psi = systems[4]
    knobs0, tuned0 = txe.plan(ctx, sysm, psi, "f64")
    assert knobs0 == dict(ngs_mul=1, proj_gt=4, back_ncg=0, grid_cap=2048, back_form=0) and not tuned0
    v0, e0, _ = txe.apply(ctx, sysm, psi, compute="f64")
    ms, knobs = txe.tune(ctx, sysm, psi, "f64", reps=2)
    print(f"tuned {knobs} at {ms:.3f} ms", flush=True)
    assert ms > 0
    assert knobs["ngs_mul"] in (1, 2, 4) and knobs["proj_gt"] in (1, 2, 3, 4)
    assert knobs["back_ncg"] in (0, 1, 2) and knobs["grid_cap"] in (1024, 2048, 4096)
    assert knobs["back_form"] in (0, 1, 2, 3)
    assert txe.plan(ctx, sysm, psi, "f64") == (knobs, True)
    v1, e1, _ = txe.apply(ctx, sysm, psi, compute="f64")
    assert abs(float(e1) - float(e0)) <= 1e-13 * abs(float(e0))
    assert float((v1 - v0).abs().max()) <= 1e-13 * float(v0.abs().max())

    path = tmp_path / "tune.json"
    txe.tune_save(ctx, path)
    cache = json.loads(path.read_text())
    assert len(cache) == 1
    ctx2 = txe.Context(0)
    try:
        sys2 = txe.System.from_workload(ctx2, systems[4][0])
        assert txe.tune_load(ctx2, path) == 1
        assert txe.plan(ctx2, sys2, psi, "f64") == (knobs, True)
        # every launch shape, forced through the cache, reproduces the default
        key = next(iter(cache))
        for shape in ([1, 1, 1, 1024, 1], [2, 3, 2, 256, 2], [4, 1, 2, 4096, 1], [1, 3, 0, 16384, 2],
                      [1, 2, 1, 2048, 2], [1, 2, 2, 2048, 1], [1, 4, 1, 2048, 2], [2, 4, 2, 512, 1]):
            ent = dict(zip(("ngs_mul", "proj_gt", "back_ncg", "grid_cap", "back_form"), shape))
            path.write_text(json.dumps({key: ent}))
            assert txe.tune_load(ctx2, path) == 1
            assert txe.plan(ctx2, sys2, psi, "f64")[0] == ent
            v, e, _ = txe.apply(ctx2, sys2, psi, compute="f64")
            torch.cuda.synchronize()
            print(f"shape {ent}: dE {abs(float(e) - float(e0)):.2e}", flush=True)
            assert abs(float(e) - float(e0)) <= 1e-13 * abs(float(e0))
            if ent["ngs_mul"] == 1:
                assert torch.equal(v, v0)
            else:
                assert float((v - v0).abs().max()) <= 1e-13 * float(v0.abs().max())
        sys2.close()
    finally:
        ctx2.close()


def test_bad_batches_and_caches_are_refused(env, tmp_path):
    ctx, systems = env
    items = items_of(systems[:2])
    sysarr, args, _ = txe._batch(items, "f64", True, False)
    # second system writes E_x over the first one's
    args[1].ex = args[0].ex
    with pytest.raises(txe.TxeError, match="overlap"):
        txe._check(txe.lib().txe_apply_batched(ctx.h, 2, sysarr, args, 2))
    with pytest.raises(txe.TxeError):
        txe._check(txe.lib().txe_apply_batched(ctx.h, 0, sysarr, args, 2))
    with pytest.raises(txe.TxeError):
        txe._check(txe.lib().txe_apply_batched(ctx.h, 2, sysarr, args, 17))
    bad = tmp_path / "bad.json"
    bad.write_text('{\n "k": {"ngs_mul": 3, "proj_gt": 2, "back_ncg": 0, "grid_cap": 2048}\n}\n')
    with pytest.raises(txe.TxeError, match="not a valid cache entry"):
        txe.tune_load(ctx, bad)
    bad.write_text('{\n "k": {"ngs_mul": 1}\n}\n')
    with pytest.raises(txe.TxeError):
        txe.tune_load(ctx, bad)
