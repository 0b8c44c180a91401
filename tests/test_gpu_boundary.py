"""The C-ABI boundary on the GPU: output aliasing and alignment errors (nothing
enqueued, outputs untouched), the library's FP64 exchange-matrix diagonal
<psi_i, Vx psi_i>_W = -sum_j e_ij against the oracle, ordering of applies
issued from two streams on one context, and stream capture (TXE_ERR_STATE
when the workspace would have to grow; a captured apply replayed several
times with eager work in between, every replay checked against eager runs).
"""
import ctypes

import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

TXE_ERR_ARG, TXE_ERR_STATE = 1, 6


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


def raw_apply(ctx, sysm, a):
    return txe.lib().txe_apply(ctx.h, sysm.h, ctypes.byref(a))


def test_output_aliasing_and_alignment_rejected(ctx):
    s = W.small_system(n=16, L=5.0, N=3, r=6, K=8, seed=51)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    keep = psi.clone()
    vx = torch.full_like(psi, 7.0)
    ex = torch.full((), 7.0, dtype=torch.float64, device="cuda")
    ep = torch.full((6,), 7.0, dtype=torch.float64, device="cuda")
    eo = torch.full((3,), 7.0, dtype=torch.float64, device="cuda")
    cases = {
        "ex inside psi": dict(ex=psi.data_ptr() + 64),
        "ex inside vxpsi": dict(ex=vx.data_ptr()),
        "e_pairs over psi": dict(e_pairs=psi.data_ptr() + psi.numel() * 8 - 16),
        "e_orb over ex": dict(e_orb=ex.data_ptr()),
        "e_orb over e_pairs": dict(e_orb=ep.data_ptr() + 8),
        "misaligned ex": dict(ex=ex.data_ptr() + 4),
        "misaligned e_orb": dict(e_orb=eo.data_ptr() + 2),
    }
    for name, over in cases.items():
        a = txe.make_args(psi, "f64", True, vx=vx, ex=ex, e_pairs=ep, e_orb=eo)
        for k, v in over.items():
            setattr(a, k, v)
        st = raw_apply(ctx, sysm, a)
        print(f"{name}: status {st} ({txe.lib().txe_last_error().decode()})", flush=True)
        assert st == TXE_ERR_ARG, name
    torch.cuda.synchronize()
    # nothing was enqueued: inputs and outputs are untouched
    assert torch.equal(psi, keep)
    assert bool((vx == 7.0).all()) and float(ex) == 7.0 and bool((ep == 7.0).all()) and bool((eo == 7.0).all())
    sysm.close()


@pytest.mark.parametrize("mode", ["symmetric", "block"])
def test_exchange_diagonal_against_oracle(ctx, mode):
    s = W.small_system(n=20, L=5.0, N=5, r=9, K=10, seed=52)
    st = O.Setup.from_system(s)
    p = s.psi.numpy()
    sym = mode == "symmetric"
    i0, Ni = (0, 5) if sym else (1, 3)
    vref, eref = O.apply(p, st, mode=mode, i0=i0, Ni=Ni)
    w3 = O.weights3d(st.q)
    dref = np.einsum("tabc,tabc,abc->t", p[i0:i0 + Ni], vref, w3)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    out = {}
    for comp in ("f64", "f32", "bf16x3"):
        vx, ex, _, eo = txe.apply(ctx, sysm, psi, compute=comp, symmetric=sym, i0=i0, Ni=Ni, want_orb=True)
        torch.cuda.synchronize()
        out[comp] = (eo.cpu().numpy(), float(ex), vx)
    d64, e64, v64 = out["f64"]
    err = np.abs(d64 - dref).max() / np.abs(dref).max()
    print(f"[{mode}] diag f64 {d64} oracle {dref} rel {err:.2e}", flush=True)
    assert err <= 1e-9
    # trace identity: block energy = 1/2 sum of the diagonal entries in symmetric mode
    if sym:
        assert abs(0.5 * d64.sum() - e64) <= 1e-12 * abs(e64)
    # the diagonal from the library equals <psi_i, (Vx psi)_i>_W of its own output
    wt = torch.as_tensor(w3, device="cuda")
    own = (psi[i0:i0 + Ni] * v64 * wt).sum(dim=(1, 2, 3)).cpu().numpy()
    assert np.abs(own - d64).max() <= 1e-12 * np.abs(d64).max()
    for comp in ("f32", "bf16x3"):
        dd = np.abs(out[comp][0] - d64).max()
        print(f"[{mode}] {comp}: max |d<psi_i, Vx psi_i>| {dd:.2e} Ha", flush=True)
        assert dd <= 1e-5
    sysm.close()


def test_system_teardown_leaves_no_runtime_error(ctx):
    """Creating and destroying systems (every device table, the collocation
    tables included) frees each allocation once: a failed runtime call would
    stay as the thread's last error and be reported by the next launch check,
    torch's included."""
    for k in range(2):
        s = W.small_system(n=16, L=5.0, N=3, r=6, K=10, seed=54 + k)
        sysm = txe.System.from_workload(ctx, s)
        vx, ex, _ = txe.apply(ctx, sysm, s.psi.cuda(), compute="f64", form="collocation")
        torch.cuda.synchronize()
        sysm.close()
        y = torch.arange(64, device="cuda", dtype=torch.float64) + 1.0  # raises on a stale error
        torch.cuda.synchronize()
        assert float(y.sum()) == 64 * 65 / 2 and bool(torch.isfinite(vx).all())


def test_two_streams_on_one_context_are_ordered(ctx):
    s = W.small_system(n=48, L=6.0, N=8, r=24, K=20, seed=53)
    sysm = txe.System.from_workload(ctx, s)
    pa = s.psi.cuda()
    pb = torch.flip(pa, dims=(0,)).contiguous() * 0.5
    ra = txe.apply(ctx, sysm, pa, compute="f32")
    rb = txe.apply(ctx, sysm, pb, compute="f32")
    torch.cuda.synchronize()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    n0 = ctx.stream_changes()
    for _ in range(3):
        with torch.cuda.stream(s1):
            va, ea, _ = txe.apply(ctx, sysm, pa, compute="f32")
        with torch.cuda.stream(s2):
            vb, eb, _ = txe.apply(ctx, sysm, pb, compute="f32")
        torch.cuda.synchronize()
        assert torch.equal(va, ra[0]) and torch.equal(vb, rb[0])
        assert float(ea) == float(ra[1]) and float(eb) == float(rb[1])
    changes = ctx.stream_changes() - n0
    print(f"stream changes ordered by an event: {changes}", flush=True)
    assert changes >= 6
    ctx.set_stream(torch.cuda.current_stream())
    sysm.close()


def test_capture_needs_reserved_workspace_and_replays_match():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = W.small_system(n=20, L=5.0, N=4, r=9, K=8, seed=54)
    c = txe.Context(0)
    sysm = txe.System.from_workload(c, s)
    psi = s.psi.cuda()
    cs = torch.cuda.Stream()
    cs.wait_stream(torch.cuda.current_stream())
    # a fresh context has no workspace: inside a capture the apply must refuse
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cs):
        g.capture_begin()
        try:
            with pytest.raises(txe.TxeError) as ei:
                txe.apply(c, sysm, psi, compute="f32")
        finally:
            g.capture_end()
    print(f"inside capture without workspace: {ei.value}", flush=True)
    assert ei.value.status == TXE_ERR_STATE
    del g
    torch.cuda.synchronize()
    # with the workspace reserved first the same apply is captured
    c.set_stream(torch.cuda.current_stream())
    c.reserve(txe.workspace_bytes(c, sysm, psi, compute="f32"))
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(cs):
        g.capture_begin()
        vx, ex, _ = txe.apply(c, sysm, psi, compute="f32")
        g.capture_end()
    torch.cuda.synchronize()
    c.set_stream(torch.cuda.current_stream())
    rng = np.random.default_rng(3)
    for rep in range(3):
        # eager work between replays: change the inputs in place, run eagerly
        psi.mul_(float(rng.uniform(0.8, 1.2)))
        ve, ee, _ = txe.apply(c, sysm, psi, compute="f32")
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        print(f"replay {rep}: E_x {float(ex):.12f} eager {float(ee):.12f}", flush=True)
        assert torch.equal(vx, ve) and float(ex) == float(ee)
    del g
    sysm.close()
    c.close()


GUARD = 4096  # guard elements on each side of every output


def guarded(n, dtype, fill=0.0):
    """(whole buffer, middle view of n elements); the guards hold a sentinel."""
    buf = torch.full((n + 2 * GUARD,), -123456.75, dtype=dtype, device="cuda")
    mid = buf[GUARD:GUARD + n]
    mid.fill_(fill)
    return buf, mid


def guards_intact(buf, n):
    return bool((buf[:GUARD] == -123456.75).all()) and bool((buf[GUARD + n:] == -123456.75).all())


@pytest.mark.parametrize("variant", ["f64 sym", "f32 sym", "bf16x3 sym", "f64 block", "f32 block chunked",
                                     "f64 collocation", "f64 pair bases", "f64 sym chunked"])
def test_outputs_stay_inside_their_buffers(ctx, variant, monkeypatch):
    """Every output written through the ABI lands inside its own buffer: each
    sits between guard bands of a sentinel value, which must come back
    unchanged, and psi is read-only."""
    s = W.small_system(n=20, L=5.0, N=7, r=10, K=8, seed=52)
    sysm = txe.System.from_workload(ctx, s)
    comp = variant.split()[0]
    symmetric = "block" not in variant
    N = s.N
    i0, Ni = (0, N) if symmetric else (2, 4)
    ng = s.psi[0].numel()
    pbuf, pmid = guarded(N * ng, torch.float64)
    pmid.copy_(s.psi.reshape(-1).cuda())
    psi = pmid.view(s.psi.shape)
    keep = psi.clone()
    npairs = N * (N + 1) // 2 if symmetric else Ni * N
    vbuf, vmid = guarded(Ni * ng, torch.float64)
    xbuf, xmid = guarded(1, torch.float64)
    ebuf, emid = guarded(npairs, torch.float64)
    obuf, omid = guarded(Ni, torch.float64)
    if "chunked" in variant:
        monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(txe.workspace_bytes(ctx, sysm, psi) // 3))
    a = txe.make_args(psi, comp, symmetric, i0, Ni, vx=vmid.view((Ni,) + tuple(s.psi.shape[1:])), ex=xmid[0],
                      e_pairs=emid, e_orb=omid, pair_bases="pair bases" in variant,
                      form="collocation" if "collocation" in variant else "core")
    assert raw_apply(ctx, sysm, a) == 0, txe.lib().txe_last_error().decode()
    torch.cuda.synchronize()
    print(f"[{variant}] E_x {float(xmid[0]):.12f}", flush=True)
    for name, buf, n in (("psi", pbuf, N * ng), ("vxpsi", vbuf, Ni * ng), ("ex", xbuf, 1), ("e_pairs", ebuf, npairs),
                         ("e_orb", obuf, Ni)):
        assert guards_intact(buf, n), f"{variant}: write outside {name}"
    assert torch.equal(psi, keep)
    assert bool(torch.isfinite(vmid).all()) and bool(torch.isfinite(emid).all()) and float(xmid[0]) < 0
    sysm.close()
