"""The allocation-free entry point (txe_apply_noalloc, a fixed per-GPU scratch
array) against txe_apply on the same inputs, through the C ABI: two calls in
a row, the second with a smaller input, in FP64 (bitwise: the chunked plan
adds every target's sources in the same order) and FP32 (|dE_x| <= 1e-5 Ha,
Vx psi to 1e-5 relative in the W-norm), symmetric and block mode, and a
problem whose one-chunk workspace exceeds the scratch (it runs chunked)."""
import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


def wrel(a, b, q):
    w3 = torch.as_tensor(O.weights3d(q), device=a.device)
    num = ((a.double() - b.double()) ** 2 * w3).sum(dim=(1, 2, 3))
    den = (b.double() ** 2 * w3).sum(dim=(1, 2, 3))
    return float(torch.sqrt(num / den).max())


@pytest.mark.parametrize("mode", ["symmetric", "block"])
def test_noalloc_matches_apply_twice(ctx, mode):
    big = W.small_system(n=48, L=6.0, N=10, r=24, K=12, seed=61)
    small = W.small_system(n=20, L=5.0, N=4, r=9, K=8, seed=62)
    for s in (big, small):   # two calls in a row, the second smaller
        sysm = txe.System.from_workload(ctx, s)
        psi = s.psi.cuda()
        sym = mode == "symmetric"
        i0, Ni = (0, s.N) if sym else (1, s.N - 2)
        for comp in ("f64", "f32"):
            kw = dict(compute=comp, symmetric=sym, i0=i0, Ni=Ni, want_pairs=True, want_orb=True)
            ref = txe.apply(ctx, sysm, psi, **kw)
            got = txe.apply_noalloc(ctx, sysm, psi, **kw)
            torch.cuda.synchronize()
            dE = abs(float(got[1]) - float(ref[1]))
            rel = wrel(got[0], ref[0], s.grid.q)
            print(f"[{mode} N={s.N} {comp}] |dE_x| {dE:.3e} Ha, Vx rel {rel:.3e}", flush=True)
            if comp == "f64":
                for a, b in zip(got, ref):
                    assert torch.equal(a, b)
            else:
                assert dE <= 1e-5 and rel <= 1e-5
                assert float((got[2] - ref[2]).abs().max()) <= 1e-5 * float(ref[2].abs().max())
        sysm.close()


def test_noalloc_runs_chunked_beyond_the_scratch(ctx):
    """64^3, r = 40, 24 orbitals: one chunk would need ~0.5 GiB of FP64
    workspace, above the scratch array, so the allocation-free apply runs in
    triangular and rectangular pair tiles; FP64 bitwise equal to txe_apply."""
    s = W.small_system(n=64, L=10.0, N=24, r=40, K=10, seed=63)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    need = txe.workspace_bytes(ctx, sysm, psi, compute="f64")
    print(f"one-chunk workspace {need / 2**20:.0f} MiB", flush=True)
    assert need > 512 << 20
    ref = txe.apply(ctx, sysm, psi, compute="f64", want_pairs=True, want_orb=True)
    got = txe.apply_noalloc(ctx, sysm, psi, compute="f64", want_pairs=True, want_orb=True)
    torch.cuda.synchronize()
    for a, b in zip(got, ref):
        assert torch.equal(a, b)
    sysm.close()


def test_noalloc_rejects_what_cannot_fit_the_scratch(ctx):
    """12,000 orbitals on a 4^3 grid, symmetric: the pair energies alone
    (72 million FP64 values) exceed the scratch array, so the apply is
    refused with TXE_ERR_NOMEM and a clear message, nothing enqueued."""
    g = W.uniform_grid(4, 2.0)
    sysm = txe.System(ctx, g.x, g.q, W.full_rank_bases(g, 1), np.array([1.0]), np.array([0.5]))
    psi = torch.zeros((12000, 4, 4, 4), dtype=torch.float64, device="cuda")
    vx = torch.full_like(psi, 3.0)
    with pytest.raises(txe.TxeError) as ei:
        txe.apply_noalloc(ctx, sysm, psi, compute="f64", vx_out=vx)
    torch.cuda.synchronize()
    print(f"{ei.value}", flush=True)
    assert ei.value.status == 3 and "scratch" in str(ei.value)
    assert bool((vx == 3.0).all())
    sysm.close()
