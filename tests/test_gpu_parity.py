"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle on
the same seeded inputs.

FP64 bar (both from the method's own tolerances): |dE_x|/|E_x| <= 1e-9 and
max_i ||dVx psi_i||_W / ||Vx psi_i||_W <= 1e-9; pair energies e_ij to 1e-9
of the largest.  Reduced precision (FP32 MFMA, split bf16) against the GPU
FP64 path: |dE_x| <= 1e-5 Ha absolute (the reduced-precision gate) for every
form; Vx psi and e_ij relative errors at 1e-5 (FP32, bf16 x6) or 2e-4 (bf16
x3, whose products keep ~16 bits per operand).
"""
import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

TOL64 = 1e-9
GATE_HA = 1e-5   # reduced precision: |dE_x| against the GPU FP64 path


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


def wnorm(v, q):
    w3 = O.weights3d(q)
    return np.sqrt((v * v * w3[None]).sum(axis=(1, 2, 3)))


def rel_vx_err(vx, ref, q):
    return float((wnorm(vx - ref, q) / wnorm(ref, q)).max())


def run_gpu(ctx, s, compute="f64", symmetric=True, i0=0, Ni=None, psi_dtype=torch.float64, **kw):
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.to(device="cuda", dtype=psi_dtype).contiguous()
    vx, ex, ep = txe.apply(ctx, sysm, psi, compute=compute, symmetric=symmetric, i0=i0, Ni=Ni,
                           want_pairs=True, **kw)
    torch.cuda.synchronize()
    out = (None if vx is None else vx.double().cpu().numpy(), float(ex.item()), ep.cpu().numpy())
    sysm.close()
    return out


def oracle_pairs_vector(pairs, N, symmetric, i0=0, Ni=None):
    if symmetric:
        return np.array([pairs[(i, j)] for i in range(N) for j in range(i, N)])
    return np.array([pairs[(i0 + t, j)] for t in range(Ni) for j in range(N)])


def check_f64(ctx, s, symmetric=True, i0=0, Ni=None, label=""):
    st = O.Setup.from_system(s)
    psi = s.psi.numpy()
    pairs = {}
    vref, eref = O.apply(psi, st, mode="symmetric" if symmetric else "block", i0=i0, Ni=Ni, pairs_out=pairs)
    vx, ex, ep = run_gpu(ctx, s, "f64", symmetric, i0, Ni)
    epref = oracle_pairs_vector(pairs, s.N, symmetric, i0, Ni)
    e_err = np.abs(ep - epref).max() / np.abs(epref).max()
    ex_err = abs(ex - eref) / abs(eref)
    vx_err = rel_vx_err(vx, vref, st.q)
    print(f"[{label}] e_ij rel {e_err:.3e}  E_x {ex:.12f} vs {eref:.12f} rel {ex_err:.3e}  Vx rel {vx_err:.3e}",
          flush=True)
    assert e_err <= TOL64
    assert ex_err <= TOL64
    assert vx_err <= TOL64


def test_library_setup_tables_match_oracle(ctx):
    s = W.small_system(n=16, L=5.0, N=2, r=6, K=8, seed=31)
    st = O.Setup.from_system(s)
    sysm = txe.System.from_workload(ctx, s)
    for d in range(3):
        C, Ch = sysm.conv(d)
        assert np.abs(C - st.C[d]).max() <= 1e-13
        assert np.abs(Ch - st.Chat[d]).max() <= 1e-12 * np.abs(st.Chat[d]).max()
    sysm.close()


def test_f64_tiny_symmetric(ctx):
    check_f64(ctx, W.small_system(n=16, L=5.0, N=3, r=6, K=8, seed=31), label="n16 r6")


def test_f64_ragged_ranks_and_grid(ctx):
    """Ranks and grid sizes that are not multiples of 16 (padded tails)."""
    check_f64(ctx, W.small_system(n=20, L=5.0, N=4, r=11, K=9, seed=32), label="n20 r11")


def test_f64_non_cubic(ctx):
    g = W.uniform_grid((16, 20, 24), (4.0, 5.0, 6.0))
    psi, _ = W.make_orbitals(g, 3, 3, (0.5, 2.0), seed=33, box=1.5)
    U = W.hosvd_bases(psi, g, (5, 7, 9))
    w, a = W.exp_sum(10)
    s = W.System(name="noncubic", grid=g, psi=psi, U=U, w=w, alpha=a)
    check_f64(ctx, s, label="non-cubic")


def test_f64_full_rank(ctx):
    """r = n: the Tucker projector is the identity (dense-kernel case)."""
    check_f64(ctx, W.small_system(n=16, L=5.0, N=2, r=16, K=6, bases="full", seed=34), label="full rank")


def test_f64_cfg1(ctx):
    check_f64(ctx, W.build_config("cfg1"), label="24^3 N=4 r=16 K=30")


def test_f64_rank_tiles(ctx):
    """Ranks spanning 2..5 tiles of 16 (every core-kernel variant)."""
    for r in (20, 40, 48, 60, 70):
        s = W.small_system(n=(max(24, r) + 3) // 4 * 4, L=6.0, N=2, r=r, K=10, seed=35)
        check_f64(ctx, s, label=f"r={r}")


def test_f32_rank_tiles_against_f64(ctx):
    """Every FP32 core-kernel variant (2..5 rank tiles) against the GPU FP64 path."""
    # K = 10 gives fewer steps per slab than LDS slab chunks at 3..5 tiles;
    # K = 24 at 4 tiles gives more
    for r, K in ((20, 10), (40, 10), (48, 10), (60, 10), (60, 24), (70, 10)):
        s = W.small_system(n=(max(24, r) + 3) // 4 * 4, L=6.0, N=2, r=r, K=K, seed=35)
        v64, e64, p64 = run_gpu(ctx, s, "f64")
        v32, e32, p32 = run_gpu(ctx, s, "f32")
        verr = rel_vx_err(v32, v64, s.grid.q)
        perr = np.abs(p32 - p64).max() / np.abs(p64).max()
        print(f"[f32 r={r}] |dE_x| {abs(e32 - e64):.3e} Ha  e_ij rel {perr:.3e}  Vx rel {verr:.3e}", flush=True)
        assert abs(e32 - e64) <= GATE_HA and perr <= 1e-5 and verr <= 1e-5


# per-mode ranks: the tile count follows the largest rank, the live chunks
# of the last tile follow modes 1 and 2 (one, three and four of four live);
# odd r0 gives the term-major cores an odd number of slab steps per group
ANISO = ((40, 20, 20), (20, 36, 44), (44, 44, 18), (18, 30, 48), (33, 40, 40), (21, 24, 24))


def test_f64_anisotropic_ranks(ctx):
    for r in ANISO:
        s = W.small_system(n=48, L=6.0, N=2, r=r, K=10, seed=41)
        check_f64(ctx, s, label=f"r={r}")


def test_f32_anisotropic_ranks_against_f64(ctx):
    for r in ANISO:
        s = W.small_system(n=48, L=6.0, N=2, r=r, K=10, seed=41)
        v64, e64, p64 = run_gpu(ctx, s, "f64")
        v32, e32, p32 = run_gpu(ctx, s, "f32")
        verr = rel_vx_err(v32, v64, s.grid.q)
        perr = np.abs(p32 - p64).max() / np.abs(p64).max()
        print(f"[f32 r={r}] |dE_x| {abs(e32 - e64):.3e} Ha  e_ij rel {perr:.3e}  Vx rel {verr:.3e}", flush=True)
        assert abs(e32 - e64) <= GATE_HA and perr <= 1e-5 and verr <= 1e-5
        vb, eb, pb = run_gpu(ctx, s, "bf16x3")
        verr = rel_vx_err(vb, v64, s.grid.q)
        perr = np.abs(pb - p64).max() / np.abs(p64).max()
        print(f"[bf16x3 r={r}] |dE_x| {abs(eb - e64):.3e} Ha  e_ij rel {perr:.3e}  Vx rel {verr:.3e}", flush=True)
        assert abs(eb - e64) <= GATE_HA and perr <= 2e-4 and verr <= 2e-4


@pytest.mark.parametrize("form,tol", [("bf16x6", 1e-5), ("bf16x3", 2e-4)])
def test_bf16_split_against_f64(ctx, form, tol):
    """Split-bf16 core kernel sums (three- or two-part operands) against the
    GPU FP64 path, every rank-tile variant.  The three-product form keeps
    ~16 bits per operand (2^-16 relative per product), the six-product form
    ~24 (FP32 level)."""
    for r in (20, 40, 48, 60, 70):
        s = W.small_system(n=(max(24, r) + 3) // 4 * 4, L=6.0, N=2, r=r, K=10, seed=35)
        v64, e64, p64 = run_gpu(ctx, s, "f64")
        vb, eb, pb = run_gpu(ctx, s, form)
        verr = rel_vx_err(vb, v64, s.grid.q)
        perr = np.abs(pb - p64).max() / np.abs(p64).max()
        print(f"[{form} r={r}] |dE_x| {abs(eb - e64):.3e} Ha (of {abs(e64):.3f})  e_ij rel {perr:.3e}  "
              f"Vx rel {verr:.3e}", flush=True)
        assert abs(eb - e64) <= GATE_HA and perr <= tol and verr <= tol


def test_f32_block_chunked(ctx, monkeypatch):
    """Block mode split into several target chunks (forced by a small
    workspace limit) gives the same result as one chunk, in both precisions."""
    s = W.small_system(n=16, L=5.0, N=6, r=7, K=8, seed=40)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    full = {c: txe.apply(ctx, sysm, psi, compute=c, symmetric=False, i0=1, Ni=4,
                         want_pairs=True) for c in ("f64", "f32")}
    need = txe.workspace_bytes(ctx, sysm, psi, symmetric=False, i0=1, Ni=4)
    monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(need // 3))
    for c in ("f64", "f32"):
        vx, ex, ep = txe.apply(ctx, sysm, psi, compute=c, symmetric=False, i0=1, Ni=4, want_pairs=True)
        torch.cuda.synchronize()
        assert torch.equal(vx, full[c][0]) and torch.equal(ep, full[c][2])
        assert float(ex) == float(full[c][1])
    monkeypatch.delenv("TXE_TEST_MAX_WORKSPACE")
    sysm.close()


@pytest.mark.parametrize("comp", ["f64", "f32", "bf16x3"])
def test_symmetric_chunked_bitwise(ctx, monkeypatch, comp):
    """Symmetric mode split into triangular and rectangular pair tiles (forced
    by small workspace limits: 3 and 6 orbital blocks) adds every target's
    sources in the same order as one chunk, so Vx psi (also scaled and
    weighted), E_x, the pair energies and the exchange-matrix diagonal are
    bitwise those of one chunk."""
    s = W.small_system(n=16, L=5.0, N=11, r=7, K=8, seed=42)
    sysm = txe.System.from_workload(ctx, s)
    # reduced forms on FP32 orbitals: with FP64 orbitals a small limit also
    # drops the FP32 orbital copy, which rounds the pair densities differently
    psi = s.psi.cuda() if comp == "f64" else s.psi.cuda().float()
    scale = torch.tensor(-1.75, dtype=torch.float64, device="cuda")
    kw = dict(compute=comp, want_pairs=True, want_orb=True)
    one = txe.apply(ctx, sysm, psi, **kw)
    onew = txe.apply(ctx, sysm, psi, out_scale=scale, out_weighted=True, **kw)
    torch.cuda.synchronize()
    need = txe.workspace_bytes(ctx, sysm, psi, compute=comp)
    for frac in (6, 25):
        monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(need // frac))
        for ref, extra in ((one, {}), (onew, dict(out_scale=scale, out_weighted=True))):
            got = txe.apply(ctx, sysm, psi, **kw, **extra)
            torch.cuda.synchronize()
            for a, b in zip(got, ref):
                assert torch.equal(a, b), f"limit need/{frac}"
        monkeypatch.delenv("TXE_TEST_MAX_WORKSPACE")
    sysm.close()


def test_block_source_chunks_bitwise(ctx, monkeypatch):
    """Block mode where one target against all sources exceeds the workspace:
    one target at a time against ascending source chunks, bitwise equal to
    one chunk in both precisions."""
    s = W.small_system(n=16, L=5.0, N=9, r=7, K=8, seed=43)
    sysm = txe.System.from_workload(ctx, s)
    for comp in ("f64", "f32"):
        psi = s.psi.cuda() if comp == "f64" else s.psi.cuda().float()
        ref = txe.apply(ctx, sysm, psi, compute=comp, symmetric=False, i0=2, Ni=5, want_pairs=True, want_orb=True)
        torch.cuda.synchronize()
        # room for about three pairs: fewer than the nine sources of one target
        full = txe.workspace_bytes(ctx, sysm, psi, compute=comp, symmetric=False, i0=2, Ni=5)
        monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(full // 14))
        got = txe.apply(ctx, sysm, psi, compute=comp, symmetric=False, i0=2, Ni=5, want_pairs=True, want_orb=True)
        torch.cuda.synchronize()
        monkeypatch.delenv("TXE_TEST_MAX_WORKSPACE")
        for a, b in zip(got, ref):
            assert torch.equal(a, b), comp
    sysm.close()


def test_f64_block_mode(ctx):
    s = W.small_system(n=16, L=5.0, N=5, r=7, K=8, seed=36)
    check_f64(ctx, s, symmetric=False, i0=1, Ni=3, label="block 1..3")


def test_constant_kernel_limit_gpu(ctx):
    """K = 1, alpha = 0, w = 1, full rank: Vx psi_i = -psi_i and E_x = -N/2."""
    g = W.uniform_grid(16, 4.0)
    psi, _ = W.make_orbitals(g, 3, 3, (0.5, 2.0), seed=8, box=1.0)
    s = W.System(name="const", grid=g, psi=psi, U=W.full_rank_bases(g, 2), w=np.array([1.0]),
                 alpha=np.array([0.0]))
    vx, ex, _ = run_gpu(ctx, s)
    p = psi.numpy()
    assert np.abs(vx + p).max() <= 1e-11 * np.abs(p).max()
    assert abs(ex + 1.5) <= 1e-11


def test_energy_only_and_scaled_weighted_output(ctx):
    s = W.small_system(n=16, L=5.0, N=3, r=6, K=8, seed=37)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    vx, ex, _ = txe.apply(ctx, sysm, psi)
    _, ex2, _ = txe.apply(ctx, sysm, psi, want_vx=False)
    scale = torch.tensor(2.5, dtype=torch.float64, device="cuda")
    vxw, ex3, _ = txe.apply(ctx, sysm, psi, out_scale=scale, out_weighted=True)
    torch.cuda.synchronize()
    w3 = torch.as_tensor(O.weights3d(s.grid.q), device="cuda")
    assert float(ex2) == float(ex) == float(ex3)
    assert torch.abs(vxw - 2.5 * w3 * vx).max().item() <= 1e-14 * torch.abs(vxw).max().item()
    sysm.close()


def test_deterministic_bitwise(ctx):
    s = W.small_system(n=20, L=5.0, N=4, r=9, K=8, seed=38)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    a = txe.apply(ctx, sysm, psi, want_pairs=True)
    b = txe.apply(ctx, sysm, psi, want_pairs=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and torch.equal(a[2], b[2])
    sysm.close()


def test_f32_against_f64(ctx):
    s = W.build_config("cfg1")
    v64, e64, p64 = run_gpu(ctx, s, "f64")
    for dt in (torch.float64, torch.float32):
        v32, e32, p32 = run_gpu(ctx, s, "f32", psi_dtype=dt)
        verr = rel_vx_err(v32, v64, s.grid.q)
        print(f"[f32 psi {dt}] |dE_x| {abs(e32 - e64):.3e} Ha  Vx rel {verr:.3e}", flush=True)
        assert abs(e32 - e64) <= 1e-5
        assert verr <= 1e-5


def test_validation_errors(ctx):
    s = W.small_system(n=16, L=5.0, N=2, r=6, K=8, seed=39)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    with pytest.raises(txe.TxeError):
        txe.apply(ctx, sysm, psi.float(), compute="f64")         # FP64 compute needs FP64 orbitals
    with pytest.raises(txe.TxeError):
        txe.apply(ctx, sysm, psi, symmetric=False, i0=1, Ni=5)   # block outside [0, N)
    bad = [u.copy() for u in s.U]
    bad[1] *= 1.001
    with pytest.raises(txe.TxeError):
        txe.System(ctx, s.grid.x, s.grid.q, bad, s.w, s.alpha)   # U not q-orthonormal
    with pytest.raises(txe.TxeError):
        txe.System(ctx, s.grid.x, s.grid.q, s.U, s.w, -np.abs(s.alpha))
    sysm.close()
