"""The 128^3 block workload at full size (1,842 orbitals on 310 rutile sites,
r = 80, K = 50, block mode): sampled parity of the FP64 path against the CPU
oracle, and the FP32 path against FP64.

The full 128 x 1,842 block is 235,776 pairs (hours for the oracle), so:
  * pair energies e_ij of sampled pairs (two targets against all sources on
    the GPU; six of those pairs recomputed by the oracle);
  * Vx psi of one target against a 16-source subset, computed whole by both;
  * FP32 against FP64 for a 4-target block against all sources
    (7,368 pairs): |dE_block| and the Vx psi relative error.
Orbitals and bases are generated on the GPU (30.9 GB of orbitals).
"""
import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = W.build_config("cfg4", device="cuda")
    torch.cuda.empty_cache()
    print(f"generated: {s.meta}", flush=True)
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    st = O.Setup(s.grid.x, s.grid.q, s.U, s.w, s.alpha)
    yield s, ctx, sysm, st
    sysm.close()
    ctx.close()


def test_sampled_pair_energies_f64(big):
    s, ctx, sysm, st = big
    N = s.N
    _, ex, ep = txe.apply(ctx, sysm, s.psi, compute="f64", symmetric=False, i0=0, Ni=2, want_vx=False,
                          want_pairs=True)
    ep = ep.cpu().numpy()
    rng = np.random.default_rng(7)
    picks = [(0, 0), (1, 1), (0, 1)] + [(int(t), int(j)) for t, j in zip(rng.integers(0, 2, 3),
                                                                          rng.integers(2, N, 3))]
    for (t, j) in picks:
        pi = s.psi[t].double().cpu().numpy()
        pj = s.psi[j].double().cpu().numpy()
        ref = O.pair(pi, pj, st)[1]
        got = ep[t * N + j]
        print(f"e[{t},{j}] gpu {got:.15e} oracle {ref:.15e} rel {abs(got - ref) / abs(ref):.2e}", flush=True)
        assert abs(got - ref) <= 1e-9 * abs(ref)
    assert abs(float(ex) + 0.5 * ep.sum()) <= 1e-12 * abs(float(ex))


def test_one_target_vx_against_subset_f64(big):
    s, ctx, sysm, st = big
    idx = [5] + list(range(100, 1842, 109))[:16]
    sub = s.psi[idx].contiguous()
    vx, ex, _ = txe.apply(ctx, sysm, sub, compute="f64", symmetric=False, i0=0, Ni=1)
    p = sub.double().cpu().numpy()
    ref = O.apply_target(p, st, 0)
    got = vx[0].cpu().numpy()
    w3 = O.weights3d(st.q)
    rel = np.sqrt((w3 * (got - ref) ** 2).sum() / (w3 * ref ** 2).sum())
    print(f"Vx psi_5 over 17 sources: W-relative error {rel:.3e}", flush=True)
    assert rel <= 1e-9


def test_f32_against_f64_block(big):
    s, ctx, sysm, st = big
    v64, e64, _ = txe.apply(ctx, sysm, s.psi, compute="f64", symmetric=False, i0=0, Ni=4)
    v32, e32, _ = txe.apply(ctx, sysm, s.psi, compute="f32", symmetric=False, i0=0, Ni=4)
    torch.cuda.synchronize()
    dE = abs(float(e32) - float(e64))
    w3 = torch.as_tensor(O.weights3d(st.q), device="cuda")
    num = ((v32 - v64) ** 2 * w3).sum(dim=(1, 2, 3))
    den = (v64 ** 2 * w3).sum(dim=(1, 2, 3))
    rel = float(torch.sqrt(num / den).max())
    print(f"4 targets x 1842 sources: E_block f64 {float(e64):.10f} f32 {float(e32):.10f} |dE| {dE:.3e} Ha, "
          f"Vx relative (W-norm, worst orbital) {rel:.3e}", flush=True)
    assert dE <= 1e-5
    assert rel <= 1e-5
