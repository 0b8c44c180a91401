"""The 128^3 block workload at full size (1,842 orbitals on 310 rutile sites,
r = 80, K = 50, block mode), in the launch configuration bench.py times: a
batch of 4 targets (orbitals 0..3) against all 1,842 sources, launch shapes
from the committed cache when it has them.

The whole 128 x 1,842 block is 235,776 pairs (hours for the oracle), so FP64
parity is checked on samples the oracle computes one by one:
  * 64 pair energies e_ij of the batch: the four diagonal pairs, for each
    target its nearest (largest e_ij) and farthest (smallest) sources, and
    random sources;
  * Vx psi of orbital 0 against a 64-source subset, computed whole by both;
and through properties that hold at any size: E_batch = -1/2 sum of the
batch's pair energies, and the library's exchange-matrix diagonal
= -sum_j e_ij.  The reduced forms (FP32 MFMA, split bf16 x3 and x6) are
checked against FP64 on the same batch: |dE_batch| <= 1e-5 Ha, the Vx psi
bar of each form, the diagonal to 1e-5 Ha.  Orbitals and bases are
generated on the GPU (30.9 GB of orbitals).
"""
import os

import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

BATCH = 4
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2401_04189_amd",
                     "tuned_shapes.json")


@pytest.fixture(scope="module")
def big():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = W.build_config("cfg4", device="cuda")
    torch.cuda.empty_cache()
    print(f"generated: {s.meta}", flush=True)
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    if os.path.exists(CACHE):
        txe.tune_load(ctx, CACHE)
    st = O.Setup(s.grid.x, s.grid.q, s.U, s.w, s.alpha)
    out = {}
    for comp in ("f64", "f32", "bf16x3", "bf16x6"):
        vx, ex, ep, eo = txe.apply(ctx, sysm, s.psi, compute=comp, symmetric=False, i0=0, Ni=BATCH,
                                   want_pairs=True, want_orb=True)
        torch.cuda.synchronize()
        out[comp] = (vx, float(ex), ep.cpu().numpy(), eo.cpu().numpy())
        print(f"{comp}: E_batch {float(ex):.12f}", flush=True)
    yield s, ctx, sysm, st, out
    sysm.close()
    ctx.close()


def test_sampled_pair_energies_f64(big):
    s, ctx, sysm, st, out = big
    N = s.N
    _, ex, ep, eo = out["f64"]
    rng = np.random.default_rng(7)
    picks = [(t, t) for t in range(BATCH)]
    for t in range(BATCH):
        row = ep[t * N:(t + 1) * N].copy()
        row[t] = np.nan
        order = np.argsort(np.nan_to_num(row, nan=-1.0))
        picks += [(t, int(j)) for j in order[-4:][::-1]]                 # nearest: largest e_tj
        picks += [(t, int(j)) for j in order[:4] if j != t]              # farthest: smallest e_tj
    while len(picks) < 64:
        t, j = int(rng.integers(0, BATCH)), int(rng.integers(0, N))
        if (t, j) not in picks:
            picks.append((t, j))
    worst = 0.0
    for (t, j) in picks:
        pi = s.psi[t].double().cpu().numpy()
        pj = s.psi[j].double().cpu().numpy()
        ref = O.pair(pi, pj, st)[1]
        got = ep[t * N + j]
        rel = abs(got - ref) / abs(ref)
        worst = max(worst, rel)
        assert rel <= 1e-9, f"e[{t},{j}] gpu {got:.15e} oracle {ref:.15e} rel {rel:.2e}"
    print(f"{len(picks)} sampled e_ij (e from {min(abs(ep)):.2e} to {max(abs(ep)):.2e}): worst relative error "
          f"{worst:.2e}", flush=True)
    # properties at full size: E_batch and the diagonal from the batch's pair energies
    assert abs(ex + 0.5 * ep.sum()) <= 1e-12 * abs(ex)
    diag = -ep.reshape(BATCH, N).sum(axis=1)
    assert np.abs(eo - diag).max() <= 1e-12 * np.abs(diag).max()


def test_one_target_vx_against_subset_f64(big):
    s, ctx, sysm, st, out = big
    idx = [0] + list(range(7, 1842, 29))[:63]
    sub = s.psi[idx].contiguous()
    vx, ex, _ = txe.apply(ctx, sysm, sub, compute="f64", symmetric=False, i0=0, Ni=1)
    p = sub.double().cpu().numpy()
    ref = O.apply_target(p, st, 0)
    got = vx[0].cpu().numpy()
    w3 = O.weights3d(st.q)
    rel = np.sqrt((w3 * (got - ref) ** 2).sum() / (w3 * ref ** 2).sum())
    print(f"Vx psi_0 over {len(idx)} sources: W-relative error {rel:.3e}", flush=True)
    assert rel <= 1e-9


@pytest.mark.parametrize("comp,vtol", [("f32", 1e-5), ("bf16x6", 1e-5), ("bf16x3", 2e-4)])
def test_reduced_precision_against_f64_batch(big, comp, vtol):
    s, ctx, sysm, st, out = big
    v64, e64, p64, d64 = out["f64"]
    v, e, p, d = out[comp]
    w3 = torch.as_tensor(O.weights3d(st.q), device="cuda")
    num = ((v - v64) ** 2 * w3).sum(dim=(1, 2, 3))
    den = (v64 ** 2 * w3).sum(dim=(1, 2, 3))
    rel = float(torch.sqrt(num / den).max())
    dE = abs(e - e64)
    dd = float(np.abs(d - d64).max())
    prel = float(np.abs(p - p64).max() / np.abs(p64).max())
    print(f"{comp}, {BATCH} targets x {s.N} sources: E_batch f64 {e64:.10f} {comp} {e:.10f} |dE| {dE:.3e} Ha, "
          f"Vx relative (W-norm, worst orbital) {rel:.3e}, diagonal {dd:.3e} Ha, e_ij {prel:.3e}", flush=True)
    assert dE <= 1e-5 and rel <= vtol and dd <= 1e-5
