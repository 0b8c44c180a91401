"""Parity on the benchmark workload itself (64^3, 64 orbitals, r = 40,
K = 40, 2,080 unique pairs) in the launch configuration bench.py times:
the committed launch-shape cache is loaded, and the test checks that every
compute form actually runs a cached shape.

  * FP64: Vx psi of one orbital (64 sources) and four sampled pair energies
    against the CPU oracle, 1e-9;
  * FP32 MFMA and split bf16 x3 / x6 against FP64: |dE_x| <= 1e-5 Ha and the
    Vx psi bar of each form.
"""
import os

import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2401_04189_amd",
                     "tuned_shapes.json")


@pytest.fixture(scope="module")
def bench(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = W.build_config("cfg2")
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    assert txe.tune_load(ctx, CACHE) > 0
    psi = s.psi.cuda()
    out = {}
    for comp in ("f64", "f32", "bf16x3", "bf16x6"):
        assert txe.plan(ctx, sysm, psi, comp)[1], f"{comp}: no cached launch shape for the bench workload"
        vx, ex, ep = txe.apply(ctx, sysm, psi, compute=comp, want_pairs=True)
        torch.cuda.synchronize()
        out[comp] = (vx.cpu().numpy(), float(ex), ep.cpu().numpy())
    yield s, out
    sysm.close()
    ctx.close()


def test_f64_against_oracle(bench):
    s, out = bench
    vx, ex, ep = out["f64"]
    st = O.Setup.from_system(s)
    p = s.psi.numpy()
    w3 = O.weights3d(st.q)
    ref = O.apply_target(p, st, 17)
    rel = np.sqrt((w3 * (vx[17] - ref) ** 2).sum() / (w3 * ref ** 2).sum())
    print(f"Vx psi_17 (64 sources): W-relative error {rel:.3e}", flush=True)
    assert rel <= 1e-9
    N = p.shape[0]
    for (i, j) in ((0, 0), (3, 40), (17, 63), (62, 63)):
        idx = i * N - i * (i - 1) // 2 + (j - i)
        e_ref = O.pair(p[i], p[j], st)[1]
        print(f"e[{i},{j}] gpu {ep[idx]:.15e} oracle {e_ref:.15e}", flush=True)
        assert abs(ep[idx] - e_ref) <= 1e-9 * abs(e_ref)
    assert abs(ex + 0.5 * (2 * ep.sum() - sum(ep[i * N - i * (i - 1) // 2] for i in range(N)))) <= 1e-12 * abs(ex)


@pytest.mark.parametrize("comp,vtol", [("f32", 1e-5), ("bf16x6", 1e-5), ("bf16x3", 2e-4)])
def test_reduced_precision_against_f64(bench, comp, vtol):
    s, out = bench
    v64, e64, _ = out["f64"]
    v, e, _ = out[comp]
    w3 = O.weights3d([np.asarray(q) for q in s.grid.q])
    num = np.sqrt((w3[None] * (v - v64) ** 2).sum(axis=(1, 2, 3)))
    den = np.sqrt((w3[None] * v64 ** 2).sum(axis=(1, 2, 3)))
    rel = float((num / den).max())
    print(f"{comp}: |dE_x| {abs(e - e64):.3e} Ha, Vx relative (W-norm, worst orbital) {rel:.3e}", flush=True)
    assert abs(e - e64) <= 1e-5 and rel <= vtol
