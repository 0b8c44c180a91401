"""E_x as a torch.autograd.Function on the 80^3 / 128-orbital workload
(8,256 unique pairs, r = 48, K = 40): the hand-written backward (the exchange
action, recomputed) against central finite differences of the GPU forward
and against the CPU oracle's gradient 2 w Vx psi.

Finite differences use the fact that perturbing psi_m changes only the pairs
that involve m: E_x = -1/2 sum_ij e_ij, and the m-dependent part equals
2 E_block(m) + e_mm / 2 with E_block(m) = -1/2 sum_j e_mj (block mode, one
target), so each difference is taken between two sums over 128 pairs
instead of two full energies.
"""
import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W
from paper_2401_04189_amd.autograd import exchange_energy

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def run():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    s = W.build_config("cfg3")
    ctx = txe.Context(0)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda().requires_grad_(True)
    E = exchange_energy(psi, sysm, ctx, "f64")
    E.backward()
    torch.cuda.synchronize()
    out = dict(s=s, ctx=ctx, sysm=sysm, psi=psi.detach(), E=float(E), grad=psi.grad.detach().clone())
    yield out
    sysm.close()
    ctx.close()


def test_forward_energy_equals_apply(run):
    _, ex, _ = txe.apply(run["ctx"], run["sysm"], run["psi"], compute="f64")
    torch.cuda.synchronize()
    print(f"E_x = {run['E']:.12f} Ha", flush=True)
    assert abs(float(ex) - run["E"]) <= 1e-13 * abs(run["E"])


def test_backward_matches_oracle_gradient(run):
    s = run["s"]
    st = O.Setup.from_system(s)
    p = s.psi.numpy()
    w3 = O.weights3d(st.q)
    g = run["grad"].cpu().numpy()
    for m in (0, 77):
        ref = 2.0 * w3 * O.apply_target(p, st, m)
        rel = np.linalg.norm(g[m] - ref) / np.linalg.norm(ref)
        print(f"orbital {m}: |grad - oracle| / |oracle| = {rel:.3e}", flush=True)
        assert rel <= 1e-9


def test_backward_central_differences(run):
    ctx, sysm, psi, grad = run["ctx"], run["sysm"], run["psi"], run["grad"]
    N = psi.shape[0]
    rng = np.random.default_rng(2024)
    pa = psi.abs()
    cand = torch.nonzero(pa > 1e-3 * pa.max()).cpu().numpy()
    picks = cand[rng.choice(len(cand), size=20, replace=False)]
    h = 1e-6
    gmax = float(grad.abs().max())

    def part(q, m):
        _, ex, ep = txe.apply(ctx, sysm, q, compute="f64", symmetric=False, i0=int(m), Ni=1, want_vx=False,
                              want_pairs=True)
        return 2.0 * float(ex) + 0.5 * float(ep[int(m)])

    worst = 0.0
    for (m, a, b, c) in picks:
        q = psi.clone()
        q[m, a, b, c] += h
        ep = part(q, m)
        q[m, a, b, c] -= 2 * h
        em = part(q, m)
        fd = (ep - em) / (2 * h)
        gv = float(grad[m, a, b, c])
        # 1e-6 relative, or the FP64 rounding floor of a difference quotient
        # with h = 1e-6 over sums of ~1 Ha (1e-15 Ha / 2h = 5e-10)
        err = abs(fd - gv)
        worst = max(worst, err / abs(gv))
        assert err <= 1e-6 * abs(gv) + 1e-9, (m, a, b, c, fd, gv)
    print(f"20 entries: worst relative difference {worst:.3e} (largest |grad| {gmax:.3e})", flush=True)


def test_f32_autograd_against_f64(run):
    ctx, sysm = run["ctx"], run["sysm"]
    psi = run["psi"].clone().requires_grad_(True)
    E32 = exchange_energy(psi, sysm, ctx, "f32")
    E32.backward()
    torch.cuda.synchronize()
    dE = abs(float(E32) - run["E"])
    g64 = run["grad"]
    rel = float(torch.linalg.vector_norm(psi.grad - g64) / torch.linalg.vector_norm(g64))
    print(f"FP32: |dE_x| = {dE:.3e} Ha, gradient relative difference {rel:.3e}", flush=True)
    assert dE <= 1e-5
    assert rel <= 1e-5
