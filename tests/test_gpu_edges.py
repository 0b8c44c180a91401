"""Edge and degenerate cases of the GPU path against the CPU oracle:
a single orbital (one self pair), one Gaussian term, rank 1 in every mode,
the largest term count the ABI takes (K = 256), the largest rank (r = 80)
at full rank, all-zero orbitals, and an empty orbital set (refused)."""
import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-9


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


def check(ctx, s, compute="f64", label=""):
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    vx, ex, _ = txe.apply(ctx, sysm, psi, compute=compute)
    torch.cuda.synchronize()
    st = O.Setup.from_system(s)
    ref_vx, ref_e = O.apply(s.psi.numpy(), st)
    w3 = O.weights3d(st.q)
    d = vx.cpu().numpy() - ref_vx
    den = np.sqrt((ref_vx * ref_vx * w3).sum(axis=(1, 2, 3)))
    rel = float((np.sqrt((d * d * w3).sum(axis=(1, 2, 3))) / den).max())
    de = abs(float(ex) - ref_e) / abs(ref_e)
    print(f"[{label}] E_x gpu {float(ex):.15e} oracle {ref_e:.15e} rel {de:.2e}  Vx rel {rel:.2e}", flush=True)
    sysm.close()
    return de, rel


def test_single_orbital(ctx):
    s = W.small_system(n=16, L=5.0, N=1, r=8, K=10, seed=61)
    de, rel = check(ctx, s, label="N=1")
    assert de <= TOL and rel <= TOL
    de, rel = check(ctx, s, compute="f32", label="N=1 f32")
    assert de <= 1e-5 and rel <= 1e-5


def test_one_term_and_rank_one(ctx):
    s = W.small_system(n=12, L=5.0, N=3, r=1, K=1, seed=62)
    de, rel = check(ctx, s, label="K=1 r=1")
    assert de <= TOL and rel <= TOL


def test_largest_term_count(ctx):
    s = W.small_system(n=12, L=5.0, N=2, r=6, K=256, seed=63)
    de, rel = check(ctx, s, label="K=256")
    assert de <= TOL and rel <= TOL


def test_largest_rank_full(ctx):
    s = W.small_system(n=80, L=8.0, N=1, r=80, K=3, seed=64, bases="full")
    de, rel = check(ctx, s, label="r=80 full rank")
    assert de <= TOL and rel <= TOL


def test_zero_orbitals(ctx):
    s = W.small_system(n=16, L=5.0, N=2, r=6, K=8, seed=65)
    sysm = txe.System.from_workload(ctx, s)
    psi = torch.zeros_like(s.psi).cuda()
    for comp in ("f64", "f32", "bf16x3"):
        vx, ex, ep = txe.apply(ctx, sysm, psi, compute=comp, want_pairs=True)
        torch.cuda.synchronize()
        assert float(ex) == 0.0 and float(vx.abs().max()) == 0.0 and float(ep.abs().max()) == 0.0
    sysm.close()


def test_empty_orbital_set_is_refused(ctx):
    s = W.small_system(n=16, L=5.0, N=2, r=6, K=8, seed=66)
    sysm = txe.System.from_workload(ctx, s)
    empty = torch.zeros((0,) + tuple(sysm.n), dtype=torch.float64, device="cuda")
    with pytest.raises(txe.TxeError):
        txe.apply(ctx, sysm, empty, compute="f64")
    sysm.close()
