"""Caller-supplied 1-D convolution matrices (txe_system_desc.C).

  * Giving the library back its own FP64 matrices reproduces the built-in
    path bitwise.
  * On a graded (non-uniform) mesh, which the built-in linear-FE builder
    refuses, the oracle's Gauss-Legendre matrices fed through the ABI give
    the oracle's exchange action and energy to the FP64 bar.
"""
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


def test_own_matrices_reproduce_builtin(ctx):
    s = W.small_system(n=20, L=5.0, N=4, r=10, K=12, seed=41)
    a = txe.System.from_workload(ctx, s)
    C = [a.conv(d)[0] for d in range(3)]
    b = txe.System(ctx, s.grid.x, s.grid.q, s.U, s.w, s.alpha, C=C)
    psi = s.psi.cuda()
    va, ea, pa = txe.apply(ctx, a, psi, compute="f64", want_pairs=True)
    vb, eb, pb = txe.apply(ctx, b, psi, compute="f64", want_pairs=True)
    torch.cuda.synchronize()
    assert torch.equal(va, vb) and torch.equal(ea, eb) and torch.equal(pa, pb)
    a.close()
    b.close()


def test_graded_mesh_against_oracle(ctx):
    g = W.graded_grid(20, 6.0, stretch=1.2)
    s = W.make_system("graded", 20, 6.0, 5, 3, (0.5, 2.0), 12, 10, seed=43, box=1.5, grid=g)
    with pytest.raises(txe.TxeError, match="uniformly spaced"):
        txe.System.from_workload(ctx, s)
    st = O.Setup(s.grid.x, s.grid.q, s.U, s.w, s.alpha)
    sysm = txe.System(ctx, s.grid.x, s.grid.q, s.U, s.w, s.alpha, C=st.C)
    vx, ex, _ = txe.apply(ctx, sysm, s.psi.cuda(), compute="f64")
    ref_vx, ref_e = O.apply(s.psi.numpy(), st)
    e = float(ex)
    print(f"graded mesh: E_x gpu {e:.15e} oracle {ref_e:.15e}", flush=True)
    assert abs(e - ref_e) <= 1e-9 * abs(ref_e)
    w3 = O.weights3d(st.q)
    d = vx.cpu().numpy() - ref_vx
    rel = np.sqrt((d * d * w3).sum(axis=(1, 2, 3)) / (ref_vx * ref_vx * w3).sum(axis=(1, 2, 3))).max()
    assert rel <= 1e-9
    sysm.close()
