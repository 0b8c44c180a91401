"""Adaptively compressed exchange on the GPU (txe_ace_build / txe_ace_apply)
against the CPU oracle, each side from its own exchange action.

  * 16^3, 6 orbitals: M, L and xi to the FP64 bar against the oracle; V_ACE
    on random trial functions against the oracle's operator;
  * exactness on the orbitals (V_ACE psi = Vx psi) on the GPU, FP64 and
    FP32, at 16^3 and on the 64^3 / 64-orbital workload;
  * a W that is not negative definite sets info to the failing column;
  * many orbitals (several 64 x 64 Gram tiles with a ragged last one, and
    several grid chunks): the build and a non-square apply against the
    oracle, with synthetic orbitals and W = -psi (M = -Gram(psi) is negative
    definite).
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


@pytest.fixture(scope="module")
def small(ctx):
    s = W.small_system(n=16, L=5.0, N=6, r=10, K=12, seed=51)
    sysm = txe.System.from_workload(ctx, s)
    st = O.Setup.from_system(s)
    p = s.psi.numpy()
    vx_ref, _ = O.apply(p, st)
    M_ref, L_ref, xi_ref = O.ace_build(p, vx_ref, st.q)
    yield s, sysm, st, vx_ref, M_ref, L_ref, xi_ref
    sysm.close()


def test_ace_build_against_oracle(ctx, small):
    s, sysm, st, vx_ref, M_ref, L_ref, xi_ref = small
    psi = s.psi.cuda()
    vx, _, _ = txe.apply(ctx, sysm, psi, compute="f64")
    xi, info, M, L = txe.ace_build(ctx, sysm, psi, vx, want_factors=True)
    torch.cuda.synchronize()
    assert int(info) == 0
    M, L, xi = M.cpu().numpy(), L.cpu().numpy(), xi.cpu().numpy()
    em = np.abs(M - M_ref).max() / np.abs(M_ref).max()
    el = np.abs(L - L_ref).max() / np.abs(L_ref).max()
    ex = np.abs(xi - xi_ref).max() / np.abs(xi_ref).max()
    print(f"M rel {em:.2e}  L rel {el:.2e}  xi rel {ex:.2e}", flush=True)
    assert em <= 1e-10 and el <= 1e-10 and ex <= 1e-9
    assert np.abs(np.triu(L, 1)).max() == 0.0


def test_ace_apply_against_oracle(ctx, small):
    s, sysm, st, vx_ref, M_ref, L_ref, xi_ref = small
    psi = s.psi.cuda()
    vx, _, _ = txe.apply(ctx, sysm, psi, compute="f64")
    xi, info = txe.ace_build(ctx, sysm, psi, vx)
    rng = np.random.default_rng(9)
    phi = rng.standard_normal((5,) + tuple(sysm.n))
    out = txe.ace_apply(ctx, sysm, xi, torch.as_tensor(phi, device="cuda")).cpu().numpy()
    ref = O.ace_apply(xi_ref, st.q, phi)
    rel = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"V_ACE phi rel {rel:.2e}", flush=True)
    assert int(info) == 0 and rel <= 1e-9


@pytest.mark.parametrize("compute,tol", [("f64", 1e-11), ("f32", 1e-5)])
def test_ace_exact_on_orbitals(ctx, small, compute, tol):
    s, sysm = small[0], small[1]
    dt = torch.float64 if compute == "f64" else torch.float32
    psi = s.psi.to(dt).cuda()
    vx, _, _ = txe.apply(ctx, sysm, psi, compute=compute)
    xi, info = txe.ace_build(ctx, sysm, psi, vx)
    out = txe.ace_apply(ctx, sysm, xi, psi)
    torch.cuda.synchronize()
    rel = float((out.double() - vx.double()).abs().max() / vx.double().abs().max())
    print(f"{compute}: |V_ACE psi - Vx psi| / |Vx psi| = {rel:.2e}", flush=True)
    assert int(info) == 0 and rel <= tol


def test_ace_exact_on_64cube_workload(ctx):
    s = W.build_config("cfg2", device="cuda")
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi
    vx, _, _ = txe.apply(ctx, sysm, psi, compute="f64")
    xi, info, M, L = txe.ace_build(ctx, sysm, psi, vx, want_factors=True)
    out = txe.ace_apply(ctx, sysm, xi, psi)
    torch.cuda.synchronize()
    rel = float((out - vx).abs().max() / vx.abs().max())
    asym = float((M - M.T).abs().max() / M.abs().max())
    print(f"64^3: info {int(info)}  |V_ACE psi - Vx psi| rel {rel:.2e}  M asymmetry {asym:.2e}", flush=True)
    assert int(info) == 0 and rel <= 1e-10 and asym <= 1e-12
    sysm.close()


def test_ace_reports_non_definite_matrix(ctx, small):
    s, sysm = small[0], small[1]
    psi = s.psi.cuda()
    # W = +psi makes M = +I (positive): the first pivot fails
    xi, info = txe.ace_build(ctx, sysm, psi, psi.clone())
    torch.cuda.synchronize()
    assert int(info) == 1


def test_ace_many_orbitals_against_oracle(ctx, small):
    """N = 150 (three Gram tiles, the last with 22 rows) on the 16^3 grid
    (16 grid chunks per tile); 70 trial functions for the apply (a 70 x 150
    Gram).  Inputs are synthetic: the build only needs W with <psi, W> < 0."""
    s, sysm, st = small[0], small[1], small[2]
    rng = np.random.default_rng(150)
    p = rng.standard_normal((150,) + tuple(sysm.n))
    w = -p
    M_ref, L_ref, xi_ref = O.ace_build(p, w, st.q)
    psi = torch.as_tensor(p, device="cuda")
    xi, info, M, L = txe.ace_build(ctx, sysm, psi, torch.as_tensor(w, device="cuda"), want_factors=True)
    phi = rng.standard_normal((70,) + tuple(sysm.n))
    out = txe.ace_apply(ctx, sysm, xi, torch.as_tensor(phi, device="cuda")).cpu().numpy()
    torch.cuda.synchronize()
    M, L, xi = M.cpu().numpy(), L.cpu().numpy(), xi.cpu().numpy()
    em = np.abs(M - M_ref).max() / np.abs(M_ref).max()
    el = np.abs(L - L_ref).max() / np.abs(L_ref).max()
    ex = np.abs(xi - xi_ref).max() / np.abs(xi_ref).max()
    ref = O.ace_apply(xi_ref, st.q, phi)
    ea = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"N=150: M rel {em:.2e}  L rel {el:.2e}  xi rel {ex:.2e}  V_ACE phi rel {ea:.2e}", flush=True)
    assert int(info) == 0
    assert em <= 1e-10 and el <= 1e-10 and ex <= 1e-9 and ea <= 1e-9
