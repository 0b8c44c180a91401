"""The collocation form on the GPU (phi = sum_k w_k G x_d (C_k^d U_d): the
1-D convolutions evaluated at every node and the field reconstructed, pair
energies as grid sums) against the oracle's collocation step, in FP64:

  * the uniform linear-element grid, symmetric and block mode;
  * order-5 Lagrange elements at GLL nodes on an adaptively refined mesh,
    with the library's own FE convolution matrices given to the system
    (and the core-space form on the same system against the oracle);
  * full rank, where the collocation form is the dense kernel apply;
  * chunked applies bitwise equal to one chunk;
  * the unsupported combinations.

Tolerance 1e-11: the two sides run the same linear algebra in FP64 (no
eigen-decomposition, no truncation choice), so they differ by summation
order only."""
import numpy as np
import pytest
import torch

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-11


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = txe.Context(0)
    yield c
    c.close()


def wrel(v, ref, q):
    w3 = O.weights3d(q)
    num = np.sqrt((w3[None] * (v - ref) ** 2).sum(axis=(1, 2, 3)))
    den = np.sqrt((w3[None] * ref ** 2).sum(axis=(1, 2, 3)))
    return float((num / den).max())


def compare(ctx, sysm, st, psi, symmetric=True, i0=0, Ni=None, form="collocation", label=""):
    p = psi.numpy()
    pairs = {}
    if form == "collocation":
        vref, eref = O.apply_collocation(p, st, mode="symmetric" if symmetric else "block", i0=i0, Ni=Ni,
                                         pairs_out=pairs)
    else:
        vref, eref = O.apply(p, st, mode="symmetric" if symmetric else "block", i0=i0, Ni=Ni)
    vx, ex, ep = txe.apply(ctx, sysm, psi.cuda(), compute="f64", symmetric=symmetric, i0=i0, Ni=Ni,
                           want_pairs=True, form=form)
    torch.cuda.synchronize()
    vx, ex, ep = vx.cpu().numpy(), float(ex), ep.cpu().numpy()
    N = p.shape[0]
    x_err = abs(ex - eref) / abs(eref)
    v_err = wrel(vx, vref, st.q)
    msg = f"[{label}] {form}: E_x rel {x_err:.2e}  Vx rel {v_err:.2e}"
    if pairs:
        if symmetric:
            epref = np.array([pairs[(i, j)] for i in range(N) for j in range(i, N)])
        else:
            epref = np.array([pairs[(i0 + t, j)] for t in range(Ni) for j in range(N)])
        e_err = np.abs(ep - epref).max() / np.abs(epref).max()
        msg += f"  e_ij rel {e_err:.2e}"
        assert e_err <= TOL
    print(msg, flush=True)
    assert x_err <= TOL and v_err <= TOL
    return vx, ex


def test_uniform_grid_symmetric_and_block(ctx):
    s = W.small_system(n=16, L=5.0, N=3, r=6, K=8, seed=71)
    st = O.Setup.from_system(s)
    sysm = txe.System.from_workload(ctx, s)
    compare(ctx, sysm, st, s.psi, label="n16 sym")
    compare(ctx, sysm, st, s.psi, symmetric=False, i0=1, Ni=2, label="n16 block")
    sysm.close()


def test_two_rank_tiles_non_cubic(ctx):
    g = W.uniform_grid((16, 20, 24), (4.0, 5.0, 6.0))
    psi, _ = W.make_orbitals(g, 3, 3, (0.5, 2.0), seed=72, box=1.5)
    U = W.hosvd_bases(psi, g, (12, 18, 20))
    w, a = W.exp_sum(10)
    s = W.System(name="noncubic", grid=g, psi=psi, U=U, w=w, alpha=a)
    st = O.Setup.from_system(s)
    sysm = txe.System.from_workload(ctx, s)
    compare(ctx, sysm, st, psi, label="non-cubic r=12,18,20")
    sysm.close()


def fe_system(p=5, seed=73):
    """Order-p elements on adaptively refined meshes around two atoms."""
    centres = [(-1.2, 0.9), (0.4, -0.8), (1.1, 0.3)]  # per mode: the atoms' coordinates
    edges = [W.adaptive_edges(L=6.0, bms=3.0, msna=0.8, centres=list(c), ball=1.2, p=p) for c in centres]
    meshes = [O.fe_mesh_1d(e, p) for e in edges]
    g = W.grid_from_nodes([m[0] for m in meshes], [m[1] for m in meshes])
    atoms = np.array([[c[0] for c in centres], [c[1] for c in centres]])
    psi, _ = W.make_orbitals(g, 3, 3, (0.5, 2.0), seed=seed, atoms=atoms)
    U = W.hosvd_bases(psi, g, (10, 10, 10))
    w, a = W.exp_sum(8)
    return edges, g, psi, U, w, a


def test_order5_adaptive_mesh(ctx):
    p = 5
    edges, g, psi, U, w, a = fe_system(p)
    # the oracle's FE matrices on its side, the library's on the GPU side
    C_or = [np.stack([O.conv_matrix_fe(e, p, ak) for ak in a]) for e in edges]
    st = O.Setup(g.x, g.q, U, w, a, C=C_or)
    xq = [txe.fe_mesh_1d(e, p) for e in edges]
    for d in range(3):
        assert np.abs(xq[d][0] - g.x[d]).max() <= 1e-14 and np.abs(xq[d][1] - g.q[d]).max() <= 1e-14
    C_lib = [txe.fe_conv_matrices(e, p, a) for e in edges]
    sysm = txe.System(ctx, [v[0] for v in xq], [v[1] for v in xq], U, w, a, C=C_lib)
    print(f"order-5 adaptive mesh: n = {g.n}", flush=True)
    compare(ctx, sysm, st, psi, label="p5 adaptive")
    compare(ctx, sysm, st, psi, form="core", label="p5 adaptive")
    sysm.close()


def test_full_rank_is_the_dense_kernel(ctx):
    g = W.uniform_grid(12, 4.0)
    psi, _ = W.make_orbitals(g, 2, 3, (0.5, 2.0), seed=74, box=1.0)
    w, a = W.exp_sum(6)
    U = W.full_rank_bases(g, 3)
    st = O.Setup(g.x, g.q, U, w, a)
    sysm = txe.System(ctx, g.x, g.q, U, w, a)
    vx, _ = compare(ctx, sysm, st, psi, label="full rank")
    p = psi.numpy()
    ref = np.zeros_like(p)
    for i in range(2):
        for j in range(2):
            ref[i] -= p[j] * O.dense_kernel_apply(p[i] * p[j], w, st.C)
    assert wrel(vx, ref, g.q) <= 1e-10
    sysm.close()


def test_chunked_bitwise(ctx, monkeypatch):
    s = W.small_system(n=16, L=5.0, N=7, r=6, K=8, seed=75)
    sysm = txe.System.from_workload(ctx, s)
    psi = s.psi.cuda()
    kw = dict(compute="f64", want_pairs=True, want_orb=True, form="collocation")
    one = txe.apply(ctx, sysm, psi, **kw)
    torch.cuda.synchronize()
    monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(txe.workspace_bytes(ctx, sysm, psi) // 4))
    got = txe.apply(ctx, sysm, psi, **kw)
    torch.cuda.synchronize()
    monkeypatch.delenv("TXE_TEST_MAX_WORKSPACE")
    for x, y in zip(got, one):
        assert torch.equal(x, y)
    blk = txe.apply(ctx, sysm, psi, compute="f64", symmetric=False, i0=2, Ni=3, form="collocation")
    monkeypatch.setenv("TXE_TEST_MAX_WORKSPACE", str(txe.workspace_bytes(ctx, sysm, psi) // 4))
    blk2 = txe.apply(ctx, sysm, psi, compute="f64", symmetric=False, i0=2, Ni=3, form="collocation")
    torch.cuda.synchronize()
    monkeypatch.delenv("TXE_TEST_MAX_WORKSPACE")
    assert torch.equal(blk[0], blk2[0]) and torch.equal(blk[1], blk2[1])
    sysm.close()


def test_unsupported_combinations(ctx):
    s = W.small_system(n=16, L=5.0, N=2, r=6, K=8, seed=76)
    sysm = txe.System.from_workload(ctx, s)
    for kw in (dict(compute="f32"), dict(compute="f64", pair_bases=True)):
        with pytest.raises(txe.TxeError) as ei:
            txe.apply(ctx, sysm, s.psi.cuda(), form="collocation", **kw)
        assert ei.value.status == 5
    sysm.close()
