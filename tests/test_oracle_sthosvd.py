"""Pins of the oracle's per-pair bases (the sequentially truncated HOSVD of each
pair density, eq. `TuckerDecompField` with per-pair factors) and of the
exchange evaluated with them, to things other than the oracle itself:

  * the factors are q-orthonormal, and at full rank the decomposition
    reproduces the field exactly;
  * the squared W-norm error of the truncation equals the sum of the squared
    singular values cut at each step (an identity of the sequential
    truncation), and stays below the sum of the squared tail singular values
    of the original unfoldings (computed here by an independent SVD);
  * a tensor built with a known multilinear rank is recovered exactly at that
    rank, and the error decreases as the ranks grow;
  * a separable (rank-1) pair density at rank (1, 1, 1) gives the exact
    energy sum_k w_k prod_d (q_d g_d)^T C_k^d g_d of the 1-D factors;
  * at full rank the per-pair result equals the dense 3-D kernel apply.
No GPU.
"""
import numpy as np
import pytest

from oracle import txe_oracle as O
from paper_2401_04189_amd import workloads as W


def wnorm2(T, q):
    return float((O.weights3d(q) * T * T).sum())


def reconstruct_field(U, G):
    return O.reconstruct(G, U)


@pytest.fixture(scope="module")
def graded():
    """A non-uniform grid (so that the W weighting matters) and a pair density."""
    g = W.graded_grid((10, 12, 9), (4.0, 4.5, 3.5), stretch=1.3)
    psi, _ = W.make_orbitals(g, 2, 3, (0.5, 2.0), seed=71, box=1.5)
    rho = psi[0].numpy() * psi[1].numpy()
    return g, rho


def test_factors_orthonormal_and_full_rank_exact(graded):
    g, rho = graded
    U, G, cut = O.sthosvd(rho, g.q, g.n)
    for d in range(3):
        M = U[d].T @ (g.q[d][:, None] * U[d])
        assert np.abs(M - np.eye(g.n[d])).max() <= 1e-12
        assert cut[d].size == 0
    rec = reconstruct_field(U, G)
    assert np.abs(rec - rho).max() <= 1e-12 * np.abs(rho).max()
    # the core of the W-orthonormal decomposition carries the W-norm
    assert abs(float((G * G).sum()) - wnorm2(rho, g.q)) <= 1e-12 * wnorm2(rho, g.q)


@pytest.mark.parametrize("ranks", [(4, 5, 3), (7, 6, 8), (2, 2, 2)])
def test_truncation_error_identity_and_bound(graded, ranks):
    g, rho = graded
    U, G, cut = O.sthosvd(rho, g.q, ranks)
    err2 = wnorm2(rho - reconstruct_field(U, G), g.q)
    cut2 = sum(float(c.sum()) for c in cut)
    assert abs(err2 - cut2) <= 1e-12 * wnorm2(rho, g.q)
    # T-HOSVD bound from the original (scaled) tensor's unfoldings
    X = rho * np.sqrt(O.weights3d(g.q))
    bound = 0.0
    for d in range(3):
        sv = np.linalg.svd(np.moveaxis(X, d, 0).reshape(X.shape[d], -1), compute_uv=False)
        bound += float((sv[ranks[d]:] ** 2).sum())
    assert err2 <= bound * (1 + 1e-12) + 1e-300


def test_known_multilinear_rank_recovered_and_error_decays():
    g = W.uniform_grid((11, 13, 12), (3.0, 3.0, 3.0))
    rng = np.random.default_rng(72)
    core = rng.normal(size=(3, 4, 2))
    A = [rng.normal(size=(g.n[d], core.shape[d])) for d in range(3)]
    T = core
    for d in range(3):
        T = O.mode_product(T, A[d], d)
    U, G, _ = O.sthosvd(T, g.q, core.shape)
    assert np.abs(reconstruct_field(U, G) - T).max() <= 1e-11 * np.abs(T).max()
    # a smooth pair density: the error falls as the ranks grow
    psi, _ = W.make_orbitals(g, 2, 3, (0.5, 2.0), seed=73, box=1.0)
    rho = psi[0].numpy() * psi[1].numpy()
    errs = []
    for r in range(1, 10):
        U, G, _ = O.sthosvd(rho, g.q, (r, r, r))
        errs.append(wnorm2(rho - reconstruct_field(U, G), g.q))
    assert all(b <= a * (1 + 1e-12) for a, b in zip(errs, errs[1:]))
    assert errs[-1] <= 1e-6 * errs[0]


def test_separable_density_rank_one_energy():
    g = W.uniform_grid((14, 12, 16), (4.0, 3.5, 4.5))
    w, a = W.exp_sum(8)
    st = O.Setup(g.x, g.q, W.full_rank_bases(g, 3), w, a)
    # single s-Gaussians psi_i, psi_j (different centres): rho is separable
    a = [np.exp(-0.7 * (g.x[d] - 0.3) ** 2) for d in range(3)]
    b = [np.exp(-1.1 * (g.x[d] + 0.2 * d) ** 2) for d in range(3)]
    sep = lambda v: v[0][:, None, None] * v[1][None, :, None] * v[2][None, None, :]  # noqa: E731
    psi_i, psi_j = sep(a), sep(b)
    f = [a[d] * b[d] for d in range(3)]
    _, e, _, _, _ = O.pair_sthosvd(psi_i, psi_j, st, (1, 1, 1))
    exact = sum(w[k] * np.prod([(g.q[d] * f[d]) @ st.C[d][k] @ f[d] for d in range(3)]) for k in range(len(w)))
    assert abs(e - exact) <= 1e-12 * abs(exact)


def test_full_rank_per_pair_equals_dense_kernel():
    g = W.uniform_grid(8, 3.0)
    psi, _ = W.make_orbitals(g, 3, 2, (0.5, 2.0), seed=74, box=1.0)
    w, a = W.exp_sum(6)
    st = O.Setup(g.x, g.q, W.full_rank_bases(g, 5), w, a)
    p = psi.numpy()
    vx, ex = O.apply_sthosvd(p, st, g.n)
    ref = np.zeros_like(p)
    eref = 0.0
    w3 = O.weights3d(g.q)
    for i in range(3):
        for j in range(3):
            phi = O.dense_kernel_apply(p[i] * p[j], w, st.C)
            ref[i] -= p[j] * phi
            eref += -0.5 * float((w3 * p[i] * p[j] * phi).sum())
    assert np.abs(vx - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(ex - eref) <= 1e-12 * abs(eref)
