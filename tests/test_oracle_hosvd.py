"""Pins of the oracle's shared-basis step (O10: the HOSVD of the stacked pair
densities in the W inner product) to facts that do not come from it:

  * the bases are q-orthonormal;
  * for separable orbitals psi_i = f_i(x) g_i(y) h_i(z) the mode-0 span of
    the stack is span{sqrt(q) f_i f_j}, found here by a QR factorisation, and
    every singular value past its dimension vanishes;
  * the Gram identity: the stack's mode-d Gram matrix is
    sum_m (P_m^T P_m) * (P_m^T P_m) over the other two indices m (P_m the
    N x n_d slice of the orbitals), evaluated here without forming any pair
    density; its eigenvalues are the squared singular values and its leading
    eigenvectors span the bases;
  * an orthogonal mixing of the orbitals leaves the singular values and the
    subspaces unchanged.
No GPU."""
import numpy as np

from oracle import txe_oracle as O
from paper_2401_04189_amd import workloads as W


def projector(U, q):
    Ut = np.sqrt(q)[:, None] * U
    return Ut @ Ut.T


def small(seed=5, n=(14, 16, 18), N=3):
    g = W.uniform_grid(n, (4.0, 4.5, 5.0))
    psi, _ = W.make_orbitals(g, N, 3, (0.5, 2.0), seed=seed, box=1.5)
    return g, psi.numpy()


def test_bases_are_q_orthonormal():
    g, psi = small()
    U, _ = O.shared_hosvd(psi, g.q, (8, 9, 10))
    for d in range(3):
        M = U[d].T @ (g.q[d][:, None] * U[d])
        assert np.abs(M - np.eye(M.shape[0])).max() <= 1e-12


def test_separable_orbitals_span_the_products():
    rng = np.random.default_rng(7)
    g = W.uniform_grid((16, 12, 12), (4.0, 4.0, 4.0))
    N = 3
    f = [np.exp(-rng.uniform(0.3, 1.5) * (g.x[0] - rng.uniform(-1, 1)) ** 2) for _ in range(N)]
    gy = [np.exp(-rng.uniform(0.3, 1.5) * (g.x[1] - rng.uniform(-1, 1)) ** 2) for _ in range(N)]
    hz = [np.exp(-rng.uniform(0.3, 1.5) * (g.x[2] - rng.uniform(-1, 1)) ** 2) for _ in range(N)]
    psi = np.stack([f[i][:, None, None] * gy[i][None, :, None] * hz[i][None, None, :] for i in range(N)])
    prods = np.stack([np.sqrt(g.q[0]) * f[i] * f[j] for i in range(N) for j in range(i, N)], axis=1)
    Q, R = np.linalg.qr(prods)
    dim = int((np.abs(np.diag(R)) > 1e-10 * np.abs(R).max()).sum())
    assert dim == N * (N + 1) // 2
    U, sv = O.shared_hosvd(psi, g.q, (dim, 4, 4))
    assert np.abs(projector(U[0], g.q[0]) - Q[:, :dim] @ Q[:, :dim].T).max() <= 1e-10
    assert sv[0][dim:].max() <= 1e-12 * sv[0][0]


def gram_identity(psi, q, d, targets=None):
    N = psi.shape[0]
    P = np.moveaxis(psi, d + 1, 1).reshape(N, psi.shape[d + 1], -1)          # (N, n_d, m)
    others = [q[e] for e in range(3) if e != d]
    qm = (others[0][:, None] * others[1][None, :]).reshape(-1)
    D = np.einsum("iam,ibm->mab", P, P)
    Pt = P if targets is None else P[list(targets)]
    DT = np.einsum("iam,ibm->mab", Pt, Pt)
    S = np.einsum("m,mab->ab", qm, D * DT)
    return np.sqrt(q[d])[:, None] * S * np.sqrt(q[d])[None, :]


def test_gram_identity_gives_the_singular_values_and_subspaces():
    g, psi = small(seed=9)
    ranks = (6, 7, 8)
    for targets in (None, [1, 2]):
        U, sv = O.shared_hosvd(psi, g.q, ranks, targets=targets)
        for d in range(3):
            S = gram_identity(psi, g.q, d, targets)
            lam, V = np.linalg.eigh(S)
            lam, V = lam[::-1], V[:, ::-1]
            k = min(len(sv[d]), 6)
            assert np.abs(lam[:k] - sv[d][:k] ** 2).max() <= 1e-10 * lam[0]
            r = ranks[d]
            assert sv[d][r] < 0.7 * sv[d][r - 1]  # a gap at the rank: the subspace is well defined
            assert np.abs(projector(U[d], g.q[d]) - V[:, :r] @ V[:, :r].T).max() <= 1e-8


def test_orbital_rotation_leaves_the_bases():
    g, psi = small(seed=11, N=4)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
    mixed = np.einsum("ij,jabc->iabc", Q, psi)
    ranks = (7, 7, 7)
    U, sv = O.shared_hosvd(psi, g.q, ranks)
    U2, sv2 = O.shared_hosvd(mixed, g.q, ranks)
    for d in range(3):
        k = 10
        assert np.abs(sv[d][:k] - sv2[d][:k]).max() <= 1e-11 * sv[d][0]
        assert np.abs(projector(U[d], g.q[d]) - projector(U2[d], g.q[d])).max() <= 1e-8
