"""The pins in test_oracle_pins must catch plausible mistakes in the oracle.

Each case plants one mistake in the oracle (on the CPU, by monkeypatching one
of its steps) and checks that at least one of the pins then fails.
"""
import numpy as np
import pytest

import tests.test_oracle_pins as P
from oracle import txe_oracle as O
from paper_2401_04189_amd import workloads as W


def _pins_fail():
    """Run a cheap subset of the pins; True when any of them fails."""
    checks = [
        P.test_full_rank_equals_dense_kernel,
        P.test_non_cubic_full_rank_equals_dense_kernel,
        P.test_constant_kernel_limit,
        P.test_single_gaussian_energy_converges_second_order,
        lambda: P.test_conv_matrix_closed_form(30.0),
    ]
    s = W.small_system(n=10, L=5.0, N=3, r=6, K=6, seed=21)
    st = O.Setup.from_system(s)
    fixture = (s, st)
    checks += [
        lambda: P.test_exchange_matrix_symmetric_nsd_trace(fixture),
        lambda: P.test_gradient_central_differences(fixture),
    ]
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError):
            return True
    return False


def test_unmutated_oracle_passes():
    assert not _pins_fail()


def _mut_project_with_U(rho, V):          # forgets the quadrature weights
    G = rho
    for d in range(3):
        G = O.mode_product(G, (V[d] / V[d].max() * 1.0).T, d)
    return G


def _mut_core_drop_last_term(G, w, Chat):
    return _orig["core_sum"](G, w[:-1], [c[:-1] for c in Chat])


def _mut_core_mode0_everywhere(G, w, Chat):
    return _orig["core_sum"](G, w, [Chat[0], Chat[0][:, :Chat[1].shape[1], :Chat[1].shape[2]]
                                    if Chat[0].shape[1] >= Chat[1].shape[1] else Chat[1], Chat[2]])


def _swap(Phi, U):
    phi = O.mode_product(Phi, U[1][:U[0].shape[0]] if U[1].shape[0] == U[0].shape[0] else U[0], 0)
    phi = O.mode_product(phi, U[0][:U[1].shape[0]] if U[0].shape[0] == U[1].shape[0] else U[1], 1)
    return O.mode_product(phi, U[2], 2)


def _mut_conv_half_hat(x, alpha, order=12):
    C = _orig["conv_matrix_1d"](x, alpha, order)
    C[:, 0] *= 0.5                        # half hat at the first node
    return C


def _mut_pair_sign(psi_i, psi_j, st):
    phi, e, G, Phi = _orig["pair"](psi_i, psi_j, st)
    return -phi, e, G, Phi


_orig = {"core_sum": O.core_sum, "conv_matrix_1d": O.conv_matrix_1d, "pair": O.pair}


@pytest.mark.parametrize("name,fn", [
    ("project", _mut_project_with_U),
    ("core_sum", _mut_core_drop_last_term),
    ("core_sum", _mut_core_mode0_everywhere),
    ("reconstruct", _swap),
    ("conv_matrix_1d", _mut_conv_half_hat),
    ("pair", _mut_pair_sign),
])
def test_planted_mistake_is_caught(monkeypatch, name, fn):
    monkeypatch.setattr(O, name, fn)
    assert _pins_fail(), f"a planted mistake in oracle step {name} ({fn.__name__}) went unnoticed"


def _ace_pins_fail():
    s = W.small_system(n=10, L=5.0, N=3, r=6, K=6, seed=21)
    st = O.Setup.from_system(s)
    psi = s.psi.numpy()
    vx, _ = O.apply(psi, st)
    M, L, xi = O.ace_build(psi, vx, st.q)
    fixture = (s, st, psi, vx, M, L, xi)
    for c in (P.test_ace_exact_on_the_orbitals, P.test_ace_factor_and_matrix,
              P.test_ace_operator_symmetric_nsd_and_rank):
        try:
            c(fixture)
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            return True
    return False


def test_unmutated_ace_passes():
    assert not _ace_pins_fail()


@pytest.mark.parametrize("mistake", ["transposed_inverse", "dropped_weights", "sign"])
def test_ace_mistakes_are_caught(monkeypatch, mistake):
    orig_build, orig_apply = O.ace_build, O.ace_apply

    def bad_build(psi, Wv, q):
        N = psi.shape[0]
        w3 = O.weights3d(q).reshape(-1)
        P_, Wm = psi.reshape(N, -1), Wv.reshape(N, -1)
        M = P_ @ (Wm * (np.ones_like(w3) if mistake == "dropped_weights" else w3)[None, :]).T
        L = np.linalg.cholesky(-M)
        Li = np.linalg.inv(L)
        if mistake == "transposed_inverse":
            Li = Li.T
        xi = (Li @ Wm).reshape(Wv.shape)
        return M, L, xi

    def bad_apply(xi, q, phi):
        out = orig_apply(xi, q, phi)
        return -out if mistake == "sign" else out

    monkeypatch.setattr(O, "ace_build", bad_build if mistake != "sign" else orig_build)
    monkeypatch.setattr(O, "ace_apply", bad_apply)
    assert _ace_pins_fail()


# ---------------------------------------------------------------------------------------
# per-pair bases (the sequentially truncated HOSVD)
# ---------------------------------------------------------------------------------------
import tests.test_oracle_sthosvd as S  # noqa: E402


def _sthosvd_pins_fail():
    g = W.graded_grid((10, 12, 9), (4.0, 4.5, 3.5), stretch=1.3)
    psi, _ = W.make_orbitals(g, 2, 3, (0.5, 2.0), seed=71, box=1.5)
    fixture = (g, psi[0].numpy() * psi[1].numpy())
    checks = [lambda: S.test_factors_orthonormal_and_full_rank_exact(fixture),
              lambda: S.test_truncation_error_identity_and_bound(fixture, (4, 5, 3)),
              S.test_known_multilinear_rank_recovered_and_error_decays,
              S.test_separable_density_rank_one_energy,
              S.test_full_rank_per_pair_equals_dense_kernel]
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, np.linalg.LinAlgError):
            return True
    return False


def test_unmutated_sthosvd_passes():
    assert not _sthosvd_pins_fail()


def _st_mutant(mistake):
    """One plausible mistake in the sequential truncation."""
    def sthosvd(rho, q, ranks):
        X = np.asarray(rho, dtype=np.float64)
        if mistake != "unweighted":
            for d in range(3):
                X = O.mode_product(X, np.diag(np.sqrt(q[d])), d)
        X0 = X.copy()
        U, cut = [], []
        for d in range(3):
            src = X0 if mistake == "not_sequential" else X
            W_, sv, _ = np.linalg.svd(O.unfold(src, d), full_matrices=False)
            Ut = W_[:, -ranks[d]:] if mistake == "trailing_vectors" else W_[:, :ranks[d]]
            cut.append(sv[ranks[d]:] ** 2)
            X = O.mode_product(X, Ut.T, d)
            U.append(Ut if mistake == "unscaled_factors" else Ut / np.sqrt(q[d])[:, None])
        return U, X, cut
    return sthosvd


@pytest.mark.parametrize("mistake", ["unweighted", "not_sequential", "trailing_vectors", "unscaled_factors"])
def test_sthosvd_mistakes_are_caught(monkeypatch, mistake):
    monkeypatch.setattr(O, "sthosvd", _st_mutant(mistake))
    assert _sthosvd_pins_fail(), f"planted mistake {mistake} in the per-pair decomposition went unnoticed"


# ---------------------------------------------------------------------------------------
# order-p elements and the collocation form
# ---------------------------------------------------------------------------------------
import tests.test_oracle_fe as FE  # noqa: E402


def _fe_pins_fail():
    checks = [lambda: FE.test_gll_rule(5), FE.test_order_one_is_the_linear_hat_construction,
              lambda: FE.test_convolution_matrix_reproduces_polynomials(5, 30.0),
              FE.test_collocation_at_full_rank_is_the_dense_kernel]
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, IndexError):
            return True
    return False


def test_unmutated_fe_passes():
    assert not _fe_pins_fail()


_orig_fe = {"gll_points": O.gll_points, "fe_mesh_1d": O.fe_mesh_1d, "pair_collocation": O.pair_collocation}


def _equispaced_nodes(p):                      # Lagrange nodes equally spaced instead of GLL
    s, w = _orig_fe["gll_points"](p)
    return np.linspace(-1.0, 1.0, p + 1), w


def _weights_without_jacobian(edges, p):       # nodal weights missing the half cell length
    x, q, cells = _orig_fe["fe_mesh_1d"](edges, p)
    return x, q * 2.0 / (edges[1] - edges[0]), cells


def _collocation_without_kernel(psi_i, psi_j, st):   # reconstruction forgets C_k
    rho = psi_i * psi_j
    G = O.project(rho, st.V)
    phi = sum(st.w[k] * O.reconstruct(G, st.U) for k in range(len(st.w)))
    return phi, float((O.weights3d(st.q) * rho * phi).sum())


@pytest.mark.parametrize("name,fn", [("gll_points", _equispaced_nodes), ("fe_mesh_1d", _weights_without_jacobian),
                                     ("pair_collocation", _collocation_without_kernel)])
def test_fe_mistakes_are_caught(monkeypatch, name, fn):
    monkeypatch.setattr(O, name, fn)
    assert _fe_pins_fail(), f"planted mistake in {name} went unnoticed"


# ---------------------------------------------------------------------------------------
# shared bases: the HOSVD of the stacked pair densities
# ---------------------------------------------------------------------------------------
import tests.test_oracle_hosvd as HO  # noqa: E402


def _hosvd_pins_fail():
    checks = [HO.test_bases_are_q_orthonormal, HO.test_separable_orbitals_span_the_products,
              HO.test_gram_identity_gives_the_singular_values_and_subspaces,
              HO.test_orbital_rotation_leaves_the_bases]
    for c in checks:
        try:
            c()
        except (AssertionError, ValueError, IndexError, np.linalg.LinAlgError):
            return True
    return False


def test_unmutated_hosvd_passes():
    assert not _hosvd_pins_fail()


def _hosvd_mutant(mistake):
    """One plausible mistake in the shared decomposition."""
    def shared_hosvd(psi, q, ranks, targets=None):
        psi = np.asarray(psi, dtype=np.float64)
        N = psi.shape[0]
        tg = range(N) if targets is None else list(targets)
        sq = [np.sqrt(np.asarray(v, dtype=np.float64)) for v in q]
        scale = sq[0][:, None, None] * sq[1][None, :, None] * sq[2][None, None, :]
        if mistake == "unweighted":
            scale = np.ones_like(scale)
        U, sv = [], []
        for d in range(3):
            dd = (d + 1) % 3 if mistake == "wrong_mode" else d
            if mistake == "unique_pairs_only":
                cols = [O.unfold(scale * psi[i] * psi[j], dd) for i in tg for j in range(N) if j >= i]
            else:
                cols = [O.unfold(scale * psi[i] * psi[j], dd) for i in tg for j in range(N)]
            W_, s_, _ = np.linalg.svd(np.concatenate(cols, axis=1), full_matrices=False)
            if W_.shape[0] != len(q[d]):
                raise ValueError("mode extent")
            U.append(W_[:, :ranks[d]] / sq[d][:, None])
            sv.append(s_)
        return U, sv
    return shared_hosvd


@pytest.mark.parametrize("mistake", ["unweighted", "wrong_mode", "unique_pairs_only"])
def test_hosvd_mistakes_are_caught(monkeypatch, mistake):
    monkeypatch.setattr(O, "shared_hosvd", _hosvd_mutant(mistake))
    assert _hosvd_pins_fail(), f"planted mistake {mistake} in the shared decomposition went unnoticed"
