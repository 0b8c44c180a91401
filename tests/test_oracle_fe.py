"""Pins of the oracle's paper-literal discretisation step (order-p Lagrange
elements at Gauss-Lobatto-Legendre points, their Gaussian convolution
matrices, and the collocation form phi = C P rho) to things other than the
oracle itself:

  * the GLL rule of order p integrates polynomials of degree 2p - 1 exactly
    and its nodes are the ends and the roots of P_p';
  * at p = 1 on the ghost-cell mesh the construction is the linear-hat one
    (itself pinned to an erf closed form);
  * the convolution matrix reproduces every polynomial of degree <= p that
    vanishes at the domain ends: sum_b C[a, b] f(x_b) equals the integral of
    exp(-alpha (x_a - t)^2) f(t), evaluated here by mpmath quadrature at 30
    digits, on a graded mesh;
  * at full rank the collocation form equals the dense kernel apply (which is
    then also the Galerkin form).
No GPU.
"""
import mpmath
import numpy as np
import pytest

from oracle import txe_oracle as O
from paper_2401_04189_amd import workloads as W


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_gll_rule(p):
    s, w = O.gll_points(p)
    assert len(s) == p + 1 and abs(s[0] + 1) < 1e-15 and abs(s[-1] - 1) < 1e-15
    if p > 1:
        dP = np.polynomial.legendre.Legendre.basis(p).deriv()
        assert np.abs(dP(s[1:-1])).max() <= 1e-12
    for m in range(2 * p):
        exact = (1 - (-1) ** (m + 1)) / (m + 1)
        assert abs((w * s ** m).sum() - exact) <= 1e-14


def test_order_one_is_the_linear_hat_construction():
    n, L = 12, 3.0
    h = 2 * L / (n - 1)
    edges = np.linspace(-L - h, L + h, n + 2)
    x, q, _ = O.fe_mesh_1d(edges, 1)
    assert np.abs(x - np.linspace(-L, L, n)).max() <= 1e-14
    assert np.abs(q - h).max() <= 1e-14
    for alpha in (0.0, 0.8, 40.0):
        assert np.abs(O.conv_matrix_fe(edges, 1, alpha) - O.conv_matrix_1d(x, alpha)).max() <= 1e-14


def _graded_edges():
    # finer cells near 0.4 (a refined region), coarser towards the ends
    return np.array([-4.0, -2.5, -1.4, -0.6, -0.1, 0.2, 0.4, 0.6, 0.9, 1.5, 2.6, 4.0])


@pytest.mark.parametrize("p", [4, 5, 6])
@pytest.mark.parametrize("alpha", [0.3, 30.0, 3000.0])
def test_convolution_matrix_reproduces_polynomials(p, alpha):
    edges = _graded_edges()
    a_, b_ = edges[0], edges[-1]
    x, q, _ = O.fe_mesh_1d(edges, p)
    C = O.conv_matrix_fe(edges, p, alpha)
    mpmath.mp.dps = 30
    rows = [0, 3, len(x) // 2, len(x) - 1]
    for mdeg in range(p - 1):                       # f = (t - a)(b - t) t^m, degree m + 2 <= p
        f = lambda t, m=mdeg: (t - a_) * (b_ - t) * t ** m  # noqa: E731
        fx = f(x)
        got = C @ fx
        scale = float(np.abs(got).max())
        for r in rows:
            xa = mpmath.mpf(float(x[r]))
            ref = mpmath.quad(lambda t: mpmath.exp(-alpha * (xa - t) ** 2) * f(t),
                              list(map(mpmath.mpf, edges.tolist())) + [])
            assert abs(got[r] - float(ref)) <= 1e-13 * max(scale, 1e-30), (p, alpha, mdeg, r)
        # the nodal weights integrate f exactly (GLL exactness, degree <= 2p - 1 per cell)
        exact = float(mpmath.quad(f, [a_, b_]))
        assert abs((q * fx).sum() - exact) <= 1e-13 * float((q * np.abs(fx)).sum())


def test_collocation_at_full_rank_is_the_dense_kernel():
    g = W.uniform_grid(8, 3.0)
    psi, _ = W.make_orbitals(g, 2, 2, (0.5, 2.0), seed=91, box=1.0)
    w, a = W.exp_sum(5)
    st = O.Setup(g.x, g.q, W.full_rank_bases(g, 4), w, a)
    p = psi.numpy()
    vx, ex = O.apply_collocation(p, st)
    vg, eg = O.apply(p, st)
    ref = np.zeros_like(p)
    for i in range(2):
        for j in range(2):
            ref[i] -= p[j] * O.dense_kernel_apply(p[i] * p[j], w, st.C)
    assert np.abs(vx - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.abs(vg - ref).max() <= 1e-12 * np.abs(ref).max()
    assert abs(ex - eg) <= 1e-12 * abs(eg)


def test_collocation_differs_from_galerkin_below_full_rank_and_converges():
    s = W.small_system(n=12, L=4.0, N=2, r=5, K=6, seed=92)
    st = O.Setup.from_system(s)
    p = s.psi.numpy()
    vx, ex = O.apply_collocation(p, st)
    vg, eg = O.apply(p, st)
    assert abs(ex - eg) > 1e-10 * abs(eg)          # a real difference at r < n
    # with more rank the two forms approach each other
    gaps = []
    for r in (4, 7, 10):
        U = W.hosvd_bases(s.psi, s.grid, (r, r, r))
        str_ = O.Setup(s.grid.x, s.grid.q, U, s.w, s.alpha)
        gaps.append(abs(O.apply_collocation(p, str_)[1] - O.apply(p, str_)[1]))
    assert gaps[2] < gaps[0]
