"""The library's host builder of order-p Lagrange elements (GLL nodes, nodal
weights, Gaussian convolution matrices; txe_fe_mesh_1d / txe_fe_conv_matrices)
against the oracle's independent construction, and its argument checks.
Host code only: no GPU."""
import numpy as np
import pytest

from oracle import txe_oracle as O
from paper_2401_04189_amd import txe, workloads as W

GRADED = np.array([-4.0, -2.5, -1.4, -0.6, -0.1, 0.2, 0.4, 0.6, 0.9, 1.5, 2.6, 4.0])


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_mesh_matches_the_oracle(p):
    x, q = txe.fe_mesh_1d(GRADED, p)
    xo, qo, _ = O.fe_mesh_1d(GRADED, p)
    assert len(x) == (len(GRADED) - 1) * p - 1
    assert np.abs(x - xo).max() <= 2e-15 * np.abs(xo).max()
    assert np.abs(q - qo).max() <= 2e-15 * qo.max()


@pytest.mark.parametrize("p", [1, 4, 5, 6])
def test_convolution_matrices_match_the_oracle(p):
    alphas = [0.0, 1e-7, 0.3, 30.0, 2981.0]
    C = txe.fe_conv_matrices(GRADED, p, alphas)
    for k, a in enumerate(alphas):
        Co = O.conv_matrix_fe(GRADED, p, a)
        assert np.abs(C[k] - Co).max() <= 1e-13 * np.abs(Co).max(), (p, a)


def test_order_one_on_the_ghost_mesh_is_the_linear_hat_setup():
    n, L = 16, 4.0
    g = W.uniform_grid(n, L)
    h = 2 * L / (n - 1)
    edges = np.linspace(-L - h, L + h, n + 2)
    for a in (0.0, 0.5, 50.0):
        C = txe.fe_conv_matrices(edges, 1, [a])[0]
        assert np.abs(C - txe.conv_matrix_1d(g.x[0], a)).max() <= 1e-14


def test_adaptive_mesh_feeds_a_valid_grid():
    edges = W.adaptive_edges(L=8.0, bms=4.0, msna=0.6, centres=[-1.3, 2.0], ball=1.5, p=5)
    p = 5
    n = (len(edges) - 1) * p - 1
    assert n % 4 == 0
    widths = np.diff(edges)
    near = np.array([min(abs(0.5 * (lo + hi) - c) for c in (-1.3, 2.0)) for lo, hi in zip(edges[:-1], edges[1:])])
    assert widths[near <= 1.0].max() <= 0.6 + 1e-12          # refined near the centres
    assert widths.max() <= 4.0 + 1e-12                       # never coarser than the base size
    assert np.all(widths[1:] / widths[:-1] <= 2.0 + 1e-12)   # neighbours differ by at most 2x
    assert np.all(widths[:-1] / widths[1:] <= 2.0 + 1e-12)
    x, q = txe.fe_mesh_1d(edges, p)
    # the nodal weights and the two held end nodes' weights add up to the domain length
    w_end = 2.0 / (p * (p + 1))
    total = q.sum() + w_end * 0.5 * (widths[0] + widths[-1])
    assert abs(total - 16.0) <= 1e-13 * 16.0


@pytest.mark.parametrize("edges,p,status", [
    ([0.0, 1.0, 1.0], 2, 1),      # not increasing
    ([0.0, np.nan, 2.0], 2, 1),   # not finite
    ([0.0, 1.0], 0, 2),           # order out of range
    ([0.0, 1.0], 11, 2),
    ([0.0, 1.0], 1, 2),           # no unknown node (n = 0)
])
def test_bad_arguments(edges, p, status):
    with pytest.raises(txe.TxeError) as ei:
        txe.fe_mesh_1d(edges, p)
    assert ei.value.status == status
    with pytest.raises(txe.TxeError):
        txe.fe_conv_matrices(np.array([0.0, 1.0, 2.0]), 2, [-1.0])
