"""CPU FP64 oracle for the Tucker-tensor Fock-exchange hot path.

TEST INFRASTRUCTURE ONLY.  Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The GPU library
never calls it, shares no code with it, and must fail loudly rather than fall
back to it.

What it computes (Subramanian, Das & Gavini, arXiv 2401.04189, section
"Algorithmic implementation"), plainly, in float64, one orbital pair at a
time, in the order the paper gives the steps:

  * O1  1-D convolution matrices of each Gaussian term on the 1-D FE mesh:
        C_k[a,b] = int exp(-alpha_k (x_a - x')^2) N_b(x') dx'  with linear
        hat functions N_b, i.e. the precomputed node sums of eqs. `quadVal` /
        `discInteg` (interpolate to quadrature points, integrate against the
        Gaussian with Jacobian x weight, swap the sums), here evaluated by
        composite Gauss-Legendre quadrature.
  * O2  Projection bases V_d = diag(q_d) U_d and core matrices
        Chat_k^d = V_d^T C_k^d U_d.
  * O3  Per pair (i, j): pair density rho = psi_i psi_j (section "Convolution
        operation"), Tucker core G = rho x0 V0^T x1 V1^T x2 V2^T (eq.
        `TuckerDecompField`, with bases shared by all pairs), core-space kernel
        sum Phi = sum_k w_k G x0 Chat_k^0 x1 Chat_k^1 x2 Chat_k^2 (eqs. `gauss`
        and `final`), reconstruction phi = Phi x0 U0 x1 U1 x2 U2, and the pair
        energy e_ij = <G, Phi>_F = <rho, phi>_W.
  * O4  Exchange action Vx psi_i = - sum_j psi_j phi_ij (eqs.
        `ExchangeOperator`, `hadam`).
  * O5  Exchange energy E_x = -1/2 sum_{i,j} e_ij (the exact-exchange term of
        the functional S with the mixing fraction set to 1).
  * O6  Gradient dE_x/dpsi_i = 2 w (Vx psi_i) with w the 3-D grid weights.
  * O7  Adaptively compressed exchange (section "ACE implementation"): from
        W_i = Vx psi_i, the matrix M_ij = <psi_i, W_j>_W, its Cholesky factor
        M = -L L^T, the projection vectors xi_k = sum_i W_i (L^-1)_ki (eq.
        `eta`) and the operator V_ACE = -sum_k xi_k <xi_k, .>_W.
  * O9  Discretisation as the paper states it (section "Convolution
        operation" and the S-FE mesh of section "Creation of Structured FE
        basis"): 1-D meshes of cells with Lagrange elements of order p, the
        nodes of a cell at its Gauss-Lobatto-Legendre points, the end nodes
        of the domain held at zero; the convolution matrices of eqs.
        `quadVal` / `discInteg` for those elements; and the convolution
        evaluated at every 1-D node and reconstructed (eq. `final`):
        phi_ij = sum_k w_k G x0 (C_k^0 U0) x1 (C_k^1 U1) x2 (C_k^2 U2), with
        e_ij = <rho_ij, phi_ij>_W on the grid.
  * O10 Bases shared by all pairs (eq. `TuckerDecompField` with one set of
        factors for every pair): per mode, the leading left singular vectors
        of the mode-d unfolding of all pair densities rho_ij (i over the
        targets, j over all orbitals) stacked side by side, in the W inner
        product -- a higher-order SVD of the stack, each mode from the whole
        stack (not truncated sequentially).
  * O8  Per-pair bases (section "Convolution operation", eq.
        `TuckerDecompField` with factors f_ij, g_ij, h_ij of each pair): the
        sequentially truncated HOSVD of each pair density (modes 0, 1, 2 in
        turn: the leading left singular vectors of the current tensor's
        unfolding, then that mode truncated), in the W inner product; the
        pair's own core matrices Chat_k^{d,ij} = V_{ij,d}^T C_k^d U_{ij,d};
        then O3-O5 with those.

Where the paper is silent the oracle takes these readings, the same ones
the GPU path takes: uniform 1-D nodes, every node carrying a full linear hat
(a ghost node beyond each end), weights q = h; bases shared by all pairs and
q-orthonormal; the kernel sum evaluated in the Tucker core and then
back-projected (phi = P C P rho).  Per-pair bases (O8): the truncation runs
modes 0, 1, 2 in that order, in the W inner product (on uniform meshes the
nodal Frobenius norm the paper measures its error in, up to a constant
factor); O8 is pinned by its own identities (tests/test_oracle_sthosvd.py).  The Tucker-truncated
(r < n) result is pinned by brute force: on tiny graded grids it equals the
dense operator P C P (P the W-orthogonal projector onto the span of the
tensor-product bases, C the separable kernel) applied to rho; the full-rank
case is pinned to a dense 3-D kernel apply.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------------------
# O1: 1-D convolution matrices by composite Gauss-Legendre quadrature
# ---------------------------------------------------------------------------------------
_GL_ORDER = 12


def _ghosted(x):
    """Nodes with one ghost node added at each end, so that every real node
    carries a full hat function (the end nodes of the extended mesh are held at
    zero)."""
    x = np.asarray(x, dtype=np.float64)
    return np.concatenate([[2 * x[0] - x[1]], x, [2 * x[-1] - x[-2]]])


def conv_matrix_1d(x, alpha, order=_GL_ORDER):
    """C[a,b] = int exp(-alpha (x_a - t)^2) N_b(t) dt for linear hats N_b.

    Each hat is split into its rising and falling linear pieces; each piece is
    cut into m equal sub-intervals of width at most 1/(4 sqrt(alpha)) and
    integrated with an `order`-point Gauss-Legendre rule."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    xg = _ghosted(x)
    t_ref, w_ref = np.polynomial.legendre.leggauss(order)
    C = np.zeros((n, n))
    for b in range(n):
        left, mid, right = xg[b], xg[b + 1], xg[b + 2]
        for lo, hi, rising in ((left, mid, True), (mid, right, False)):
            width = hi - lo
            m = 1 if alpha <= 0 else max(1, int(math.ceil(width * 4.0 * math.sqrt(alpha))))
            edges = lo + width * np.arange(m + 1) / m
            a_ = edges[:-1, None]
            b_ = edges[1:, None]
            t = 0.5 * (b_ - a_) * t_ref[None, :] + 0.5 * (a_ + b_)          # (m, order)
            wt = 0.5 * (b_ - a_) * w_ref[None, :]
            hat = (t - lo) / width if rising else (hi - t) / width
            t = t.reshape(-1)
            wh = (wt * hat).reshape(-1)
            C[:, b] += np.exp(-alpha * (x[:, None] - t[None, :]) ** 2) @ wh
    return C


def conv_matrices(x, alphas):
    return np.stack([conv_matrix_1d(x, float(a)) for a in alphas])


# ---------------------------------------------------------------------------------------
# O2: projection bases and core matrices
# ---------------------------------------------------------------------------------------
class Setup:
    """Per-system precomputation: V_d, C_k^d and Chat_k^d for d = 0, 1, 2."""

    def __init__(self, x, q, U, w, alpha, C=None):
        self.x = [np.asarray(v, dtype=np.float64) for v in x]
        self.q = [np.asarray(v, dtype=np.float64) for v in q]
        self.U = [np.asarray(u, dtype=np.float64) for u in U]
        self.w = np.asarray(w, dtype=np.float64)
        self.alpha = np.asarray(alpha, dtype=np.float64)
        self.V = [self.q[d][:, None] * self.U[d] for d in range(3)]
        if C is None:
            cache = {}
            C = []
            for d in range(3):
                key = self.x[d].tobytes()
                if key not in cache:
                    cache[key] = conv_matrices(self.x[d], self.alpha)
                C.append(cache[key])
        self.C = [np.asarray(c, dtype=np.float64) for c in C]
        self.Chat = [np.einsum("ap,kab,bs->kps", self.V[d], self.C[d], self.U[d]) for d in range(3)]

    @classmethod
    def from_system(cls, sysm):
        return cls(sysm.grid.x, sysm.grid.q, sysm.U, sysm.w, sysm.alpha)


# ---------------------------------------------------------------------------------------
# O3: one pair
# ---------------------------------------------------------------------------------------
def mode_product(T, M, d):
    """(T x_d M)[.., i', ..] = sum_i M[i', i] T[.., i, ..]."""
    return np.moveaxis(np.tensordot(M, T, axes=(1, d)), 0, d)


def project(rho, V):
    G = rho
    for d in range(3):
        G = mode_product(G, V[d].T, d)
    return G


def core_sum(G, w, Chat):
    Phi = np.zeros_like(G)
    for k in range(len(w)):
        T = G
        for d in range(3):
            T = mode_product(T, Chat[d][k], d)
        Phi += w[k] * T
    return Phi


def reconstruct(Phi, U):
    phi = Phi
    for d in range(3):
        phi = mode_product(phi, U[d], d)
    return phi


def pair(psi_i, psi_j, st: Setup):
    """(phi_ij, e_ij, G, Phi) for one pair."""
    rho = psi_i * psi_j
    G = project(rho, st.V)
    Phi = core_sum(G, st.w, st.Chat)
    phi = reconstruct(Phi, st.U)
    e = float(np.sum(G * Phi))
    return phi, e, G, Phi


# ---------------------------------------------------------------------------------------
# O4 / O5: exchange action and energy
# ---------------------------------------------------------------------------------------
def apply(psi, st: Setup, mode="symmetric", i0=0, Ni=None, want_vx=True, pairs_out=None):
    """Vx psi and E_x.

    mode="symmetric": all unique pairs i <= j of the N orbitals; each unique pair
    feeds target i (times psi_j) and target j (times psi_i).  Returns Vx psi for
    all N orbitals and E_x = -1/2 sum over all ordered pairs.

    mode="block": targets i in [i0, i0+Ni) against all N sources; returns
    Vx psi for the Ni targets and E_x = -1/2 sum_{i in block} sum_j e_ij.

    When `pairs_out` is a dict it receives e_ij keyed by (i, j)."""
    psi = np.asarray(psi, dtype=np.float64)
    N = psi.shape[0]
    if mode == "symmetric":
        targets = list(range(N))
        vx = np.zeros_like(psi) if want_vx else None
        ex = 0.0
        for i in range(N):
            for j in range(i, N):
                phi, e, _, _ = pair(psi[i], psi[j], st)
                if pairs_out is not None:
                    pairs_out[(i, j)] = e
                if want_vx:
                    vx[i] -= psi[j] * phi
                    if j != i:
                        vx[j] -= psi[i] * phi
                ex += -0.5 * e if i == j else -e
        return vx, ex
    Ni = N - i0 if Ni is None else Ni
    targets = list(range(i0, i0 + Ni))
    vx = np.zeros((Ni,) + psi.shape[1:]) if want_vx else None
    ex = 0.0
    for t, i in enumerate(targets):
        for j in range(N):
            phi, e, _, _ = pair(psi[i], psi[j], st)
            if pairs_out is not None:
                pairs_out[(i, j)] = e
            if want_vx:
                vx[t] -= psi[j] * phi
            ex += -0.5 * e
    return vx, ex


def apply_target(psi, st: Setup, i, sources=None):
    """Vx psi_i for one target against the given sources (all by default)."""
    psi = np.asarray(psi, dtype=np.float64)
    sources = range(psi.shape[0]) if sources is None else sources
    out = np.zeros(psi.shape[1:])
    for j in sources:
        phi, _, _, _ = pair(psi[i], psi[j], st)
        out -= psi[j] * phi
    return out


def pair_energy(psi, st: Setup, i, j):
    return pair(np.asarray(psi[i], dtype=np.float64), np.asarray(psi[j], dtype=np.float64), st)[1]


# ---------------------------------------------------------------------------------------
# O8: per-pair bases by the sequentially truncated HOSVD
# ---------------------------------------------------------------------------------------
def unfold(T, d):
    """Mode-d unfolding: rows = index d, columns = the other indices in C order."""
    return np.moveaxis(T, d, 0).reshape(T.shape[d], -1)


def sthosvd(rho, q, ranks):
    """Sequentially truncated HOSVD of one field in the W inner product.

    The field is scaled by sqrt(q_d) along every mode (so the Frobenius norm
    of the scaled tensor is the W-norm of the field).  Modes 0, 1, 2 in turn:
    the leading r_d left singular vectors Ut_d of the unfolding of the
    current tensor, then the current tensor is replaced by its product with
    Ut_d^T along mode d.  Returns (U, G, discarded): q-orthonormal factors
    U_d = Ut_d / sqrt(q_d) (U_d^T diag(q_d) U_d = I), the core G, and per mode
    the squared singular values that were cut off."""
    X = np.asarray(rho, dtype=np.float64)
    for d in range(3):
        X = mode_product(X, np.diag(np.sqrt(q[d])), d)
    U, cut = [], []
    for d in range(3):
        W_, sv, _ = np.linalg.svd(unfold(X, d), full_matrices=False)
        Ut = W_[:, :ranks[d]]
        cut.append(sv[ranks[d]:] ** 2)
        X = mode_product(X, Ut.T, d)
        U.append(Ut / np.sqrt(q[d])[:, None])
    return U, X, cut


def pair_sthosvd(psi_i, psi_j, st: Setup, ranks):
    """(phi_ij, e_ij, G, Phi, U) for one pair with its own bases: O8 then the
    kernel sum with the pair's core matrices and the reconstruction in its
    bases."""
    rho = psi_i * psi_j
    U, G, _ = sthosvd(rho, st.q, ranks)
    V = [st.q[d][:, None] * U[d] for d in range(3)]
    Chat = [np.einsum("ap,kab,bs->kps", V[d], st.C[d], U[d]) for d in range(3)]
    Phi = core_sum(G, st.w, Chat)
    phi = reconstruct(Phi, U)
    return phi, float(np.sum(G * Phi)), G, Phi, U


def apply_sthosvd(psi, st: Setup, ranks, mode="symmetric", i0=0, Ni=None, pairs_out=None):
    """Vx psi and E_x with per-pair bases (the exchange action of O4 and the
    energy of O5, each pair through pair_sthosvd)."""
    psi = np.asarray(psi, dtype=np.float64)
    N = psi.shape[0]
    if mode == "symmetric":
        vx = np.zeros_like(psi)
        ex = 0.0
        for i in range(N):
            for j in range(i, N):
                phi, e, _, _, _ = pair_sthosvd(psi[i], psi[j], st, ranks)
                if pairs_out is not None:
                    pairs_out[(i, j)] = e
                vx[i] -= psi[j] * phi
                if j != i:
                    vx[j] -= psi[i] * phi
                ex += -0.5 * e if i == j else -e
        return vx, ex
    Ni = N - i0 if Ni is None else Ni
    vx = np.zeros((Ni,) + psi.shape[1:])
    ex = 0.0
    for t, i in enumerate(range(i0, i0 + Ni)):
        for j in range(N):
            phi, e, _, _, _ = pair_sthosvd(psi[i], psi[j], st, ranks)
            if pairs_out is not None:
                pairs_out[(i, j)] = e
            vx[t] -= psi[j] * phi
            ex += -0.5 * e
    return vx, ex


# ---------------------------------------------------------------------------------------
# O10: shared bases, the HOSVD of the stacked pair densities
# ---------------------------------------------------------------------------------------
def shared_hosvd(psi, q, ranks, targets=None):
    """(U, sv): q-orthonormal bases U_d (n_d x r_d, U_d^T diag(q_d) U_d = I)
    spanning the leading left singular vectors of the mode-d unfolding of the
    stack of every sqrt(w)-scaled pair density psi_i psi_j, i over `targets`
    (all orbitals when None), j over all orbitals; sv[d] holds all singular
    values of that unfolding, descending.  Each pair density is formed
    explicitly: small cases only."""
    psi = np.asarray(psi, dtype=np.float64)
    N = psi.shape[0]
    tg = range(N) if targets is None else list(targets)
    sq = [np.sqrt(np.asarray(v, dtype=np.float64)) for v in q]
    scale = sq[0][:, None, None] * sq[1][None, :, None] * sq[2][None, None, :]
    U, sv = [], []
    for d in range(3):
        cols = [unfold(scale * psi[i] * psi[j], d) for i in tg for j in range(N)]
        W_, s_, _ = np.linalg.svd(np.concatenate(cols, axis=1), full_matrices=False)
        U.append(W_[:, :ranks[d]] / sq[d][:, None])
        sv.append(s_)
    return U, sv


# ---------------------------------------------------------------------------------------
# O9: Lagrange elements of order p, their convolution matrices, and collocation
# ---------------------------------------------------------------------------------------
def gll_points(p):
    """The p + 1 Gauss-Lobatto-Legendre points of [-1, 1] (the ends and the
    roots of P_p'), and their quadrature weights 2 / (p (p+1) P_p(s)^2)."""
    Pp = np.polynomial.legendre.Legendre.basis(p)
    inner = np.sort(Pp.deriv().roots().real) if p > 1 else np.array([])
    s = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (p * (p + 1) * Pp(s) ** 2)
    return s, w


def fe_mesh_1d(edges, p):
    """Nodes and nodal quadrature weights of a 1-D mesh of cells
    [edges[e], edges[e+1]] with order-p Lagrange elements at the GLL points of
    each cell; the two end nodes of the domain carry zero (Dirichlet) and are
    not unknowns.  Returns (x, q, cells): the n = ncell p - 1 unknown nodes,
    their weights (GLL weight times half the cell length, summed over the
    cells a node belongs to), and per cell the node indices of its p + 1
    points (-1 for a held end node)."""
    edges = np.asarray(edges, dtype=np.float64)
    s, w = gll_points(p)
    nc = len(edges) - 1
    xs = np.zeros(nc * p + 1)
    qs = np.zeros(nc * p + 1)
    cells = []
    for e in range(nc):
        lo, hi = edges[e], edges[e + 1]
        idx = e * p + np.arange(p + 1)
        xs[idx] = lo + 0.5 * (s + 1.0) * (hi - lo)
        qs[idx] += w * 0.5 * (hi - lo)
        cells.append(idx - 1)
    cells = [np.where((c < 0) | (c >= nc * p - 1), -1, c) for c in cells]
    return xs[1:-1], qs[1:-1], cells


def lagrange_eval(nodes, k, t):
    """The k-th Lagrange polynomial of `nodes` at points t."""
    out = np.ones_like(t)
    for m, xm in enumerate(nodes):
        if m != k:
            out *= (t - xm) / (nodes[k] - xm)
    return out


def conv_matrix_fe(edges, p, alpha, order=_GL_ORDER):
    """C[a, b] = int exp(-alpha (x_a - t)^2) N_b(t) dt for the order-p
    Lagrange basis N_b of fe_mesh_1d (eqs. `quadVal`, `discInteg`), by
    composite Gauss-Legendre quadrature on every cell, cut into pieces of
    width at most 1/(4 sqrt(alpha))."""
    x, _, cells = fe_mesh_1d(edges, p)
    edges = np.asarray(edges, dtype=np.float64)
    s, _ = gll_points(p)
    t_ref, w_ref = np.polynomial.legendre.leggauss(order)
    C = np.zeros((len(x), len(x)))
    for e, idx in enumerate(cells):
        lo, hi = edges[e], edges[e + 1]
        nodes = lo + 0.5 * (s + 1.0) * (hi - lo)
        width = hi - lo
        m = 1 if alpha <= 0 else max(1, int(math.ceil(width * 4.0 * math.sqrt(alpha))))
        cuts = lo + width * np.arange(m + 1) / m
        a_, b_ = cuts[:-1, None], cuts[1:, None]
        t = (0.5 * (b_ - a_) * t_ref[None, :] + 0.5 * (a_ + b_)).reshape(-1)
        wt = (0.5 * (b_ - a_) * w_ref[None, :]).reshape(-1)
        kern = np.exp(-alpha * (x[:, None] - t[None, :]) ** 2) * wt[None, :]
        for k, b in enumerate(idx):
            if b >= 0:
                C[:, b] += kern @ lagrange_eval(nodes, k, t)
    return C


def pair_collocation(psi_i, psi_j, st: Setup):
    """(phi_ij, e_ij) with the convolution evaluated at every 1-D node and
    reconstructed: phi = sum_k w_k G x0 (C_k^0 U0) x1 (C_k^1 U1) x2 (C_k^2 U2),
    e_ij = <rho_ij, phi>_W (grid sum)."""
    rho = psi_i * psi_j
    G = project(rho, st.V)
    phi = np.zeros_like(rho)
    for k in range(len(st.w)):
        T = G
        for d in range(3):
            T = mode_product(T, st.C[d][k] @ st.U[d], d)
        phi += st.w[k] * T
    return phi, float((weights3d(st.q) * rho * phi).sum())


def apply_collocation(psi, st: Setup, mode="symmetric", i0=0, Ni=None, pairs_out=None):
    """Vx psi and E_x with the collocation form of every pair (O4, O5)."""
    psi = np.asarray(psi, dtype=np.float64)
    N = psi.shape[0]
    if mode == "symmetric":
        vx = np.zeros_like(psi)
        ex = 0.0
        for i in range(N):
            for j in range(i, N):
                phi, e = pair_collocation(psi[i], psi[j], st)
                if pairs_out is not None:
                    pairs_out[(i, j)] = e
                vx[i] -= psi[j] * phi
                if j != i:
                    vx[j] -= psi[i] * phi
                ex += -0.5 * e if i == j else -e
        return vx, ex
    Ni = N - i0 if Ni is None else Ni
    vx = np.zeros((Ni,) + psi.shape[1:])
    ex = 0.0
    for t, i in enumerate(range(i0, i0 + Ni)):
        for j in range(N):
            phi, e = pair_collocation(psi[i], psi[j], st)
            if pairs_out is not None:
                pairs_out[(i, j)] = e
            vx[t] -= psi[j] * phi
            ex += -0.5 * e
    return vx, ex


# ---------------------------------------------------------------------------------------
# O6: gradient
# ---------------------------------------------------------------------------------------
def weights3d(q):
    return q[0][:, None, None] * q[1][None, :, None] * q[2][None, None, :]


def gradient(psi, st: Setup):
    """dE_x/dpsi (raw grid values) = 2 w (Vx psi), symmetric mode over all orbitals."""
    vx, _ = apply(psi, st, mode="symmetric")
    return 2.0 * weights3d(st.q)[None] * vx


def energy_change_one_orbital(psi, st: Setup, m, delta):
    """E_x(psi with psi_m += delta) - E_x(psi), from the 2N-1 pairs that involve
    orbital m only (all other pair energies are unchanged)."""
    psi = np.asarray(psi, dtype=np.float64)
    N = psi.shape[0]
    new = psi[m] + delta

    def contrib(pm):
        tot = 0.0
        for j in range(N):
            pj = pm if j == m else psi[j]
            _, e, _, _ = pair(pm, pj, st)
            tot += -0.5 * e if j == m else -e
        return tot

    return contrib(new) - contrib(psi[m])


# ---------------------------------------------------------------------------------------
# O7: adaptively compressed exchange (section "ACE implementation")
# ---------------------------------------------------------------------------------------
def ace_build(psi, W, q):
    """The ACE projection vectors from the orbitals psi_i and their exchange
    actions W_i = Vx psi_i (arrays N x n0 x n1 x n2):

        M_ij = <psi_i, W_j>_W            (the paper's integral, on the grid)
        M = -L L^T                       (Cholesky factor of -M)
        xi_k = sum_i W_i (L^{-1})_{ki}

    Returns (M, L, xi)."""
    N = psi.shape[0]
    w3 = weights3d(q).reshape(-1)
    P = psi.reshape(N, -1)
    Wm = W.reshape(N, -1)
    M = P @ (Wm * w3[None, :]).T
    L = np.linalg.cholesky(-M)
    Linv = np.linalg.inv(L)
    xi = (Linv @ Wm).reshape(W.shape)
    return M, L, xi


def ace_apply(xi, q, phi):
    """V_ACE phi_j = - sum_k xi_k <xi_k, phi_j>_W for trial functions phi
    (Nphi x n0 x n1 x n2)."""
    w3 = weights3d(q).reshape(-1)
    X = xi.reshape(xi.shape[0], -1)
    F = phi.reshape(phi.shape[0], -1)
    C = X @ (F * w3[None, :]).T          # C[k, j] = <xi_k, phi_j>_W
    return (-(C.T @ X)).reshape(phi.shape)


# ---------------------------------------------------------------------------------------
# references used to pin the oracle (dense, brute force)
# ---------------------------------------------------------------------------------------
def dense_kernel_apply(rho, w, C):
    """sum_k w_k (C_k^0 (x) C_k^1 (x) C_k^2) rho with the dense 3-D kernel matrix
    formed explicitly (tiny grids only)."""
    n = rho.shape
    out = np.zeros(rho.size)
    for k in range(len(w)):
        A = np.kron(np.kron(C[0][k], C[1][k]), C[2][k])
        out += w[k] * (A @ rho.reshape(-1))
    return out.reshape(n)
