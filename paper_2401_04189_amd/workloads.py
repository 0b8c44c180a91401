"""Seeded synthetic inputs for the Tucker-tensor exchange hot path.

This module only *creates inputs*: tensor-product grids with their 1-D
quadrature weights, Gaussian-type orbitals placed on cluster geometries,
their Loewdin orthonormalisation in the grid inner product, the
exponential-sum coefficients (w_k, alpha_k) that stand in for 1/r, and
q-orthonormal per-mode Tucker bases U_d from a higher-order SVD of the stacked
pair densities.  It holds none of the exchange arithmetic itself (no 1-D
convolution matrices, no projection, no kernel sums, no back-projection):
the CPU oracle and the GPU library each do that part on their own, from what
this module returns.

Workload shapes follow the paper's benchmark systems only in outline (Pt
clusters on an fcc lattice, a TiO2 cluster on rutile sites; paper section
"Results and Discussion"); the orbitals are seeded Gaussians, not DFT states.

Everything is float64.  Large configurations can be generated on a GPU by
passing ``device="cuda"``; the arithmetic is the same torch code either way.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

DT = torch.float64


# --------------------------------------------------------------------------------------
# grid and kernel coefficients
# --------------------------------------------------------------------------------------
@dataclass
class Grid:
    """Tensor-product grid: per-mode 1-D nodes x[d] and quadrature weights q[d].

    Nodes are uniform on [-L, L] (n nodes, spacing h = 2L/(n-1)); every node
    carries weight h, i.e. the nodes are the interior nodes of a uniform
    linear finite-element mesh on [-L-h, L+h] whose end nodes are clamped to
    zero, so each node owns a full hat function (paper section "Creation of
    Structured FE basis": tensor product of three 1-D meshes, lexicographic
    numbering, only 1-D coordinates stored).
    """

    n: tuple
    L: tuple
    x: list
    q: list

    @property
    def shape(self):
        return tuple(self.n)

    @property
    def h(self):
        return tuple(2.0 * L / (n - 1) for n, L in zip(self.n, self.L))

    def weights3d(self, device="cpu"):
        q = [torch.as_tensor(v, dtype=DT, device=device) for v in self.q]
        return q[0][:, None, None] * q[1][None, :, None] * q[2][None, None, :]


def graded_grid(n, L, stretch=1.5) -> Grid:
    """Non-uniform nodes x = L sinh(stretch t) / sinh(stretch), t uniform on
    [-1, 1] (fine at the centre, coarse at the ends); q = the integral of each
    node's linear hat, with one mirrored ghost node beyond each end."""
    n = tuple(int(v) for v in (n if isinstance(n, (tuple, list)) else (n, n, n)))
    L = tuple(float(v) for v in (L if isinstance(L, (tuple, list)) else (L, L, L)))
    xs, qs = [], []
    for nd, Ld in zip(n, L):
        t = np.linspace(-1.0, 1.0, nd)
        x = Ld * np.sinh(stretch * t) / np.sinh(stretch)
        xg = np.concatenate([[2 * x[0] - x[1]], x, [2 * x[-1] - x[-2]]])
        xs.append(x)
        qs.append(0.5 * (xg[2:] - xg[:-2]))
    return Grid(n=n, L=L, x=xs, q=qs)


def uniform_grid(n, L) -> Grid:
    n = tuple(int(v) for v in (n if isinstance(n, (tuple, list)) else (n, n, n)))
    L = tuple(float(v) for v in (L if isinstance(L, (tuple, list)) else (L, L, L)))
    xs, qs = [], []
    for nd, Ld in zip(n, L):
        x = np.linspace(-Ld, Ld, nd)
        h = 2.0 * Ld / (nd - 1)
        xs.append(x)
        qs.append(np.full(nd, h))
    return Grid(n=n, L=L, x=xs, q=qs)


def adaptive_edges(L, bms, msna, centres, ball, p):
    """Cell edges of a 1-D mesh on [-L, L] made the way the paper builds its
    structured FE mesh (section "Creation of Structured FE basis"): start
    from uniform cells no larger than the base mesh size `bms`, then bisect
    every cell that reaches within `ball` of an atom coordinate in `centres`
    until those cells are no larger than the mesh size near the atoms `msna`.
    Two steps are this generator's own: neighbouring cells are balanced to a
    width ratio of at most 2 (the coarser one is bisected), and the widest
    cells are bisected until the mesh has n = ncells p - 1 unknowns with n a
    multiple of 4 (the library's grid extents), which needs p odd."""
    if p % 2 == 0:
        raise ValueError("n = ncells * p - 1 is odd for even p; use an odd order")
    nc = max(1, int(math.ceil(2.0 * L / bms - 1e-12)))
    edges = list(np.linspace(-L, L, nc + 1))
    near = lambda lo, hi: any(lo <= c + ball and hi >= c - ball for c in centres)  # noqa: E731
    changed = True
    while changed:
        changed, out = False, [edges[0]]
        for lo, hi in zip(edges[:-1], edges[1:]):
            if hi - lo > msna and near(lo, hi):
                out.append(0.5 * (lo + hi))
                changed = True
            out.append(hi)
        edges = out
    while True:
        w = np.diff(edges)
        split = [i for i in range(len(w)) if (i > 0 and w[i] > 2.0 * w[i - 1] * (1 + 1e-12))
                 or (i + 1 < len(w) and w[i] > 2.0 * w[i + 1] * (1 + 1e-12))]
        if not split:
            break
        for i in sorted(split, reverse=True):
            edges.insert(i + 1, 0.5 * (edges[i] + edges[i + 1]))
    while ((len(edges) - 1) * p - 1) % 4 != 0:
        w = np.diff(edges)
        i = int(np.argmax(w))
        edges.insert(i + 1, 0.5 * (edges[i] + edges[i + 1]))
    return np.array(edges)


def grid_from_nodes(xs, qs) -> Grid:
    """A grid from given per-mode nodes and weights (e.g. of an FE mesh)."""
    xs = [np.asarray(v, dtype=np.float64) for v in xs]
    qs = [np.asarray(v, dtype=np.float64) for v in qs]
    return Grid(n=tuple(len(v) for v in xs), L=tuple(float(max(abs(v[0]), abs(v[-1]))) for v in xs), x=xs, q=qs)


def exp_sum(K, s_lo=-8.0, s_hi=4.0):
    """Coefficients of 1/r ~ sum_k w_k exp(-alpha_k r^2).

    Sinc (trapezoid) quadrature of 1/r = 2/sqrt(pi) * int exp(-r^2 e^{2s}) e^s ds
    on K equally spaced nodes s_k in [s_lo, s_hi] (both ends included, full
    weight at both ends): w_k = 2/sqrt(pi) * h_s * e^{s_k}, alpha_k = e^{2 s_k}.
    The paper uses a T-term Gaussian fit of 1/r (paper eq. `gauss`, T = 35);
    its coefficients are not printed, so these stand in for them.
    """
    K = int(K)
    if K == 1:  # one node at the middle of the interval, carrying all of it
        hs = s_hi - s_lo
        s = np.array([0.5 * (s_lo + s_hi)])
    else:
        hs = (s_hi - s_lo) / (K - 1)
        s = s_lo + hs * np.arange(K)
    w = 2.0 / math.sqrt(math.pi) * hs * np.exp(s)
    alpha = np.exp(2.0 * s)
    return w, alpha


# --------------------------------------------------------------------------------------
# geometries
# --------------------------------------------------------------------------------------
def fcc_sites(count, nn=2.8):
    """The `count` fcc lattice sites nearest the origin (nearest-neighbour
    distance `nn` bohr).  Ties in distance are cut by lexicographic order of the
    integer lattice coordinates (i, j, k), i + j + k even."""
    R = 1
    while True:
        rng_ = np.arange(-R, R + 1)
        I, J, Kk = np.meshgrid(rng_, rng_, rng_, indexing="ij")
        m = ((I + J + Kk) % 2) == 0
        pts = np.stack([I[m], J[m], Kk[m]], axis=1)
        if len(pts) >= 8 * count + 64:
            break
        R += 1
    d2 = (pts ** 2).sum(1)
    order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0], d2))
    pts = pts[order][:count]
    return pts.astype(np.float64) * (nn / math.sqrt(2.0))


def rutile_sites(count=310, rmax=12.0, a=8.68, c=5.59, u=0.305):
    """The `count` rutile (TiO2) sites nearest a Ti site at the origin, scaled
    uniformly so that the farthest kept site lies at most `rmax` bohr away."""
    basis = np.array([
        [0.0, 0.0, 0.0], [0.5, 0.5, 0.5],                      # Ti
        [u, u, 0.0], [-u, -u, 0.0],                             # O
        [0.5 + u, 0.5 - u, 0.5], [0.5 - u, 0.5 + u, 0.5],       # O
    ])
    cells = []
    R = 4
    rr = np.arange(-R, R + 1)
    for i in rr:
        for j in rr:
            for k in rr:
                cells.append(basis + np.array([i, j, k], dtype=np.float64))
    frac = np.concatenate(cells, axis=0)
    xyz = frac * np.array([a, a, c])
    d = np.sqrt((xyz ** 2).sum(1))
    key = np.round(xyz, 9)
    order = np.lexsort((key[:, 2], key[:, 1], key[:, 0], np.round(d, 9)))
    xyz = xyz[order][:count]
    dmax = np.sqrt((xyz ** 2).sum(1)).max()
    if dmax > rmax:
        xyz = xyz * (rmax / dmax)
    return xyz


# --------------------------------------------------------------------------------------
# orbitals
# --------------------------------------------------------------------------------------
@dataclass
class GaussSpec:
    centres: np.ndarray   # (N, ng, 3)
    exps: np.ndarray      # (N, ng)
    coefs: np.ndarray     # (N, ng)


def draw_gaussians(rng, N, ng, exp_range, atoms=None, box=None):
    """Per orbital, per Gaussian, in this order: centre, exponent, coefficient.
    Centres are a uniformly drawn atom (when `atoms` is given) or uniform in
    the cube [-box, box]^3."""
    C = np.zeros((N, ng, 3))
    E = np.zeros((N, ng))
    A = np.zeros((N, ng))
    for i in range(N):
        for g in range(ng):
            if atoms is not None:
                C[i, g] = atoms[int(rng.integers(len(atoms)))]
            else:
                C[i, g] = rng.uniform(-box, box, size=3)
            E[i, g] = rng.uniform(exp_range[0], exp_range[1])
            A[i, g] = rng.normal()
    return GaussSpec(C, E, A)


def eval_gaussians(spec: GaussSpec, grid: Grid, device="cpu", chunk=64):
    """chi_i(r) = sum_g c_ig exp(-a_ig |r - R_ig|^2) on the grid, (N, n0, n1, n2)."""
    N = spec.exps.shape[0]
    out = torch.empty((N,) + grid.shape, dtype=DT, device=device)
    xs = [torch.as_tensor(x, dtype=DT, device=device) for x in grid.x]
    Cc = torch.as_tensor(spec.centres, dtype=DT, device=device)
    Ee = torch.as_tensor(spec.exps, dtype=DT, device=device)
    Aa = torch.as_tensor(spec.coefs, dtype=DT, device=device)
    for s in range(0, N, chunk):
        e = slice(s, min(N, s + chunk))
        f = [torch.exp(-Ee[e, :, None] * (xs[d][None, None, :] - Cc[e, :, d, None]) ** 2) for d in range(3)]
        f0 = f[0] * Aa[e, :, None]
        out[e] = torch.einsum("iga,igb,igc->iabc", f0, f[1], f[2])
    return out


def loewdin(chi, grid: Grid, cond_max=1e8):
    """psi = S^{-1/2} chi with S_ij = <chi_i, chi_j>_W, W = q0 (x) q1 (x) q2."""
    N = chi.shape[0]
    w = grid.weights3d(chi.device).reshape(-1)
    X = chi.reshape(N, -1)
    S = (X * w) @ X.T
    S = 0.5 * (S + S.T)
    lam, V = torch.linalg.eigh(S)
    cond = float(lam.max() / lam.min()) if float(lam.min()) > 0 else float("inf")
    if not (cond < cond_max):
        return None, cond
    Sm = (V * lam.rsqrt()) @ V.T
    psi = (Sm @ X).reshape(chi.shape)
    return psi, cond


# --------------------------------------------------------------------------------------
# shared Tucker bases (HOSVD of the stacked pair densities)
# --------------------------------------------------------------------------------------
def _mode_gram(psi, grid: Grid, d, targets=None, chunk_rest=4096):
    """Gram matrix of the mode-d unfolding of all sqrt(w)-scaled pair densities
    rho_ij = psi_i psi_j, i over `targets` (all when None), j over all.

    S[a,a'] = sum_rest sqrt(q(a) q(a')) q_rest D_T(a,a',rest) D(a,a',rest),
    D(a,a',rest) = sum_i psi_i(a,rest) psi_i(a',rest), which is the sum over
    pairs without forming any pair density."""
    N = psi.shape[0]
    dev = psi.device
    P = torch.movedim(psi, d + 1, 1).reshape(N, grid.n[d], -1)         # (N, n_d, R)
    qd = torch.as_tensor(grid.q[d], dtype=DT, device=dev)
    others = [torch.as_tensor(grid.q[e], dtype=DT, device=dev) for e in range(3) if e != d]
    qrest = (others[0][:, None] * others[1][None, :]).reshape(-1)
    R = P.shape[2]
    S = torch.zeros((grid.n[d], grid.n[d]), dtype=DT, device=dev)
    for s in range(0, R, chunk_rest):
        e = slice(s, min(R, s + chunk_rest))
        Pc = P[:, :, e].permute(2, 0, 1).contiguous()                   # (Rc, N, n_d)
        D = torch.bmm(Pc.transpose(1, 2).contiguous(), Pc)              # (Rc, n_d, n_d)
        if targets is None:
            DT_ = D
        else:
            Pt = Pc[:, targets, :]
            DT_ = torch.bmm(Pt.transpose(1, 2).contiguous(), Pt)
        S += torch.einsum("r,rab->ab", qrest[e], D * DT_)
    S = S * torch.sqrt(qd[:, None] * qd[None, :])
    return 0.5 * (S + S.T)


def hosvd_bases(psi, grid: Grid, r, targets=None):
    """Leading-r q-orthonormal bases U_d (n_d x r) of the stacked pair densities:
    U_d^T diag(q_d) U_d = I.  Columns are ordered by decreasing singular value
    and signed so that their largest-magnitude entry is positive."""
    rr = r if isinstance(r, (tuple, list)) else (r, r, r)
    Us = []
    for d in range(3):
        S = _mode_gram(psi, grid, d, targets)
        lam, V = torch.linalg.eigh(S)
        V = V[:, torch.argsort(lam, descending=True)][:, : rr[d]]
        idx = torch.argmax(V.abs(), dim=0)
        sgn = torch.sign(V[idx, torch.arange(V.shape[1], device=V.device)])
        sgn[sgn == 0] = 1
        V = V * sgn
        qd = torch.as_tensor(grid.q[d], dtype=DT, device=V.device)
        Us.append((V / torch.sqrt(qd)[:, None]).cpu().numpy())
    return Us


def full_rank_bases(grid: Grid, seed=0):
    """Square q-orthonormal bases (r = n): a seeded random orthogonal matrix
    scaled by diag(q)^{-1/2}.  With them the projector onto the Tucker space is
    the identity."""
    rng = np.random.default_rng(seed)
    Us = []
    for d in range(3):
        n = grid.n[d]
        Qm, _ = np.linalg.qr(rng.normal(size=(n, n)))
        Us.append(Qm / np.sqrt(grid.q[d])[:, None])
    return Us


# --------------------------------------------------------------------------------------
# systems
# --------------------------------------------------------------------------------------
@dataclass
class System:
    """One exchange problem: grid, orbitals, bases, exponential sum, pair set."""

    name: str
    grid: Grid
    psi: torch.Tensor                 # (N, n0, n1, n2) float64
    U: list                           # 3 x (n_d, r_d) float64 numpy, q-orthonormal
    w: np.ndarray                     # (K,)
    alpha: np.ndarray                 # (K,)
    mode: str = "symmetric"           # "symmetric": all unique pairs; "block": targets x all
    i0: int = 0
    Ni: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return int(self.psi.shape[0])

    @property
    def r(self):
        return tuple(int(u.shape[1]) for u in self.U)

    @property
    def K(self):
        return int(len(self.w))

    def n_pairs(self):
        if self.mode == "symmetric":
            return self.N * (self.N + 1) // 2
        return self.Ni * self.N


def make_orbitals(grid, N, ng, exp_range, seed, atoms=None, box=None, device="cpu", cond_max=1e8):
    """Draw, evaluate and Loewdin-orthonormalise N Gaussian orbitals; redraw
    with the next sub-seed when the overlap matrix has condition >= cond_max."""
    for attempt in range(20):
        rng = np.random.default_rng([seed, attempt])
        spec = draw_gaussians(rng, N, ng, exp_range, atoms=atoms, box=box)
        chi = eval_gaussians(spec, grid, device=device)
        psi, cond = loewdin(chi, grid, cond_max=cond_max)
        del chi
        if psi is not None:
            return psi, {"overlap_cond": cond, "draw_attempt": attempt}
    raise RuntimeError("could not draw a well-conditioned orbital set")


def make_system(name, n, L, N, ng, exp_range, r, K, seed, atoms=None, box=None,
                mode="symmetric", i0=0, Ni=0, device="cpu", bases="hosvd",
                s_range=(-8.0, 4.0), cond_max=1e8, grid=None):
    grid = uniform_grid(n, L) if grid is None else grid
    psi, meta = make_orbitals(grid, N, ng, exp_range, seed, atoms=atoms, box=box, device=device,
                              cond_max=cond_max)
    if bases == "full":
        U = full_rank_bases(grid, seed)
    else:
        targets = None if mode == "symmetric" else torch.arange(i0, i0 + Ni, device=psi.device)
        U = hosvd_bases(psi, grid, r, targets=targets)
    w, alpha = exp_sum(K, *s_range)
    meta.update({"seed": seed, "exp_range": tuple(exp_range), "ng": ng, "s_range": s_range})
    return System(name=name, grid=grid, psi=psi, U=U, w=w, alpha=alpha, mode=mode,
                  i0=i0, Ni=(Ni if mode == "block" else N), meta=meta)


# The five workloads.  Sizes follow the hot-path scope of the method: grid,
# orbital count, Tucker rank r, Gaussian-term count K and pair set.
CONFIGS = {
    "cfg1": dict(n=24, L=6.0, N=4, ng=3, exp_range=(0.5, 2.0), r=16, K=30, seed=1, box=2.0),
    "cfg2": dict(n=64, L=10.0, N=64, ng=6, exp_range=(0.3, 3.0), r=40, K=40, seed=2, atoms=("fcc", 13)),
    "cfg3": dict(n=80, L=12.0, N=128, ng=6, exp_range=(0.3, 3.0), r=48, K=40, seed=3, atoms=("fcc", 40)),
    # 1842 orbitals from Gaussians on 310 sites are nearly dependent (the
    # overlap matrix has condition ~1e9); FP64 Loewdin still orthonormalises
    # them to ~1e-7
    "cfg4": dict(n=128, L=16.0, N=1842, ng=6, exp_range=(0.3, 3.0), r=80, K=50, seed=4,
                 atoms=("rutile", 310), mode="block", i0=0, Ni=128, cond_max=1e11),
}

WORKLOAD_NAMES = {
    "cfg1": "fp64 exchange apply, 24^3 grid on [-6,6]^3, 4 orbitals, r=16, K=30, 10 unique pairs",
    "cfg2": "exchange apply, 64^3 grid on [-10,10]^3, 64 orbitals on a 13-atom fcc cluster, r=40, K=40, 2080 unique pairs",
    "cfg3": "differentiable E_x, 80^3 grid on [-12,12]^3, 128 orbitals on a 40-atom fcc cluster, r=48, K=40, 8256 unique pairs",
    "cfg4": "block exchange, 128^3 grid on [-16,16]^3, 1842 orbitals on 310 rutile sites, 128 targets x 1842 sources, r=80, K=50",
    "cfg5": "24 uneven systems, grids 48^3..96^3, 10..120 orbitals, r=24..64, K=40",
}


def _atoms(spec):
    if spec is None:
        return None
    kind, count = spec
    if kind == "fcc":
        return fcc_sites(count)
    if kind == "rutile":
        return rutile_sites(count)
    raise ValueError(kind)


def build_config(name, device="cpu", **overrides):
    """Generate one of the named workloads (optionally with overrides, e.g. a
    smaller N or r for a quick test)."""
    c = dict(CONFIGS[name])
    c.update(overrides)
    atoms = _atoms(c.pop("atoms", None))
    return make_system(name, c.pop("n"), c.pop("L"), c.pop("N"), c.pop("ng"), c.pop("exp_range"),
                       c.pop("r"), c.pop("K"), c.pop("seed"), atoms=atoms, box=c.pop("box", None),
                       device=device, **c)


def cfg5_specs(seed=5, count=24):
    """Per-system parameters of the batched workload: n in {48,56,...,96},
    L = 10 (n-1)/63 (spacing of the 64^3 case), N in {10..120}, an fcc cluster
    of max(1, round(N/5)) atoms, r in {24..64} capped at n, K = 40."""
    rng = np.random.default_rng(seed)
    specs = []
    for s in range(count):
        n = int(rng.choice(np.arange(48, 97, 8)))
        N = int(rng.integers(10, 121))
        r = int(min(n, rng.integers(24, 65)))
        specs.append(dict(n=n, L=10.0 * (n - 1) / 63.0, N=N, r=r, K=40, seed=1000 * seed + s,
                          atoms=max(1, int(round(N / 5)))))
    return specs


def build_cfg5(device="cpu", count=24, **overrides):
    out = []
    for sp in cfg5_specs(count=count):
        sp.update(overrides)
        out.append(make_system(f"cfg5_{len(out)}", sp["n"], sp["L"], sp["N"], 6, (0.3, 3.0), sp["r"],
                               sp["K"], sp["seed"], atoms=fcc_sites(sp["atoms"]), device=device))
    return out


def small_system(n=12, L=5.0, N=3, ng=3, r=6, K=8, seed=11, bases="hosvd", exp_range=(0.5, 2.0),
                 box=1.5, mode="symmetric", i0=0, Ni=0, s_range=(-8.0, 4.0)):
    """A tiny system for pins and parity at sizes the oracle finishes at once."""
    return make_system(f"small_n{n}_N{N}_r{r}", n, L, N, ng, exp_range, r, K, seed, box=box,
                       mode=mode, i0=i0, Ni=Ni, bases=bases, s_range=s_range)
