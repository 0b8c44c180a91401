// Host-side FP64 setup for order-p Lagrange finite elements (paper section
// "Creation of Structured FE basis": 1-D meshes of cells whose nodes are the
// Gauss-Lobatto-Legendre points of each cell, the 3-D basis the tensor product
// of the 1-D Lagrange polynomials; section "Convolution operation", eqs.
// `quadVal` and `discInteg`: the 1-D convolution of every Gaussian term with
// every basis function, precomputed once per mesh and term).
//
// Unknowns are the mesh nodes without the two ends of the domain, which are
// held at zero.  A node's quadrature weight is the sum of the GLL weights of
// the cells it belongs to (scaled by half the cell length), so that nodal sums
// are the GLL quadrature of the mesh.
//
// The convolution integral C[a][b] = int exp(-alpha (x_a - t)^2) N_b(t) dt is
// taken cell by cell with Gauss-Legendre quadrature on pieces no wider than
// 1 / (2 sqrt(alpha)), over the part of the cell where the Gaussian around
// x_a is above exp(-800) (the rest is below the double range).
#include <algorithm>
#include <cmath>
#include <vector>

#include "txe_internal.h"

namespace txe {

namespace {

typedef long double ld;
constexpr ld PI_L = 3.141592653589793238462643383279502884L;
constexpr int GL_POINTS = 20;

// P_m(x) and, for |x| < 1, P_m'(x), from the three-term recurrence
void legendre(int m, ld x, ld &P, ld &dP) {
  ld pm1 = 1.0L, p = x;
  if (m == 0) {
    P = 1.0L;
    dP = 0.0L;
    return;
  }
  for (int k = 2; k <= m; ++k) {
    const ld pn = ((2 * k - 1) * x * p - (k - 1) * pm1) / k;
    pm1 = p;
    p = pn;
  }
  P = p;
  dP = m * (x * p - pm1) / (x * x - 1.0L);
}

// m-point Gauss-Legendre rule on [-1, 1]: Newton on P_m from the Chebyshev-
// like first guesses cos(pi (i + 3/4) / (m + 1/2))
void gauss_legendre(int m, ld *t, ld *w) {
  for (int i = 0; i < m; ++i) {
    ld x = cosl(PI_L * (i + 0.75L) / (m + 0.5L)), P, dP;
    for (int it = 0; it < 100; ++it) {
      legendre(m, x, P, dP);
      const ld dx = P / dP;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    legendre(m, x, P, dP);
    t[i] = x;
    w[i] = 2.0L / ((1.0L - x * x) * dP * dP);
  }
}

}  // namespace

void gll_points(int p, double *s_out, double *w_out) {
  std::vector<ld> s(p + 1);
  s[0] = -1.0L;
  s[p] = 1.0L;
  // interior points: roots of P_p', by Newton with P_p'' from Legendre's
  // equation (1 - x^2) P'' = 2x P' - p(p+1) P
  for (int i = 1; i < p; ++i) {
    ld x = -cosl(PI_L * i / p), P, dP;
    for (int it = 0; it < 100; ++it) {
      legendre(p, x, P, dP);
      const ld d2P = (2.0L * x * dP - (ld)p * (p + 1) * P) / (1.0L - x * x);
      const ld dx = dP / d2P;
      x -= dx;
      if (fabsl(dx) < 1e-19L) break;
    }
    s[i] = x;
  }
  for (int i = 0; i <= p; ++i) {
    ld P, dP;
    legendre(p, s[i], P, dP);
    if (s_out) s_out[i] = (double)s[i];
    if (w_out) w_out[i] = (double)(2.0L / ((ld)p * (p + 1) * P * P));
  }
}

void fe_mesh_1d(const double *edges, int ncells, int p, double *x, double *q) {
  std::vector<double> s(p + 1), w(p + 1);
  gll_points(p, s.data(), w.data());
  const int nall = ncells * p + 1;
  std::vector<ld> xs(nall, 0.0L), qs(nall, 0.0L);
  for (int e = 0; e < ncells; ++e) {
    const ld lo = edges[e], hi = edges[e + 1];
    for (int m = 0; m <= p; ++m) {
      const int g = e * p + m;
      // the shared end node of two cells takes its position from the cell edge
      xs[g] = m == 0 ? lo : m == p ? hi : lo + 0.5L * ((ld)s[m] + 1.0L) * (hi - lo);
      qs[g] += (ld)w[m] * 0.5L * (hi - lo);
    }
  }
  for (int g = 1; g < nall - 1; ++g) {
    if (x) x[g - 1] = (double)xs[g];
    if (q) q[g - 1] = (double)qs[g];
  }
}

void fe_conv_matrix(const double *edges, int ncells, int p, double alpha, double *C) {
  const int n = ncells * p - 1;
  std::vector<double> sd(p + 1);
  gll_points(p, sd.data(), nullptr);
  std::vector<double> xn(n);
  fe_mesh_1d(edges, ncells, p, xn.data(), nullptr);
  ld gt[GL_POINTS], gw[GL_POINTS];
  gauss_legendre(GL_POINTS, gt, gw);
  const ld a = alpha;
  const ld reach = a > 0 ? sqrtl(800.0L / a) : INFINITY;  // exp(-a u^2) < exp(-800) beyond
  const ld piece = a > 0 ? 0.5L / sqrtl(a) : INFINITY;
  std::vector<ld> row(n), nodes(p + 1), L(p + 1);
  for (int ia = 0; ia < n; ++ia) {
    const ld xa = xn[ia];
    for (int b = 0; b < n; ++b) row[b] = 0.0L;
    for (int e = 0; e < ncells; ++e) {
      const ld lo = edges[e], hi = edges[e + 1];
      const ld u0 = std::max(lo, xa - reach), u1 = std::min(hi, xa + reach);
      if (!(u1 > u0)) continue;
      for (int m = 0; m <= p; ++m) nodes[m] = lo + 0.5L * ((ld)sd[m] + 1.0L) * (hi - lo);
      const int npc = std::isfinite((double)piece) ? std::max(1, (int)ceill((u1 - u0) / piece)) : 1;
      const ld pw = (u1 - u0) / npc;
      for (int c = 0; c < npc; ++c) {
        const ld c0 = u0 + c * pw, half = 0.5L * pw, mid = c0 + half;
        for (int g = 0; g < GL_POINTS; ++g) {
          const ld t = mid + half * gt[g];
          const ld d = xa - t;
          const ld f = half * gw[g] * expl(-a * d * d);
          for (int m = 0; m <= p; ++m) {
            ld v = 1.0L;
            for (int j = 0; j <= p; ++j)
              if (j != m) v *= (t - nodes[j]) / (nodes[m] - nodes[j]);
            L[m] = v;
          }
          for (int m = 0; m <= p; ++m) {
            const int b = e * p + m - 1;  // unknown index (the domain ends are held)
            if (b >= 0 && b < n) row[b] += f * L[m];
          }
        }
      }
    }
    for (int b = 0; b < n; ++b) C[(size_t)ia * n + b] = (double)row[b];
  }
}

}  // namespace txe
