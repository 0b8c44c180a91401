// Host-side FP64 setup of one exchange system: the 1-D Gaussian convolution
// matrices C_k^d on a linear finite-element mesh, the projection bases
// V_d = diag(q_d) U_d and the core-space matrices Chat_k^d = V_d^T C_k^d U_d
// (paper section "Convolution operation", eqs. `quadVal` and `discInteg`:
// the node sums are precomputed once per mesh and Gaussian term).
//
// The paper integrates the Gaussian against the interpolated field with many
// quadrature points; with linear shape functions the integral of a Gaussian
// against one hat has a closed form in erf / exp, evaluated here in extended
// precision.
#include <cmath>
#include <cstring>
#include <vector>

#include "txe_internal.h"

namespace txe {

namespace {

typedef long double ld;

// int_{s1}^{s2} exp(-a s^2) ds  (a > 0), without cancellation when both ends
// lie on the same side of 0.
ld gauss_int0(ld a, ld s1, ld s2) {
  const ld ra = sqrtl(a);
  const ld z1 = ra * s1, z2 = ra * s2;
  const ld c = sqrtl((ld)M_PI) / (2.0L * ra);
  if (z1 >= 0) return c * (erfcl(z1) - erfcl(z2));
  if (z2 <= 0) return c * (erfcl(-z2) - erfcl(-z1));
  return c * (erfl(z2) - erfl(z1));
}

// int_{s1}^{s2} s exp(-a s^2) ds  (a > 0) = (e^{-a s1^2} - e^{-a s2^2}) / (2a),
// through expm1 so that small a s^2 keep their digits.
ld gauss_int1(ld a, ld s1, ld s2) {
  return (expm1l(-a * s1 * s1) - expm1l(-a * s2 * s2)) / (2.0L * a);
}

// int_{lo}^{hi} exp(-a (t - xa)^2) hat(t) dt with hat rising (t-lo)/W or
// falling (hi-t)/W on [lo, hi], W = hi - lo.
ld hat_piece(ld a, ld xa, ld lo, ld hi, bool rising) {
  const ld W = hi - lo;
  const ld s1 = lo - xa, s2 = hi - xa;
  ld J0, J1;
  if (a == 0) {
    J0 = s2 - s1;
    J1 = 0.5L * (s2 * s2 - s1 * s1);
  } else {
    J0 = gauss_int0(a, s1, s2);
    J1 = gauss_int1(a, s1, s2);
  }
  return rising ? (J1 - s1 * J0) / W : (s2 * J0 - J1) / W;
}

}  // namespace

void conv_matrix_1d(int n, const double *x, double alpha, double *C) {
  // ghost nodes extend the mesh by one element at each end so that every real
  // node carries a full hat (the ghost nodes themselves are held at zero)
  std::vector<ld> xg(n + 2);
  for (int i = 0; i < n; ++i) xg[i + 1] = x[i];
  xg[0] = 2.0L * x[0] - x[1];
  xg[n + 1] = 2.0L * x[n - 1] - x[n - 2];
  const ld a = alpha;
  for (int ia = 0; ia < n; ++ia) {
    const ld xa = x[ia];
    for (int b = 0; b < n; ++b) {
      const ld v = hat_piece(a, xa, xg[b], xg[b + 1], true) + hat_piece(a, xa, xg[b + 1], xg[b + 2], false);
      C[(size_t)ia * n + b] = (double)v;
    }
  }
}

// Chat = V^T C U  (r x r) with V = diag(q) U, all FP64 (long double sums).
void core_matrix(int n, int r, const double *q, const double *U, const double *C, double *Chat) {
  std::vector<ld> CU((size_t)n * r, 0.0L);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b) {
      const ld c = C[(size_t)a * n + b];
      if (c == 0) continue;
      for (int s = 0; s < r; ++s) CU[(size_t)a * r + s] += c * (ld)U[(size_t)b * r + s];
    }
  for (int p = 0; p < r; ++p)
    for (int s = 0; s < r; ++s) {
      ld acc = 0;
      for (int a = 0; a < n; ++a) acc += (ld)q[a] * (ld)U[(size_t)a * r + p] * CU[(size_t)a * r + s];
      Chat[(size_t)p * r + s] = (double)acc;
    }
}

}  // namespace txe
