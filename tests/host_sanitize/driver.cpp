// Host-only driver for an AddressSanitizer / UndefinedBehaviorSanitizer build
// of the library's host setup code (the linear-hat and order-p convolution
// matrices, the core matrices, the GLL rule): every routine on meshes of
// several sizes, orders 1-10, and Gaussian exponents from 0 to 1e6.  Prints
// a checksum line; any sanitizer report aborts the run.
#include <cmath>
#include <cstdio>
#include <vector>

#include "txe_internal.h"

int main() {
  double sum = 0.0;
  const double alphas[] = {0.0, 1e-7, 0.3, 30.0, 2981.0, 1e6};
  // order-p elements on a graded mesh, every order
  const std::vector<double> edges = {-4.0, -2.5, -1.4, -0.6, -0.1, 0.2, 0.9, 2.6, 4.0};
  for (int p = 1; p <= txe::FE_MAX_ORDER; ++p) {
    const int nc = (int)edges.size() - 1, n = nc * p - 1;
    std::vector<double> s(p + 1), w(p + 1), x(n), q(n), C((size_t)n * n);
    txe::gll_points(p, s.data(), w.data());
    txe::fe_mesh_1d(edges.data(), nc, p, x.data(), q.data());
    for (double a : alphas) {
      txe::fe_conv_matrix(edges.data(), nc, p, a, C.data());
      for (double v : C) sum += v;
    }
    for (int i = 0; i <= p; ++i) sum += s[i] + w[i];
  }
  // one cell, the smallest mesh with unknowns
  {
    const double e1[] = {0.0, 1.0};
    std::vector<double> x(1), q(1), C(1);
    txe::fe_mesh_1d(e1, 1, 2, x.data(), q.data());
    txe::fe_conv_matrix(e1, 1, 2, 5.0, C.data());
    sum += C[0];
  }
  // linear hats on uniform grids, and the core matrices of random q-orthonormal-ish bases
  for (int n : {4, 5, 16, 33}) {
    std::vector<double> x(n), q(n), C((size_t)n * n);
    for (int i = 0; i < n; ++i) {
      x[i] = -3.0 + 6.0 * i / (n - 1);
      q[i] = 6.0 / (n - 1);
    }
    for (double a : alphas) {
      txe::conv_matrix_1d(n, x.data(), a, C.data());
      for (double v : C) sum += v;
    }
    const int r = n / 2 > 0 ? n / 2 : 1;
    std::vector<double> U((size_t)n * r), Chat((size_t)r * r);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < r; ++k) U[(size_t)i * r + k] = std::cos(0.3 * (i + 1) * (k + 1)) / std::sqrt(q[i] * n);
    txe::core_matrix(n, r, q.data(), U.data(), C.data(), Chat.data());
    for (double v : Chat) sum += v;
  }
  std::printf("host setup checksum %.17g\n", sum);
  return std::isfinite(sum) ? 0 : 1;
}
