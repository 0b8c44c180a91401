// The collocation form of the pair convolution (paper section "Convolution
// operation", eq. `final` with the 1-D convolutions of eqs. `quadVal` /
// `discInteg` evaluated at every 1-D node, then the 3-D field reconstructed):
//
//   phi_ij = sum_k w_k G_ij x0 (C_k^0 U0) x1 (C_k^1 U1) x2 (C_k^2 U2),
//   e_ij   = <rho_ij, phi_ij>_W (grid sum),
//
// with G_ij the projection of rho_ij onto the shared bases (the same
// projection kernels as the core-space form).  FP64 throughout.  Per chunk:
//   projection       G (k_proj12m / k_proj3)
//   per group of COLLOC_GROUP terms:
//     for each term  Y0 = G x2 A2_k, Ys[t] = Y0 x1 A1_k   (A_k^d = C_k^d U_d,
//                    n_d x r_d, built on the host in FP64)
//     phi (+)= Ys x0 A0s   one contraction over (t, alpha), the weights w_k
//                    folded into the stacked A0s, so that phi is read and
//                    written once per group rather than once per term
//   (G is zero past the ranks, so the stack's padding rows are zero)
//   k_col_epair      e_ij, one workgroup per pair, fixed order
//   accumulation     Vx psi_t -= sum_s psi_s phi_ts, sources ascending
#include <algorithm>

#include "txe_dev.h"
#include "txe_modes.h"

namespace txe {

namespace {

// e_ij = sum_g q0[a] q1[b] q2[c] psi_i(g) psi_j(g) phi_ij(g): one workgroup per
// pair, each thread a strided partial sum, then a fixed tree in LDS
__global__ __launch_bounds__(256) void k_col_epair(const double *__restrict__ phi, const double *__restrict__ psi,
                                                   Dims D, PairMap pm, const double *__restrict__ q0,
                                                   const double *__restrict__ q1, const double *__restrict__ q2,
                                                   double *__restrict__ epair) {
  __shared__ double part[256];
  const int p = blockIdx.x;
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  int i, j;
  pair_ij(pm, p, i, j);
  const double *pi = psi + (size_t)i * ng, *pj = psi + (size_t)j * ng, *ph = phi + (size_t)p * ng;
  double s = 0.0;
  for (long long g = threadIdx.x; g < ng; g += 256) {
    const int c = (int)(g % D.n2), b = (int)((g / D.n2) % D.n1), a = (int)(g / ((long long)D.n1 * D.n2));
    s += q0[a] * q1[b] * q2[c] * pi[g] * pj[g] * ph[g];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) epair[apply_pair(pm, i, j)] = part[0];
}

}  // namespace

hipError_t run_chunk_colloc(const Tables<double> &tb, const CollocArgs &cl, const ChunkArgs<double> &a, bool want_vx,
                            hipStream_t s, Prof *prof) {
  const Dims &D = a.D;
  const int P = a.P, RP = D.rp0;
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  hipError_t e = launch_projection<double, double>(tb, a, s, prof);
  if (e != hipSuccess) return e;
  // G: (RP, RP, RP) per pair, zero past the ranks
  prof->begin(K_CORE, s);
  const int GR = COLLOC_GROUP;
  const long long s0 = (long long)RP * RP * RP, s1 = (long long)RP * RP * D.n2;
  const long long st = (long long)RP * D.n1 * D.n2, ss = (long long)GR * st;  // one term's block of the stack
  for (int g = 0; g * GR < D.K && e == hipSuccess; ++g) {
    const int nt = std::min(GR, D.K - g * GR);
    for (int t = 0; t < nt && e == hipSuccess; ++t) {
      const int k = g * GR + t;
      e = launch_mode_f64(a.G, s0, RP, RP, RP, 2, D.r2, cl.A[2] + (size_t)k * D.n2 * D.r2, 0, D.r2, 1, D.n2, nullptr,
                          1.0, 0, cl.Y0, s1, P, s);
      if (e == hipSuccess)
        e = launch_mode_f64(cl.Y0, s1, RP, RP, D.n2, 1, D.r1, cl.A[1] + (size_t)k * D.n1 * D.r1, 0, D.r1, 1, D.n1,
                            nullptr, 1.0, 0, cl.Ys + (size_t)t * st, ss, P, s);
    }
    if (e == hipSuccess)
      e = launch_mode_f64(cl.Ys, ss, nt * RP, D.n1, D.n2, 0, nt * RP, cl.A0s + (size_t)g * D.n0 * GR * RP, 0, GR * RP,
                          1, D.n0, nullptr, 1.0, g > 0 ? 1 : 0, cl.phi, ng, P, s);
  }
  prof->end(s);
  if (e != hipSuccess) return e;
  prof->begin(K_EPAIR, s);
  hipLaunchKernelGGL(k_col_epair, dim3(P), dim3(256), 0, s, (const double *)cl.phi, (const double *)a.psi, D, a.pm,
                     a.qdev[0], a.qdev[1], a.qdev[2], a.epair);
  prof->end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!want_vx) return hipSuccess;
  prof->begin(K_BACK, s);
  for (int b = 0; b < a.nbr && e == hipSuccess; ++b)
    e = launch_accum_f64(cl.phi, 0, (const double *)a.psi, D, a.pm, a.br[b], (double *)a.vx, a.out_scale, a.weighted,
                         a.qdev, s);
  prof->end(s);
  return e;
}

}  // namespace txe
