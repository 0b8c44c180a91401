// Generic FP64 tensor-mode products and the Hadamard accumulation of Vx psi
// over sources, shared by the per-pair-bases path and the collocation path
// (host launchers; the kernels live in txe_modes.hip).
#pragma once

#include "txe_internal.h"

namespace txe {

// element of the mode-d unfolding of a tensor with extents (A, B, C): row
// `row` (index along mode d), column m (the other two indices, C order)
__device__ __forceinline__ long long unfold_at(int d, int B, int C, int row, long long m) {
  if (d == 0) return (long long)row * B * C + m;
  if (d == 1) return ((m / C) * B + row) * (long long)C + (m % C);
  return m * C + row;
}

// Y[p] (=|+=) yscale * (X[p] x_d M_p) for the P tensors of a chunk:
//   Y(.., o, ..) = f_o sum_{i < nin} M_p(i, o) X(.., i, ..),
// M_p(i, o) = Mt ? M[p][o][i] : M[p][i][o] (row-major, leading dimension ldm,
// pair stride ms, 0 = one matrix for all), f_o = 1 / sqrt(qout[o]) (1 when
// qout is null).  X has extents (A, B, C) (pair stride xs); Y the same with
// the mode-d extent replaced by nout (pair stride ys).  accum: add to Y
// instead of overwriting it.
hipError_t launch_mode_f64(const double *X, long long xs, int A, int B, int C, int d, int nin, const double *M,
                           long long ms, int ldm, int Mt, int nout, const double *qout, double yscale, int accum,
                           double *Y, long long ys, int P, hipStream_t s);

// Vx psi_t (+)= -sum_s psi_s phi_ts over the sources of a back-projection
// range, ascending, phi stored per local pair in [a][c][b] (phi_acb = 1) or
// [a][b][c] order; acc_in / finish as in the shared-basis back-projection
// (raw sums in vx between chunks; the last one writes -scale * sum, times the
// quadrature weight when weighted).
hipError_t launch_accum_f64(const double *phi, int phi_acb, const double *psi, const Dims &D, const PairMap &pm,
                            const BackRange &br, double *vx, const double *out_scale, int weighted,
                            const double *const q[3], hipStream_t s);

}  // namespace txe
