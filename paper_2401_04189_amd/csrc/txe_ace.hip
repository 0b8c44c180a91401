// Adaptively compressed exchange (section "ACE implementation"): from the
// orbitals psi_i and their exchange actions W_i = Vx psi_i,
//   M_ij = <psi_i, W_j>_W,   M = -L L^T,   xi_k = sum_i W_i (L^-1)_ki   (eq. `eta`)
// and the operator V_ACE phi = -sum_k xi_k <xi_k, phi>_W.
//
// Three kernels, all FP64 arithmetic (inputs may be FP32):
//   k_gram     G[i][j] = sum_g w(g) X_i(g) Y_j(g): FP64 MFMA 16x16x4 per
//              (i tile, j tile, grid chunk), chunk partials summed in order
//              by k_gram_reduce (no atomics, bitwise repeatable)
//   k_chol_inv one workgroup: Cholesky of -M (left-looking, a column at a
//              time) and the inverse of the triangular factor, column per
//              thread
//   k_comb     out[m][g] = s * sum_i A[m][i] X_i(g): FP64 MFMA with the
//              grid point as the output column
#include <hip/hip_runtime.h>

#include <cmath>

#include "txe_internal.h"

namespace txe {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// One wavefront per (chunk, i tile, j tile).  Lane (lr, lg) reads four
// consecutive grid points base + 4 lg + q (q = 0..3) of row 16 ti + lr of X
// and of row 16 tj + lr of Y; step q is one MFMA whose K index is lg.  The
// four points share (a, b) because n2 is a multiple of 4.
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_gram(const TX *__restrict__ X, int NX, const TY *__restrict__ Y, int NY,
                                              int n0, int n1, int n2, const double *__restrict__ q0,
                                              const double *__restrict__ q1, const double *__restrict__ q2,
                                              long long chunk, int nchunks, double *__restrict__ part) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nti = (NX + 15) >> 4, ntj = (NY + 15) >> 4;
  const long long item = (long long)blockIdx.x * 4 + wave;
  const long long total = (long long)nchunks * nti * ntj;
  if (item >= total) return;  // whole wavefront (item is uniform)
  const int tj = (int)(item % ntj);
  const int ti = (int)((item / ntj) % nti);
  const int ch = (int)(item / ((long long)ntj * nti));
  const long long ng = (long long)n0 * n1 * n2;
  const long long g_begin = ch * chunk;
  const long long g_end = g_begin + chunk < ng ? g_begin + chunk : ng;
  const int ix = min(16 * ti + lr, NX - 1), iy = min(16 * tj + lr, NY - 1);
  const bool vx = 16 * ti + lr < NX, vy = 16 * tj + lr < NY;
  const TX *xr = X + (size_t)ix * ng;
  const TY *yr = Y + (size_t)iy * ng;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (long long base = g_begin; base < g_end; base += 16) {
    const long long p = base + 4 * lg;  // multiple of 4: same (a, b) for the four points
    const int c = (int)(p % n2);
    const long long ab = p / n2;
    const int b = (int)(ab % n1), a = (int)(ab / n1);
    const double wab = q0[a] * q1[b];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const double xv = vx ? (double)xr[p + q] : 0.0;
      const double yv = vy ? (double)yr[p + q] * (wab * q2[c + q]) : 0.0;
      acc = mfma64(xv, yv, acc);
    }
  }
  // f64 MFMA result: row 4 v + lg, column lr
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int i = 16 * ti + 4 * v + lg, j = 16 * tj + lr;
    if (i < NX && j < NY) part[((size_t)ch * NX + i) * NY + j] = acc[v];
  }
}

__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ part, int nchunks, long long nxy,
                                                     double *__restrict__ G) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nxy) return;
  double s = 0.0;
  for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * nxy + e];
  G[e] = s;
}

// Cholesky of -M and the inverse of its factor, in one workgroup of 256.
// info: 0 on success, j + 1 when the pivot of column j is not positive
// (M not negative definite); L and T are then undefined.
__global__ __launch_bounds__(256) void k_chol_inv(const double *__restrict__ M, int N, double *__restrict__ L,
                                                  double *__restrict__ T, int *__restrict__ info) {
  __shared__ double red[256];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (long long e = tid; e < (long long)N * N; e += 256) {
    const int i = (int)(e / N), j = (int)(e % N);
    if (j > i) {
      L[e] = 0.0;
      T[e] = 0.0;
    }
  }
  __syncthreads();
  for (int j = 0; j < N; ++j) {
    // pivot: -M[j][j] - sum_{k<j} L[j][k]^2, each thread a strided part in
    // order, then a fixed-shape tree
    double s = 0.0;
    for (int k = tid; k < j; k += 256) s += L[(size_t)j * N + k] * L[(size_t)j * N + k];
    red[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    const double d = -M[(size_t)j * N + j] - red[0];
    __syncthreads();  // red[0] read by everyone before it is overwritten
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) {
        bad = j + 1;
        *info = j + 1;
      }
      break;  // uniform: every thread computed the same d
    }
    const double ljj = sqrt(d);
    if (tid == 0) L[(size_t)j * N + j] = ljj;
    for (int i = j + 1 + tid; i < N; i += 256) {
      double t = -M[(size_t)i * N + j];
      for (int k = 0; k < j; ++k) t -= L[(size_t)i * N + k] * L[(size_t)j * N + k];
      L[(size_t)i * N + j] = t / ljj;
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) return;
  if (tid == 0) *info = 0;
  // T = L^-1 (lower): column c by one thread, rows in order
  for (int c = tid; c < N; c += 256) {
    T[(size_t)c * N + c] = 1.0 / L[(size_t)c * N + c];
    for (int i = c + 1; i < N; ++i) {
      double t = 0.0;
      for (int k = c; k < i; ++k) t += L[(size_t)i * N + k] * T[(size_t)k * N + c];
      T[(size_t)i * N + c] = -t / L[(size_t)i * N + i];
    }
  }
}

// out[m][g] = scale * sum_i A[m][i] X_i(g); A is MR x K row-major (FP64).
// One wavefront per (16-point grid tile, group of MG m tiles); lane (lr, lg)
// reads X_{i0 + lg}(g0 + lr) (B operand) and A[16 mt + lr][i0 + lg] (A
// operand).  With lower = 1, A[m][i] = 0 for i > m and those chunks are
// skipped.
template <typename TX, typename TO, int MG>
__global__ __launch_bounds__(256) void k_comb(const double *__restrict__ A, int MR, int K,
                                              const TX *__restrict__ X, long long ng, double scale, int lower,
                                              TO *__restrict__ out) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nmt = (MR + 15) >> 4, nmg = (nmt + MG - 1) / MG;
  const long long item = (long long)blockIdx.x * 4 + wave;
  const long long ngt = ng >> 4;
  if (item >= ngt * nmg) return;
  const int mgi = (int)(item % nmg);
  const long long gt = item / nmg;
  const long long g = 16 * gt + lr;
  const int mt0 = mgi * MG;
  d4 acc[MG];
#pragma unroll
  for (int u = 0; u < MG; ++u) acc[u] = d4{0.0, 0.0, 0.0, 0.0};
  // last column that can be nonzero for this group's rows
  const int mlast = min(MR, 16 * (mt0 + MG)) - 1;
  const int kend = lower ? min(K, mlast + 1) : K;
  for (int i0 = 0; i0 < kend; i0 += 4) {
    const int i = i0 + lg;
    const double b = i < K ? (double)X[(size_t)i * ng + g] : 0.0;
#pragma unroll
    for (int u = 0; u < MG; ++u) {
      const int m = 16 * (mt0 + u) + lr;
      const double a = (m < MR && i < K) ? A[(size_t)m * K + i] : 0.0;
      acc[u] = mfma64(a, b, acc[u]);
    }
  }
#pragma unroll
  for (int u = 0; u < MG; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = 16 * (mt0 + u) + 4 * v + lg;
      if (m < MR) out[(size_t)m * ng + g] = (TO)(scale * acc[u][v]);
    }
}

constexpr int COMB_MG = 4;

}  // namespace

// ------------------------------------------------------------------------------------
// host-side launchers (argument checks are done by the caller)
// ------------------------------------------------------------------------------------
// Grid points per chunk of the Gram kernel: about 8192 wavefronts in all,
// chunks of at least 64 points, a multiple of 16.
static long long gram_chunk_len(int NX, int NY, long long ng) {
  const long long tiles = (long long)((NX + 15) / 16) * ((NY + 15) / 16);
  long long nch = (8192 + tiles - 1) / tiles;
  const long long maxch = ng / 64;
  if (nch > maxch) nch = maxch;
  if (nch < 1) nch = 1;
  const long long chunk = (ng + nch - 1) / nch;
  return (chunk + 15) / 16 * 16;
}

int gram_nchunks(int NX, int NY, long long ng) {
  const long long chunk = gram_chunk_len(NX, NY, ng);
  return (int)((ng + chunk - 1) / chunk);
}

template <typename TX, typename TY>
static hipError_t gram_t(const TX *X, int NX, const TY *Y, int NY, const Dims &D, const double *const qdev[3],
                         double *part, double *G, hipStream_t s) {
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  const long long chunk = gram_chunk_len(NX, NY, ng);
  const int nchunks = gram_nchunks(NX, NY, ng);
  const long long waves = (long long)nchunks * ((NX + 15) / 16) * ((NY + 15) / 16);
  hipLaunchKernelGGL((k_gram<TX, TY>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, X, NX, Y, NY, D.n0, D.n1,
                     D.n2, qdev[0], qdev[1], qdev[2], chunk, nchunks, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long nxy = (long long)NX * NY;
  hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)((nxy + 255) / 256)), dim3(256), 0, s, part, nchunks, nxy, G);
  return hipGetLastError();
}

hipError_t ace_gram(bool x64, bool y64, const void *X, int NX, const void *Y, int NY, const Dims &D,
                    const double *const qdev[3], double *part, double *G, hipStream_t s) {
  if (x64 && y64) return gram_t((const double *)X, NX, (const double *)Y, NY, D, qdev, part, G, s);
  if (!x64 && !y64) return gram_t((const float *)X, NX, (const float *)Y, NY, D, qdev, part, G, s);
  if (!x64 && y64) return gram_t((const float *)X, NX, (const double *)Y, NY, D, qdev, part, G, s);
  return gram_t((const double *)X, NX, (const float *)Y, NY, D, qdev, part, G, s);
}

hipError_t ace_chol_inv(const double *M, int N, double *L, double *T, int *info, hipStream_t s) {
  hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(256), 0, s, M, N, L, T, info);
  return hipGetLastError();
}

template <typename TX, typename TO>
static hipError_t comb_t(const double *A, int MR, int K, const TX *X, long long ng, double scale, int lower, TO *out,
                         hipStream_t s) {
  const int nmg = ((MR + 15) / 16 + COMB_MG - 1) / COMB_MG;
  const long long waves = (ng / 16) * nmg;
  hipLaunchKernelGGL((k_comb<TX, TO, COMB_MG>), dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, A, MR, K, X, ng,
                     scale, lower, out);
  return hipGetLastError();
}

hipError_t ace_comb(bool x64, bool o64, const double *A, int MR, int K, const void *X, long long ng, double scale,
                    int lower, void *out, hipStream_t s) {
  if (x64 && o64) return comb_t(A, MR, K, (const double *)X, ng, scale, lower, (double *)out, s);
  if (!x64 && o64) return comb_t(A, MR, K, (const float *)X, ng, scale, lower, (double *)out, s);
  if (x64 && !o64) return comb_t(A, MR, K, (const double *)X, ng, scale, lower, (float *)out, s);
  return comb_t(A, MR, K, (const float *)X, ng, scale, lower, (float *)out, s);
}

}  // namespace txe
