// Adaptively compressed exchange (section "ACE implementation"): from the
// orbitals psi_i and their exchange actions W_i = Vx psi_i,
//   M_ij = <psi_i, W_j>_W,   M = -L L^T,   xi_k = sum_i W_i (L^-1)_ki   (eq. `eta`)
// and the operator V_ACE phi = -sum_k xi_k <xi_k, phi>_W.
//
// Three kernels, all FP64 arithmetic (inputs may be FP32):
//   k_gram     G[i][j] = sum_g w(g) X_i(g) Y_j(g): FP64 MFMA 16x16x4 per
//              (64 x 64 output tile, grid chunk), operands staged in LDS,
//              chunk partials summed in order by k_gram_reduce (no atomics,
//              bitwise repeatable)
//   k_chol     one workgroup: Cholesky of -M (left-looking, a column at a
//              time, the pivot row's prefix in LDS)
//   k_tri_inv  the inverse of the triangular factor, a column per thread
//              over as many workgroups as it takes
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

// One workgroup per (grid chunk, 64-row i tile, 64-column j tile); each
// wavefront holds a 32 x 32 corner (2 x 2 MFMA tiles).  The chunk is walked
// in slices of GS grid points: rows of X and of w Y are staged in LDS (thread
// t takes point t mod GS of the slice and eight rows of each, so a point's
// weight is formed once per slice), then each wavefront runs GS / 4 MFMA K
// steps from LDS.  Every staged value serves four MFMA tiles.
constexpr int GT = 64;       // output tile edge
constexpr int GS = 32;       // grid points per slice
constexpr int GP = GS + 2;   // padded LDS row (doubles): a fragment read hits 64 distinct banks
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void k_gram(const TX *__restrict__ X, int NX, const TY *__restrict__ Y, int NY,
                                              int n0, int n1, int n2, const double *__restrict__ q0,
                                              const double *__restrict__ q1, const double *__restrict__ q2,
                                              long long chunk, int nchunks, double *__restrict__ part) {
  __shared__ double Xs[GT * GP], Ys[GT * GP];
  const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane((int)(tid >> 6));
  const int nti = (NX + GT - 1) / GT, ntj = (NY + GT - 1) / GT;
  const long long blk = blockIdx.x;
  const int tj = (int)(blk % ntj);
  const int ti = (int)((blk / ntj) % nti);
  const int ch = (int)(blk / ((long long)ntj * nti));
  const long long ng = (long long)n0 * n1 * n2;
  const long long g_begin = ch * chunk;
  const long long g_end = g_begin + chunk < ng ? g_begin + chunk : ng;
  const int ib = 32 * (wave >> 1), jb = 32 * (wave & 1);
  // staging: point sp = tid mod GS of the slice, rows r0 + 8 k (k < 8)
  const int sp = tid % GS, r0 = tid / GS;
  typedef double d4v __attribute__((ext_vector_type(4)));
  d4v acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
  for (long long base = g_begin; base < g_end; base += GS) {
    const long long g = base + sp;
    const bool live = g < g_end;
    double w = 0.0;
    if (live) {
      const int c = (int)(g % n2);
      const long long ab = g / n2;
      w = q0[ab / n1] * q1[ab % n1] * q2[c];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = r0 + 8 * k;
      const int ix = GT * ti + r, iy = GT * tj + r;
      Xs[r * GP + sp] = live && ix < NX ? (double)X[(size_t)ix * ng + g] : 0.0;
      Ys[r * GP + sp] = live && iy < NY ? w * (double)Y[(size_t)iy * ng + g] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < GS; k0 += 4) {
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = Xs[(ib + 16 * a + lr) * GP + k0 + lg];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = Ys[(jb + 16 * b + lr) * GP + k0 + lg];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma64(av[a], bv[b], acc[a][b]);
    }
    __syncthreads();  // the next slice overwrites the staged rows
  }
  // f64 MFMA result: row 4 v + lg, column lr of each tile
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = GT * ti + ib + 16 * a + 4 * v + lg, j = GT * tj + jb + 16 * b + lr;
        if (i < NX && j < NY) part[((size_t)ch * NX + i) * NY + j] = acc[a][b][v];
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

// Cholesky of -M in one workgroup of 256 (left-looking, a column at a time):
// the pivot row's finished prefix L[j][0..j) is staged in LDS, and each
// thread forms its rows' dot products with four partial sums (a fixed order
// per thread).  info: 0 on success, j + 1 when the pivot of column j is not
// positive (M not negative definite); L is then undefined.
constexpr int CHOL_MAX = 2048;
__global__ __launch_bounds__(256) void k_chol(const double *__restrict__ M, int N, double *__restrict__ L,
                                              int *__restrict__ info) {
  __shared__ double red[256];
  __shared__ double lj[CHOL_MAX];
  const int tid = threadIdx.x;
  for (long long e = tid; e < (long long)N * N; e += 256) {
    const int i = (int)(e / N), j = (int)(e % N);
    if (j > i) L[e] = 0.0;
  }
  for (int j = 0; j < N; ++j) {
    // the pivot row's prefix, and its squares summed: each thread a strided
    // part in order, then a fixed-shape tree
    double s = 0.0;
    for (int k = tid; k < j; k += 256) {
      const double v = L[(size_t)j * N + k];
      lj[k] = v;
      s += v * v;
    }
    red[tid] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if (tid < off) red[tid] += red[tid + off];
      __syncthreads();
    }
    const double d = -M[(size_t)j * N + j] - red[0];
    __syncthreads();  // red[0] read by everyone before it is overwritten
    if (!(d > 0.0) || !isfinite(d)) {
      if (tid == 0) *info = j + 1;
      return;  // uniform: every thread computed the same d
    }
    const double ljj = sqrt(d);
    if (tid == 0) L[(size_t)j * N + j] = ljj;
    for (int i = j + 1 + tid; i < N; i += 256) {
      const double *li = L + (size_t)i * N;
      double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
      int k = 0;
      for (; k + 3 < j; k += 4) {
        t0 += li[k] * lj[k];
        t1 += li[k + 1] * lj[k + 1];
        t2 += li[k + 2] * lj[k + 2];
        t3 += li[k + 3] * lj[k + 3];
      }
      for (; k < j; ++k) t0 += li[k] * lj[k];
      L[(size_t)i * N + j] = (-M[(size_t)i * N + j] - ((t0 + t1) + (t2 + t3))) / ljj;
    }
    __syncthreads();  // column j is complete before row j + 1 is staged
  }
  if (tid == 0) *info = 0;
}

// T = L^-1 (lower triangular), one column per thread (the columns are
// independent: column c solves L t = e_c by forward substitution, rows in
// order, four partial sums per row); skipped unless the factorisation
// succeeded.
__global__ __launch_bounds__(256) void k_tri_inv(const double *__restrict__ L, int N, const int *__restrict__ info,
                                                 double *__restrict__ T) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= N || *info != 0) return;
  for (int i = 0; i < c; ++i) T[(size_t)i * N + c] = 0.0;
  T[(size_t)c * N + c] = 1.0 / L[(size_t)c * N + c];
  for (int i = c + 1; i < N; ++i) {
    const double *li = L + (size_t)i * N;
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, t3 = 0.0;
    int k = c;
    for (; k + 3 < i; k += 4) {
      t0 += li[k] * T[(size_t)k * N + c];
      t1 += li[k + 1] * T[(size_t)(k + 1) * N + c];
      t2 += li[k + 2] * T[(size_t)(k + 2) * N + c];
      t3 += li[k + 3] * T[(size_t)(k + 3) * N + c];
    }
    for (; k < i; ++k) t0 += li[k] * T[(size_t)k * N + c];
    T[(size_t)i * N + c] = -((t0 + t1) + (t2 + t3)) / L[(size_t)i * N + i];
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
// Grid points per chunk of the Gram kernel: about 2048 workgroups in all,
// chunks of at least 256 points, a multiple of the slice.
static long long gram_chunk_len(int NX, int NY, long long ng) {
  const long long tiles = (long long)((NX + GT - 1) / GT) * ((NY + GT - 1) / GT);
  long long nch = (2048 + tiles - 1) / tiles;
  const long long maxch = ng / 256;
  if (nch > maxch) nch = maxch;
  if (nch < 1) nch = 1;
  const long long chunk = (ng + nch - 1) / nch;
  return (chunk + GS - 1) / GS * GS;
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
  const long long blocks = (long long)nchunks * ((NX + GT - 1) / GT) * ((NY + GT - 1) / GT);
  hipLaunchKernelGGL((k_gram<TX, TY>), dim3((unsigned)blocks), dim3(256), 0, s, X, NX, Y, NY, D.n0, D.n1, D.n2,
                     qdev[0], qdev[1], qdev[2], chunk, nchunks, part);
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
  if (N > CHOL_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_chol, dim3(1), dim3(256), 0, s, M, N, L, info);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tri_inv, dim3((N + 255) / 256), dim3(256), 0, s, L, N, (const int *)info, T);
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
