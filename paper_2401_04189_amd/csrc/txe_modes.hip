// Generic FP64 tensor-mode products on 16x16x4 FP64 MFMA and the Hadamard
// accumulation of Vx psi over sources (see txe_modes.h).
#include <algorithm>

#include "txe_dev.h"
#include "txe_modes.h"

namespace txe {

namespace {

// One workgroup per (pair, 64 rows of o, 64 columns of the unfolding): the
// contraction runs over chunks of KC values of i; per chunk the 64 x KC block
// of M and the KC x 64 block of X are loaded into LDS with coalesced reads
// (along each operand's contiguous index) and each wavefront accumulates a
// 32 x 32 corner (2 x 2 MFMA tiles) from LDS.  For mode 2, whose output is
// contiguous along o, X is the A operand so that the lanes of an accumulator
// row run along o.
constexpr int LT = 64;      // output tile edge
constexpr int KC = 64;      // contraction chunk (at most)
constexpr int XS = LT + 2;  // padded row of the X block
// the chunk a product uses (nin rounded up to 4, at most KC) and the padded M
// row: the LDS is sized by them, so short contractions fit three blocks per CU
__host__ __device__ inline int kc_of(int nin) { return nin < KC ? (nin + 3) & ~3 : KC; }
// Element (row i, column j) of the mode-d unfolding of an (A, B, C) tensor
// sits at col_off(j) + i * row_stride: the column part is formed once per
// thread and block (a thread keeps its column across the K chunks), so no
// division runs per element.
__device__ __forceinline__ long long col_off(int d, int B, int C, long long j) {
  if (d == 0) return j;
  if (d == 1) {
    const unsigned long long q = (unsigned long long)j / (unsigned)C;  // once per thread and block
    return (long long)q * B * C + (long long)(j - (long long)q * C);
  }
  return j * C;
}
__device__ __forceinline__ long long row_stride(int d, int B, int C) {
  return d == 0 ? (long long)B * C : d == 1 ? (long long)C : 1;
}

__global__ __launch_bounds__(256) void k_mode_lds(const double *__restrict__ X, long long xs, int A, int B, int C,
                                                  int d, int nin, const double *__restrict__ Mm, long long ms, int ldm,
                                                  int Mt, int nout, const double *__restrict__ qout, double yscale,
                                                  int accum, double *__restrict__ Y, long long ys) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int kc = kc_of(nin), MS = kc + 2;
  double *Ms = reinterpret_cast<double *>(smem_raw);  // [LT][MS]: M(i, o) at [o][i - c0]
  double *Xs = Ms + LT * MS;                          // [kc][XS]: X(i, j) at [i - c0][j - j0]
  const int tid = threadIdx.x, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int ext = d == 0 ? A : d == 1 ? B : C;
  const long long J = (long long)A * B * C / ext;
  const int Bo = d == 1 ? nout : B, Co = d == 2 ? nout : C;
  const int nto = (nout + LT - 1) / LT;
  const long long ntj = (J + LT - 1) / LT;
  const long long blk = blockIdx.x;
  const long long tj = blk % ntj;
  const int to = (int)((blk / ntj) % nto);
  const int p = (int)(blk / (ntj * nto));
  const double *Xp = X + (size_t)p * xs;
  const double *Mp = Mm + (size_t)p * ms;
  const int o0 = LT * to;
  const long long j0 = LT * tj;
  const int ob = 32 * (wave >> 1), jb = 32 * (wave & 1);
  const long long xr = row_stride(d, B, C);
  // modes 0 and 1: X is staged along j, and thread tid keeps column tid mod LT
  // in every pass of the staging loop (256 is a multiple of LT)
  const long long jt = j0 + (tid % LT);
  const long long xcol = d != 2 && jt < J ? col_off(d, B, C, jt) : 0;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = (d4){0.0, 0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < nin; c0 += kc) {
    const int nc = min(kc, nin - c0), NI = (nc + 3) & ~3;
    // M block, read along its contiguous index
    for (int e = tid; e < LT * NI; e += 256) {
      int o, i;
      if (Mt) { o = e / NI; i = e % NI; } else { i = e / LT; o = e % LT; }
      const int og = o0 + o, ig = c0 + i;
      Ms[o * MS + i] = (og < nout && i < nc) ? (Mt ? Mp[(size_t)og * ldm + ig] : Mp[(size_t)ig * ldm + og]) : 0.0;
    }
    // X block, read along its contiguous index (j for modes 0 and 1, i for mode 2)
    if (d == 2) {
      for (int e = tid; e < LT * NI; e += 256) {
        const int jl = e / NI, i = e % NI;
        const long long j = j0 + jl;
        Xs[i * XS + jl] = (j < J && i < nc) ? Xp[j * C + c0 + i] : 0.0;
      }
    } else {
      for (int e = tid; e < LT * NI; e += 256) {
        const int i = e / LT, jl = e % LT;  // jl == tid % LT
        Xs[i * XS + jl] = (jt < J && i < nc) ? Xp[xcol + (long long)(c0 + i) * xr] : 0.0;
      }
    }
    __syncthreads();
    if (d == 2) {
#pragma unroll 2
      for (int i0 = 0; i0 < NI; i0 += 4) {
        double xv[2], mv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) xv[a] = Xs[(i0 + lg) * XS + jb + 16 * a + lr];
#pragma unroll
        for (int b = 0; b < 2; ++b) mv[b] = Ms[(ob + 16 * b + lr) * MS + i0 + lg];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[a], mv[b], acc[a][b], 0, 0, 0);
      }
    } else {
#pragma unroll 2
      for (int i0 = 0; i0 < NI; i0 += 4) {
        double av[2], bv[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) av[a] = Ms[(ob + 16 * a + lr) * MS + i0 + lg];
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Xs[(i0 + lg) * XS + jb + 16 * b + lr];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();  // the next chunk overwrites the blocks
  }
  double *Yp = Y + (size_t)p * ys;
  const long long yr = row_stride(d, Bo, Co);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    // the lane's fixed index of tile t: column j (modes 0, 1) or row o (mode 2)
    const int fo = o0 + ob + 16 * t + lr;
    const long long fj = j0 + jb + 16 * t + lr;
    const long long ycol = d != 2 && fj < J ? col_off(d, Bo, Co, fj) : 0;
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // FP64 accumulator row 4v + lg, column lr of tile (a, b)
        int o;
        long long j, at;
        double r;
        if (d == 2) {  // tile (a = u, b = t): lanes along o
          o = fo;
          j = j0 + jb + 16 * u + 4 * v + lg;
          at = j * Co + o;
          r = acc[u][t][v];
        } else {  // tile (a = u, b = t): lanes along j
          o = o0 + ob + 16 * u + 4 * v + lg;
          j = fj;
          at = ycol + (long long)o * yr;
          r = acc[u][t][v];
        }
        if (o < nout && j < J) {
          double val = yscale * (qout ? r / sqrt(qout[o]) : r);
          double *y = Yp + at;
          if (accum) val += *y;
          *y = val;
        }
      }
  }
}

__global__ __launch_bounds__(256) void k_accum(const double *__restrict__ phi, int phi_acb,
                                               const double *__restrict__ psi, Dims D, PairMap pm, BackRange br,
                                               double *__restrict__ vx, const double *__restrict__ out_scale,
                                               int weighted, const double *__restrict__ q0,
                                               const double *__restrict__ q1, const double *__restrict__ q2) {
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  const long long total = (long long)br.nt * ng;
  const double scale = out_scale ? *out_scale : 1.0;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int tl = (int)(e / ng);
    const long long g = e - (long long)tl * ng;
    const int c = (int)(g % D.n2), b = (int)((g / D.n2) % D.n1), a = (int)(g / ((long long)D.n1 * D.n2));
    const int t = br.t0 + tl;
    double *out = vx + (size_t)(t - br.out0) * ng + g;
    double acc = br.acc_in ? *out : 0.0;
    const long long pg = phi_acb ? ((long long)a * D.n2 + c) * D.n1 + b : g;
    for (int s = br.s0; s < br.s0 + br.ns; ++s) {
      const long long pl = local_pair(pm, br, t, s);
      acc += psi[(size_t)s * ng + g] * phi[(size_t)pl * ng + pg];
    }
    if (br.finish) {
      double val = -scale * acc;
      if (weighted) val *= q0[a] * q1[b] * q2[c];
      *out = val;
    } else {
      *out = acc;
    }
  }
}

inline unsigned grid_for(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 65536); }

}  // namespace

hipError_t launch_mode_f64(const double *X, long long xs, int A, int B, int C, int d, int nin, const double *M,
                           long long ms, int ldm, int Mt, int nout, const double *qout, double yscale, int accum,
                           double *Y, long long ys, int P, hipStream_t s) {
  const int ext = d == 0 ? A : d == 1 ? B : C;
  const long long J = (long long)A * B * C / ext;
  const long long blocks = (long long)P * ((nout + LT - 1) / LT) * ((J + LT - 1) / LT);
  const int kc = kc_of(nin);
  // the launch takes what its chunk needs (42.6 KB at nin = 40); the opt-in is the largest
  const size_t lds = ((size_t)LT * (kc + 2) + (size_t)kc * XS) * sizeof(double);
  constexpr size_t lds_max = ((size_t)LT * (KC + 2) + (size_t)KC * XS) * sizeof(double);  // 67.6 KB
  const hipError_t ea = hipFuncSetAttribute((const void *)k_mode_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                                            (int)lds_max);
  if (ea != hipSuccess) return ea;
  hipLaunchKernelGGL(k_mode_lds, dim3((unsigned)blocks), dim3(256), lds, s, X, xs, A, B, C, d, nin, M, ms, ldm, Mt,
                     nout, qout, yscale, accum, Y, ys);
  return hipGetLastError();
}

hipError_t launch_accum_f64(const double *phi, int phi_acb, const double *psi, const Dims &D, const PairMap &pm,
                            const BackRange &br, double *vx, const double *out_scale, int weighted,
                            const double *const q[3], hipStream_t s) {
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  hipLaunchKernelGGL(k_accum, dim3(grid_for((long long)br.nt * ng)), dim3(256), 0, s, phi, phi_acb, psi, D, pm, br, vx,
                     out_scale, weighted, q[0], q[1], q[2]);
  return hipGetLastError();
}

}  // namespace txe
