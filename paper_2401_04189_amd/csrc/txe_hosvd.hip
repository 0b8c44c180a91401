// Bases shared by all pairs (eq. `TuckerDecompField` with one set of factors
// for every pair): per mode d, the leading eigenvectors of the Gram matrix of
// the mode-d unfolding of every sqrt(w)-scaled pair density psi_i psi_j
// (i over the targets, j over all orbitals), i.e. a higher-order SVD of the
// stacked pair densities, without forming any pair density:
//
//   S_d[a][a'] = sqrt(q_a q_a') sum_m q(m) D_T(a, a', m) D(a, a', m),
//   D(a, a', m) = sum_i psi_i(a, m) psi_i(a', m)   (all orbitals),
//   D_T         = the same sum over the targets,
//
// m running over the other two grid indices with weight q(m) (the Gram
// identity: sum_{i,j} rho_ij(a,m) rho_ij(a',m) factorises over i and j).
//
//   k_hv_pack    a chunk of m values of the orbitals, transposed to
//                [m][i][a] (FP64) so that a fragment row is contiguous
//   k_hv_gram    one wavefront per (16 x 16 tile of S, group of m values):
//                D and D_T of each m on 16x16x4 FP64 MFMA, their product
//                weighted by q(m) accumulated on the accumulator registers;
//                partial tiles per group
//   k_hv_reduce  S = the groups' partial tiles summed in a fixed order, the
//                sqrt(q) scaling, mirrored to the lower triangle
//   k_hv_jacobi  S = V diag(lambda) V^T by cyclic Jacobi rotations with S and
//                V in global memory (one workgroup; n <= 512)
#include <algorithm>
#include <cmath>
#include <vector>

#include "txe_dev.h"

namespace txe {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

// T[ml][i][a] = psi_i at mode-d index a and other-index m0 + ml (FP64)
template <typename Tin>
__global__ __launch_bounds__(256) void k_hv_pack(const Tin *__restrict__ psi, Dims D, int d, int N, long long m0,
                                                 int mc, double *__restrict__ T) {
  const int nd = d == 0 ? D.n0 : d == 1 ? D.n1 : D.n2;
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  const long long total = (long long)mc * N * nd;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int a = (int)(e % nd);
    const int i = (int)((e / nd) % N);
    const long long m = m0 + e / ((long long)nd * N);
    long long g;  // grid index of (a at mode d, m over the other two in C order)
    if (d == 0) g = (long long)a * D.n1 * D.n2 + m;
    else if (d == 1) g = ((m / D.n2) * D.n1 + a) * D.n2 + (m % D.n2);
    else g = m * D.n2 + a;
    T[e] = (double)psi[(size_t)i * ng + g];
  }
}

// One wavefront per (upper tile pair (ta <= tb), group of m values of the
// chunk).  Spart[group][ta][tb] holds the group's 16 x 16 partial tile in the
// FP64 accumulator layout ([v][lane]), summed over the chunks in order.
__global__ __launch_bounds__(256) void k_hv_gram(const double *__restrict__ T, int N, int t0, int nt, int nd, int mc,
                                                 long long m0, const double *__restrict__ qm, int ngroups,
                                                 int chunk_index, double *__restrict__ Spart) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int ntile = (nd + 15) >> 4;
  const int npairs_t = ntile * (ntile + 1) / 2;
  const long long item = (long long)blockIdx.x * 4 + wave;
  if (item >= (long long)npairs_t * ngroups) return;  // whole wavefront
  const int grp = (int)(item / npairs_t);
  int tp = (int)(item % npairs_t), ta = 0;
  while (tp >= ntile - ta) {  // upper-triangle tile pair number -> (ta, tb)
    tp -= ntile - ta;
    ++ta;
  }
  const int tb = ta + tp;
  const int per = (mc + ngroups - 1) / ngroups;
  const int ml0 = grp * per, ml1 = min(mc, ml0 + per);
  const int a = 16 * ta + lr, b = 16 * tb + lr;
  const bool va = a < nd, vb = b < nd;
  const int ac = va ? a : nd - 1, bc = vb ? b : nd - 1;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  const bool same = t0 == 0 && nt == N;
  for (int ml = ml0; ml < ml1; ++ml) {
    const double *Tm = T + (size_t)ml * N * nd;
    d4 Dm = {0.0, 0.0, 0.0, 0.0}, Dt = {0.0, 0.0, 0.0, 0.0};
    for (int i0 = 0; i0 < N; i0 += 4) {
      const int i = i0 + lg;
      const bool vi = i < N;
      const int ic = vi ? i : N - 1;
      const double x = Tm[(size_t)ic * nd + ac], y = Tm[(size_t)ic * nd + bc];
      Dm = __builtin_amdgcn_mfma_f64_16x16x4f64((vi && va) ? x : 0.0, (vi && vb) ? y : 0.0, Dm, 0, 0, 0);
    }
    if (same) {
      Dt = Dm;
    } else {
      for (int i0 = t0; i0 < t0 + nt; i0 += 4) {
        const int i = i0 + lg;
        const bool vi = i < t0 + nt;
        const int ic = vi ? i : t0 + nt - 1;
        const double x = Tm[(size_t)ic * nd + ac], y = Tm[(size_t)ic * nd + bc];
        Dt = __builtin_amdgcn_mfma_f64_16x16x4f64((vi && va) ? x : 0.0, (vi && vb) ? y : 0.0, Dt, 0, 0, 0);
      }
    }
    const double w = qm[m0 + ml];
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[v] += w * Dm[v] * Dt[v];
  }
  // one slot per group, accumulated over the chunks in order
  double *out = Spart + (((size_t)grp * ntile * ntile) + (size_t)ta * ntile + tb) * 256;
#pragma unroll
  for (int v = 0; v < 4; ++v) out[v * 64 + lane] = (chunk_index > 0 ? out[v * 64 + lane] : 0.0) + acc[v];
}

// S[a][b] (n x n) = sqrt(q_a q_b) * sum over the groups (in order) of the
// partial tiles; both triangles written
__global__ __launch_bounds__(256) void k_hv_reduce(const double *__restrict__ Spart, int nparts, int nd,
                                                   const double *__restrict__ q, double *__restrict__ S) {
  const int ntile = (nd + 15) >> 4;
  for (int e = blockIdx.x * 256 + threadIdx.x; e < nd * nd; e += gridDim.x * 256) {
    const int a = e / nd, b = e % nd;
    const int lo = min(a, b), hi = max(a, b);
    const int ta = lo >> 4, tb = hi >> 4;
    // element (lo, hi) of tile (ta, tb): row lo % 16 = 4v + lg, column hi % 16 = lane % 16
    const int rr = lo & 15, cc = hi & 15;
    const int v = rr >> 2, lg = rr & 3;
    const int lane = lg * 16 + cc;
    double s = 0.0;
    for (int k = 0; k < nparts; ++k) s += Spart[((size_t)k * ntile * ntile + (size_t)ta * ntile + tb) * 256 + v * 64 + lane];
    S[e] = sqrt(q[a] * q[b]) * s;
  }
}

// Cyclic Jacobi (round-robin ordering: n/2 disjoint rotations per round, n-1
// rounds per sweep) on A (n x n, symmetric) with V accumulating the
// rotations, both in global memory; one workgroup of 1024 threads.  A
// rotation is skipped when |a_pq| is below 1e-18 sqrt(|a_pp a_qq|) or below
// 1e-17 times the trace (such entries move no leading eigenvector); sweeps
// stop when a sweep rotates nothing, at most 40.  n is even.
__global__ __launch_bounds__(1024) void k_hv_jacobi(double *__restrict__ A, double *__restrict__ V, int n,
                                                    const double *__restrict__ trace_in) {
  __shared__ double cs[256], sn[256];
  __shared__ int pp[256], qq[256];
  __shared__ int rot_any;
  const int tid = threadIdx.x, nth = blockDim.x;
  for (int e = tid; e < n * n; e += nth) V[e] = (e / n == e % n) ? 1.0 : 0.0;
  __syncthreads();
  const double floor_abs = 1e-17 * *trace_in;
  const int h = n / 2, m = n - 1;
  for (int sweep = 0; sweep < 40; ++sweep) {
    if (tid == 0) rot_any = 0;
    __syncthreads();
    for (int t = 0; t < m; ++t) {
      if (tid < h) {
        int a = tid == 0 ? m : (t + tid) % m;
        int b = tid == 0 ? t : (t - tid + m) % m;
        if (a > b) {
          const int x = a;
          a = b;
          b = x;
        }
        const double app = A[(size_t)a * n + a], aqq = A[(size_t)b * n + b], apq = A[(size_t)a * n + b];
        double c = 1.0, s = 0.0;
        if (apq != 0.0 && fabs(apq) > 1e-18 * sqrt(fabs(app * aqq)) && fabs(apq) > floor_abs) {
          const double tau = (aqq - app) / (2.0 * apq);
          const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          rot_any = 1;
        }
        cs[tid] = c;
        sn[tid] = s;
        pp[tid] = a;
        qq[tid] = b;
      }
      __syncthreads();
      for (int e = tid; e < h * n; e += nth) {  // rows a, b
        const int k = e / n, j = e % n;
        if (sn[k] == 0.0) continue;
        const int a = pp[k], b = qq[k];
        const double c = cs[k], s = sn[k];
        const double xa = A[(size_t)a * n + j], xb = A[(size_t)b * n + j];
        A[(size_t)a * n + j] = c * xa - s * xb;
        A[(size_t)b * n + j] = s * xa + c * xb;
      }
      __syncthreads();
      for (int e = tid; e < h * n; e += nth) {  // columns a, b of A and of V
        const int i = e / h, k = e % h;           // lanes along one row: nearby addresses
        if (sn[k] == 0.0) continue;
        const int a = pp[k], b = qq[k];
        const double c = cs[k], s = sn[k];
        const double xa = A[(size_t)i * n + a], xb = A[(size_t)i * n + b];
        A[(size_t)i * n + a] = c * xa - s * xb;
        A[(size_t)i * n + b] = s * xa + c * xb;
        const double va = V[(size_t)i * n + a], vb = V[(size_t)i * n + b];
        V[(size_t)i * n + a] = c * va - s * vb;
        V[(size_t)i * n + b] = s * va + c * vb;
      }
      __syncthreads();
    }
    if (!rot_any) break;  // uniform: read after the last barrier of the sweep
    __syncthreads();
  }
}

__global__ void k_hv_trace(const double *__restrict__ S, int n, double *__restrict__ tr) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < n; ++i) t += fabs(S[(size_t)i * n + i]);
    *tr = t;
  }
}

inline unsigned grid_for(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 65536); }

}  // namespace

hipError_t hosvd_mode_gram(const void *psi, bool psi64, const Dims &D, int d, int N, int t0, int nt,
                           const double *qm_dev, const double *qd_dev, double *T, long long tcap, double *Spart,
                           int ngroups, double *S, hipStream_t s) {
  const int nd = d == 0 ? D.n0 : d == 1 ? D.n1 : D.n2;
  const long long mtot = (long long)D.n0 * D.n1 * D.n2 / nd;
  const long long per_m = (long long)N * nd;
  const int mc = (int)std::max<long long>(1, std::min<long long>(mtot, tcap / per_m));
  const int nchunks = (int)((mtot + mc - 1) / mc);
  const int ntile = (nd + 15) / 16;
  const long long items = (long long)ntile * (ntile + 1) / 2 * ngroups;
  hipError_t e = hipSuccess;
  for (int c = 0; c < nchunks && e == hipSuccess; ++c) {
    const long long m0 = (long long)c * mc;
    const int mcc = (int)std::min<long long>(mc, mtot - m0);
    if (psi64)
      hipLaunchKernelGGL(k_hv_pack<double>, dim3(grid_for((long long)mcc * per_m)), dim3(256), 0, s,
                         (const double *)psi, D, d, N, m0, mcc, T);
    else
      hipLaunchKernelGGL(k_hv_pack<float>, dim3(grid_for((long long)mcc * per_m)), dim3(256), 0, s,
                         (const float *)psi, D, d, N, m0, mcc, T);
    hipLaunchKernelGGL(k_hv_gram, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, s, (const double *)T, N, t0, nt,
                       nd, mcc, m0, qm_dev, ngroups, c, Spart);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hv_reduce, dim3(grid_for((long long)nd * nd)), dim3(256), 0, s, (const double *)Spart,
                     ngroups, nd, qd_dev, S);
  return hipGetLastError();
}

hipError_t hosvd_eigen(double *S, double *V, int n, double *trace_tmp, hipStream_t s) {
  hipLaunchKernelGGL(k_hv_trace, dim3(1), dim3(64), 0, s, (const double *)S, n, trace_tmp);
  hipLaunchKernelGGL(k_hv_jacobi, dim3(1), dim3(1024), 0, s, S, V, n, (const double *)trace_tmp);
  return hipGetLastError();
}

}  // namespace txe
