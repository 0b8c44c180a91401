// Per-pair Tucker bases (section "Convolution operation", eq.
// `TuckerDecompField` with factors of each pair): the sequentially truncated
// HOSVD of every pair density, the pair's own core matrices, and the
// back-projection in the pair's bases.  FP64 throughout.  Per chunk of pairs:
//
//   k_pp_rho     X = rho_ij scaled by sqrt(q0 q1 q2) (its Frobenius norm is
//                the W-norm of rho_ij)
//   then for modes d = 0, 1, 2 of the current tensor X:
//     k_pp_gram    S = X_(d) X_(d)^T (FP64 MFMA), the Gram matrix of the
//                  mode-d unfolding
//     k_pp_jacobi  S = V diag(lambda) V^T by cyclic Jacobi rotations in LDS
//                  (one workgroup per pair)
//     mode product B = X x_d V^T, the unfolding in that eigenbasis
//     k_pp_gram    S = B_(d) B_(d)^T, nearly diagonal
//     k_pp_jacobi  its r_d leading eigenvectors Wr
//     k_pp_rotate  Ut_d = V Wr, the leading left singular vectors of X_(d)
//     mode product X <- B x_d Wr^T = X x_d Ut_d^T, the truncation of mode d
//   The second stage recovers the accuracy the Gram matrix loses: one
//   eigen-decomposition of X X^T fixes a singular vector only to about
//   eps sigma_1^2 / (sigma_i^2 - sigma_j^2), while the rows of B carry their
//   own scale, so Jacobi on B B^T (relative accuracy for such graded,
//   nearly diagonal matrices) fixes it to about eps sigma_1 / (sigma_i -
//   sigma_j), as an SVD of X_(d) does.
//   k_pp_pad     the core G in the padded layout of the core kernel
//   k_pp_tables  Chat_k^d = V_d^T C_k^d U_d = Ut_d^T (D C_k^d D^-1) Ut_d
//                (D = diag(sqrt(q_d))) written in the core kernel's FP64
//                table layouts, plus the U0 fragments of its epilogue
//   core kernel  (the shared-basis kernel, tables offset per pair)
//   mode products S1 x U2, then x U1: phi of every pair
//   accumulation Vx psi_t -= sum_s psi_s phi_ts, sources ascending
//
// U_d = Ut_d / sqrt(q_d) is q-orthonormal, V_d = diag(q_d) U_d, so G, Phi and
// e_ij = <G, Phi> keep the meaning they have with shared bases.
#include "txe_dev.h"
#include "txe_modes.h"

namespace txe {

// X[p] = sqrt(q0[a] q1[b] q2[c]) psi_i[a,b,c] psi_j[a,b,c] for every pair of the chunk
__global__ __launch_bounds__(256) void k_pp_rho(const double *__restrict__ psi, Dims D, PairMap pm, int P,
                                                const double *__restrict__ q0, const double *__restrict__ q1,
                                                const double *__restrict__ q2, double *__restrict__ X) {
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  const long long total = (long long)P * ng;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int p = (int)(e / ng);
    const long long g = e - (long long)p * ng;
    const int c = (int)(g % D.n2);
    const int b = (int)((g / D.n2) % D.n1);
    const int a = (int)(g / ((long long)D.n1 * D.n2));
    int i, j;
    pair_ij(pm, p, i, j);
    X[e] = sqrt(q0[a] * q1[b] * q2[c]) * psi[(size_t)i * ng + g] * psi[(size_t)j * ng + g];
  }
}

// S[p] = X_(d) X_(d)^T for tensors of extents (A, B, C) (pair stride A B C),
// nd = extent along d, S stored n x n with leading dimension ld.  One
// wavefront per (pair, 16 x 16 tile of S); K = 4 MFMA steps over the
// unfolding's columns, the tail and the rows past nd masked to zero.
__global__ __launch_bounds__(256) void k_pp_gram(const double *__restrict__ X, int P, int d, int A, int B, int C,
                                                 int ld, double *__restrict__ S) {
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nd = d == 0 ? A : d == 1 ? B : C;
  const int nt = (nd + 15) >> 4;
  const long long item = (long long)blockIdx.x * 4 + wave;
  if (item >= (long long)P * nt * nt) return;  // whole wavefront (item is uniform)
  const int tj = (int)(item % nt), ti = (int)((item / nt) % nt), p = (int)(item / ((long long)nt * nt));
  const long long vol = (long long)A * B * C;
  const long long M = vol / nd;
  const double *Xp = X + (size_t)p * vol;
  const int ri = 16 * ti + lr, rj = 16 * tj + lr;
  const bool vi = ri < nd, vj = rj < nd;
  const int ci = vi ? ri : nd - 1, cj = vj ? rj : nd - 1;
  typedef double d4 __attribute__((ext_vector_type(4)));
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (long long m0 = 0; m0 < M; m0 += 4) {
    const long long m = m0 + lg;
    const bool vm = m < M;
    const long long mm = vm ? m : M - 1;
    const double xa = Xp[unfold_at(d, B, C, ci, mm)];
    const double xb = Xp[unfold_at(d, B, C, cj, mm)];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64((vi && vm) ? xa : 0.0, (vj && vm) ? xb : 0.0, acc, 0, 0, 0);
  }
  double *Sp = S + (size_t)p * ld * ld;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 16 * ti + 4 * v + lg, col = 16 * tj + lr;  // FP64 accumulator row order
    if (row < nd && col < nd) Sp[(size_t)row * ld + col] = acc[v];
  }
}

// Eigen-decomposition of one symmetric n x n matrix per workgroup by cyclic
// Jacobi rotations (round-robin ordering: n/2 disjoint rotations per round,
// n - 1 rounds per sweep, sweeps until every off-diagonal entry is
// negligible against its diagonal pair, at most 30), S and the rotation
// product V in LDS.  Writes the eigenvectors of the r largest eigenvalues
// (descending, ties by index) as the columns of Ut[p] (n x r, row-major,
// pair stride ostride).  n is even (the grid extents are multiples of 4).
__global__ __launch_bounds__(256) void k_pp_jacobi(const double *__restrict__ S, int n, int ld, int r,
                                                   double *__restrict__ Ut, long long ostride) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *As = reinterpret_cast<double *>(smem_raw);   // n x n
  double *Vs = As + n * n;                             // n x n
  __shared__ double cs[64], sn[64];
  __shared__ int pp[64], qq[64];
  __shared__ int rot_any;
  const int tid = threadIdx.x;
  const int p = blockIdx.x;
  const double *Sp = S + (size_t)p * ld * ld;
  for (int e = tid; e < n * n; e += 256) {
    const int i = e / n, j = e % n;
    As[e] = 0.5 * (Sp[(size_t)i * ld + j] + Sp[(size_t)j * ld + i]);  // exactly symmetric
    Vs[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int h = n / 2, m = n - 1;
  for (int sweep = 0; sweep < 30; ++sweep) {
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
        const double app = As[a * n + a], aqq = As[b * n + b], apq = As[a * n + b];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > 1e-18 * sqrt(fabs(app * aqq)) && apq != 0.0) {
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
      // rows a, b of S (left factor J^T)
      for (int e = tid; e < h * n; e += 256) {
        const int k = e / n, j = e % n;
        const int a = pp[k], b = qq[k];
        const double c = cs[k], s = sn[k];
        const double xa = As[a * n + j], xb = As[b * n + j];
        As[a * n + j] = c * xa - s * xb;
        As[b * n + j] = s * xa + c * xb;
      }
      __syncthreads();
      // columns a, b of S and of V (right factor J); consecutive lanes take
      // consecutive rotations of one row (distinct columns, distinct banks)
      for (int e = tid; e < h * n; e += 256) {
        const int i = e / h, k = e % h;
        const int a = pp[k], b = qq[k];
        const double c = cs[k], s = sn[k];
        const double xa = As[i * n + a], xb = As[i * n + b];
        As[i * n + a] = c * xa - s * xb;
        As[i * n + b] = s * xa + c * xb;
        const double va = Vs[i * n + a], vb = Vs[i * n + b];
        Vs[i * n + a] = c * va - s * vb;
        Vs[i * n + b] = s * va + c * vb;
      }
      __syncthreads();
    }
    if (!rot_any) break;  // uniform: read after the last barrier of the sweep
    __syncthreads();
  }
  // rank of each eigenvalue (descending, ties by index), then the r leading
  // eigenvectors as columns of Ut
  double *Up = Ut + (size_t)p * ostride;
  for (int i = tid; i < n; i += 256) {
    const double li = As[i * n + i];
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      const double lj = As[j * n + j];
      rank += (lj > li || (lj == li && j < i)) ? 1 : 0;
    }
    if (rank < r)
      for (int row = 0; row < n; ++row) Up[(size_t)row * r + rank] = Vs[row * n + i];
  }
}

// Ut[p] = V[p] Wr[p]: V n x n (row-major), Wr n x r (row-major), both with
// pair stride vs; Ut n x r with pair stride us
__global__ __launch_bounds__(256) void k_pp_rotate(const double *__restrict__ V, const double *__restrict__ Wr,
                                                   long long vs, int n, int r, double *__restrict__ Ut, long long us,
                                                   int P) {
  const long long per = (long long)n * r;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < (long long)P * per; e += (long long)gridDim.x * 256) {
    const int p = (int)(e / per);
    const int f = (int)(e - (long long)p * per);
    const int a = f / r, s = f % r;
    const double *Vp = V + (size_t)p * vs + (size_t)a * n;
    const double *Wp = Wr + (size_t)p * vs + s;
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc += Vp[i] * Wp[(size_t)i * r];
    Ut[(size_t)p * us + f] = acc;
  }
}

// G[p] in the core kernel's padded layout RP^3 (zeros past the ranks) from
// the dense r0 x r1 x r2 core
__global__ __launch_bounds__(256) void k_pp_pad(const double *__restrict__ X3, Dims D, int P, double *__restrict__ G) {
  const int RP = D.rp0;
  const long long F3 = (long long)RP * RP * RP, v3 = (long long)D.r0 * D.r1 * D.r2;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < (long long)P * F3; e += (long long)gridDim.x * 256) {
    const int p = (int)(e / F3);
    const long long f = e - (long long)p * F3;
    const int g = (int)(f % RP), b = (int)((f / RP) % RP), a = (int)(f / ((long long)RP * RP));
    G[e] = (a < D.r0 && b < D.r1 && g < D.r2) ? X3[(size_t)p * v3 + ((size_t)a * D.r1 + b) * D.r2 + g] : 0.0;
  }
}

// Per-pair core matrices of mode d and term k (one workgroup each), from
// Ut_d (n x r): T = Cs_k Ut (n x r, in LDS), Chat = Ut^T T (r x r), written
// in the core kernel's FP64 layouts (zeros in the padding and for k >= K):
//   d = 0: Ahat[alpha][k][alpha'] = w_k Chat0_k[alpha'][alpha]   ([r0][Kp][rp])
//   d = 1: C1f[k][beta][beta'] = Chat1_k[beta'][beta]           ([Kp][rp][rp])
//   d = 2: C2chain[k][mt'][mg][v][l] = Chat2_k[16mt' + l%16][16mg + 4v + l/16]
// Cs_k = D C_k^d D^-1 with D = diag(sqrt(q_d)) ([K][n][n], FP64).
__global__ __launch_bounds__(256) void k_pp_tables(const double *__restrict__ Ut, long long ustride, int d, int n,
                                                   int r, Dims D, const double *__restrict__ Cs,
                                                   const double *__restrict__ w, double *__restrict__ tab,
                                                   long long tstride) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double *Ts = reinterpret_cast<double *>(smem_raw);  // n x r
  const int k = blockIdx.x % D.Kp;
  const int p = blockIdx.x / D.Kp;
  const int RP = D.rp0, MT = D.MT0;
  const double *U = Ut + (size_t)p * ustride;
  double *tp = tab + (size_t)p * tstride;
  const bool live = k < D.K;
  if (live) {
    const double *Ck = Cs + (size_t)k * n * n;
    for (int e = threadIdx.x; e < n * r; e += 256) {
      const int a = e / r, s = e % r;
      double acc = 0.0;
      for (int b = 0; b < n; ++b) acc += Ck[(size_t)a * n + b] * U[(size_t)b * r + s];
      Ts[e] = acc;
    }
  }
  __syncthreads();
  auto chat = [&](int pr, int s) -> double {  // Chat_k[pr][s]
    if (!live || pr >= r || s >= r) return 0.0;
    double acc = 0.0;
    for (int a = 0; a < n; ++a) acc += U[(size_t)a * r + pr] * Ts[a * r + s];
    return acc;
  };
  if (d == 0) {
    for (int e = threadIdx.x; e < D.r0 * RP; e += 256) {
      const int al = e / RP, ap = e % RP;
      tp[((size_t)al * D.Kp + k) * RP + ap] = live ? w[k] * chat(ap, al) : 0.0;
    }
  } else if (d == 1) {
    for (int e = threadIdx.x; e < RP * RP; e += 256) {
      const int be = e / RP, bp = e % RP;
      tp[((size_t)k * RP + be) * RP + bp] = chat(bp, be);
    }
  } else {
    for (int e = threadIdx.x; e < MT * MT * 256; e += 256) {
      const int l = e & 63, v = (e >> 6) & 3, mg = (e >> 8) % MT, mtp = (e >> 8) / MT;
      tp[(size_t)k * MT * MT * 256 + e] = chat(16 * mtp + (l & 15), 16 * mg + 4 * v + (l >> 4));
      (void)v;
    }
  }
}

// U0 fragments of the core kernel's epilogue (FP64 row order) per pair:
// U0chain[ma][mt][v][l] = U0[a = 16 ma + l%16][alpha' = 16 mt + 4v + l/16],
// U0 = Ut0 / sqrt(q0)
__global__ __launch_bounds__(256) void k_pp_u0chain(const double *__restrict__ Ut0, long long ustride, Dims D,
                                                    const double *__restrict__ q0, int P, double *__restrict__ out,
                                                    long long ostride) {
  const int nat = D.na0 >> 4, MT = D.MT0;
  const long long per = (long long)nat * MT * 256;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < (long long)P * per; e += (long long)gridDim.x * 256) {
    const int p = (int)(e / per);
    const long long f = e - (long long)p * per;
    const int l = (int)(f & 63), v = (int)((f >> 6) & 3), mt = (int)((f >> 8) % MT), ma = (int)((f >> 8) / MT);
    const int a = 16 * ma + (l & 15), ap = 16 * mt + 4 * v + (l >> 4);
    out[(size_t)p * ostride + f] =
        (a < D.n0 && ap < D.r0) ? Ut0[(size_t)p * ustride + (size_t)a * D.r0 + ap] / sqrt(q0[a]) : 0.0;
  }
}

// ------------------------------------------------------------------------------------
// one chunk with per-pair bases
// ------------------------------------------------------------------------------------
namespace {
inline unsigned grid_for(long long n) { return (unsigned)std::min<long long>((n + 255) / 256, 65536); }
inline unsigned waves_grid(long long waves) { return (unsigned)((waves + 3) / 4); }
}  // namespace

hipError_t run_chunk_pp(const Tables<double> &tb, const PairBasesArgs &pb, const ChunkArgs<double> &a, bool want_vx,
                        hipStream_t s, Prof *prof) {
  const Dims &D = a.D;
  const int P = a.P;
  const int n[3] = {D.n0, D.n1, D.n2};
  const int r[3] = {D.r0, D.r1, D.r2};
  const long long ng = (long long)D.n0 * D.n1 * D.n2;
  hipError_t e;
  prof->begin(K_PROJ12, s);
  // scaled pair densities, then the sequential truncation mode by mode
  hipLaunchKernelGGL(k_pp_rho, dim3(grid_for((long long)P * ng)), dim3(256), 0, s, (const double *)a.psi, D, a.pm, P,
                     a.qdev[0], a.qdev[1], a.qdev[2], pb.X);
  const double *cur = pb.X;
  int ext[3] = {D.n0, D.n1, D.n2};
  double *nxt[3] = {pb.X1, pb.X2, pb.X3};
  const long long ss = (long long)pb.ldS * pb.ldS;  // pair stride of S, V and Wr
  for (int d = 0; d < 3; ++d) {
    const long long vol = (long long)ext[0] * ext[1] * ext[2];
    const int nt = (n[d] + 15) / 16;
    const size_t lds = (size_t)2 * n[d] * n[d] * sizeof(double);
    if (lds > 64 * 1024) {
      if ((e = hipFuncSetAttribute((const void *)k_pp_jacobi, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
          hipSuccess)
        return e;
    }
    // first stage: eigenvectors V of X_(d) X_(d)^T, then B = X x_d V^T
    hipLaunchKernelGGL(k_pp_gram, dim3(waves_grid((long long)P * nt * nt)), dim3(256), 0, s, cur, P, d, ext[0],
                       ext[1], ext[2], pb.ldS, pb.S);
    hipLaunchKernelGGL(k_pp_jacobi, dim3(P), dim3(256), lds, s, (const double *)pb.S, n[d], pb.ldS, n[d], pb.V, ss);
    if ((e = launch_mode_f64(cur, vol, ext[0], ext[1], ext[2], d, n[d], pb.V, ss, n[d], 0, n[d], nullptr, 1.0, 0, pb.B,
                             vol, P, s)) != hipSuccess)
      return e;
    // second stage: the r_d leading eigenvectors Wr of B_(d) B_(d)^T, Ut_d = V Wr
    hipLaunchKernelGGL(k_pp_gram, dim3(waves_grid((long long)P * nt * nt)), dim3(256), 0, s, (const double *)pb.B, P,
                       d, ext[0], ext[1], ext[2], pb.ldS, pb.S);
    hipLaunchKernelGGL(k_pp_jacobi, dim3(P), dim3(256), lds, s, (const double *)pb.S, n[d], pb.ldS, r[d], pb.Wr, ss);
    hipLaunchKernelGGL(k_pp_rotate, dim3(grid_for((long long)P * n[d] * r[d])), dim3(256), 0, s, (const double *)pb.V,
                       (const double *)pb.Wr, ss, n[d], r[d], pb.Ut[d], (long long)n[d] * r[d], P);
    // truncation: X <- B x_d Wr^T
    int oext[3] = {ext[0], ext[1], ext[2]};
    oext[d] = r[d];
    const long long ovol = (long long)oext[0] * oext[1] * oext[2];
    if ((e = launch_mode_f64(pb.B, vol, ext[0], ext[1], ext[2], d, n[d], pb.Wr, ss, r[d], 0, r[d], nullptr, 1.0, 0,
                             nxt[d], ovol, P, s)) != hipSuccess)
      return e;
    cur = nxt[d];
    ext[d] = r[d];
  }
  prof->end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  prof->begin(K_PROJ3, s);
  hipLaunchKernelGGL(k_pp_pad, dim3(grid_for((long long)P * D.rp0 * D.rp0 * D.rp0)), dim3(256), 0, s, pb.X3, D, P,
                     a.G);
  // per-pair tables in the core kernel's layouts
  double *tabs[3] = {tb.Ahat, tb.C1f, tb.C2chain};
  const long long tstr[3] = {pb.ps_ah, pb.ps_c1, pb.ps_c2};
  for (int d = 0; d < 3; ++d) {
    const size_t lds = (size_t)n[d] * r[d] * sizeof(double);
    if (lds > 64 * 1024) {
      if ((e = hipFuncSetAttribute((const void *)k_pp_tables, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) !=
          hipSuccess)
        return e;
    }
    hipLaunchKernelGGL(k_pp_tables, dim3((unsigned)((long long)P * D.Kp)), dim3(256), lds, s, (const double *)pb.Ut[d],
                       (long long)n[d] * r[d], d, n[d], r[d], D, pb.Cs[d], pb.w, tabs[d], tstr[d]);
  }
  if (want_vx)
    hipLaunchKernelGGL(k_pp_u0chain, dim3(grid_for((long long)P * (D.na0 / 16) * D.MT0 * 256)), dim3(256), 0, s,
                       (const double *)pb.Ut[0], (long long)D.n0 * D.r0, D, a.qdev[0], P, tb.U0chain, pb.ps_u0);
  prof->end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the core kernel with the tables offset per pair
  prof->begin(K_CORE, s);
  e = launch_core_f64(tb, a, want_vx, s);
  prof->end(s);
  if (e != hipSuccess) return e;
  {
    const int parts = D.MT1 * a.NGS;
    prof->begin(K_EPAIR, s);
    e = launch_epair(a.epart, P, parts, a.pm, a.epair, s);
    prof->end(s);
    if (e != hipSuccess) return e;
  }
  if (!want_vx) return hipSuccess;
  prof->begin(K_BACK, s);
  // S1[p] (n0 x RP(gamma') x RP(beta'), rows gamma' < r2) x_gamma' U2 -> (n0, n2, RP), then x_beta' U1 -> phi [a][c][b]
  {
    const int RP = D.rp0;
    e = launch_mode_f64(a.S1, (long long)D.n0 * RP * RP, D.n0, RP, RP, 1, D.r2, pb.Ut[2], (long long)D.n2 * D.r2,
                        D.r2, 1, D.n2, a.qdev[2], 1.0, 0, pb.X1, (long long)D.n0 * D.n2 * RP, P, s);
    if (e == hipSuccess)
      e = launch_mode_f64(pb.X1, (long long)D.n0 * D.n2 * RP, D.n0, D.n2, RP, 2, D.r1, pb.Ut[1],
                          (long long)D.n1 * D.r1, D.r1, 1, D.n1, a.qdev[1], 1.0, 0, pb.X, ng, P, s);
  }
  for (int b = 0; b < a.nbr && e == hipSuccess; ++b)
    e = launch_accum_f64(pb.X, 1, (const double *)a.psi, D, a.pm, a.br[b], (double *)a.vx, a.out_scale, a.weighted,
                         a.qdev, s);
  prof->end(s);
  return e;
}

}  // namespace txe
