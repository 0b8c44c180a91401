// Projection of the pair densities onto the shared Tucker bases (eq.
// `TuckerDecompField` with bases shared by all pairs):
//   proj12  pair density rho = psi_i psi_j formed on load; T1 = rho x2 V2^T
//           (mode-2 product) chained on the MFMA accumulators into
//           T2 = T1 x1 V1^T (mode-1 product), one a-slab per wavefront
//   proj3   G = T2 x0 V0^T (mode-0 product), batched GEMM
#include "txe_dev.h"

namespace txe {

// -------------------------------------------------------------------------------------
// proj12: T2[p][a][beta][gamma] = sum_b V1[b][beta] sum_c psi_i[a,b,c] psi_j[a,b,c] V2[c][gamma]
// one wavefront per (pair, a-slab, group of GT gamma tiles)
// -------------------------------------------------------------------------------------
template <typename T, typename Tin, int GT, bool LDS_TAB>
__global__ __launch_bounds__(256) void k_proj12(const Tin *__restrict__ psi, Dims D, PairMap pm, int P,
                                                Tables<T> tb, T *__restrict__ T2) {
  using M = MF<T>;
  using acc = typename M::acc;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int ngg = (D.MT2 + GT - 1) / GT;
  const int nbt = D.nb1 >> 4, nct = D.nc2 >> 4;
  // the shared operands (V2 and the chained V1 fragments) are staged once per
  // workgroup; the workgroup then walks its items
  const T *V2 = tb.V2B, *V1c = tb.V1chain;
  if constexpr (LDS_TAB) {
    T *s2 = reinterpret_cast<T *>(smem_raw);
    T *s1 = s2 + (size_t)D.nc2 * D.rp2;
    const int m2 = D.nc2 * D.rp2, m1 = D.MT1 * nbt * 256;
    for (int idx = threadIdx.x; idx < m2; idx += 256) s2[idx] = tb.V2B[idx];
    for (int idx = threadIdx.x; idx < m1; idx += 256) s1[idx] = tb.V1chain[idx];
    __syncthreads();
    V2 = s2;
    V1c = s1;
  }
  const long long total = (long long)P * D.n0 * ngg;
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
  const int gg = (int)(item % ngg);
  const long long rest = item / ngg;
  const int a = (int)(rest % D.n0);
  const int p = (int)(rest / D.n0);
  int i, j;
  pair_ij(pm, p, i, j);
  const size_t plane = (size_t)D.n1 * D.n2;
  const Tin *pi = psi + ((size_t)i * D.n0 + a) * plane;
  const Tin *pj = psi + ((size_t)j * D.n0 + a) * plane;
  const int g0 = gg * GT;

  acc T2a[MAX_MT][GT];
#pragma unroll
  for (int mt = 0; mt < MAX_MT; ++mt)
#pragma unroll
    for (int gt = 0; gt < GT; ++gt) T2a[mt][gt] = zero4<acc>();

  for (int mb = 0; mb < nbt; ++mb) {
    acc T1[GT];
#pragma unroll
    for (int gt = 0; gt < GT; ++gt) T1[gt] = zero4<acc>();
    const int b = 16 * mb + lr;
    for (int J = 0; J < nct; ++J) {
      const int c = 16 * J + 4 * lg;
      double x[4] = {0.0, 0.0, 0.0, 0.0};
      if (b < D.n1 && c < D.n2) {
        double y[4];
        load4(pi + (size_t)b * D.n2 + c, x);
        load4(pj + (size_t)b * D.n2 + c, y);
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] *= y[q];
      }
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const T *vrow = V2 + (size_t)(c + jj) * D.rp2 + 16 * g0 + lr;
        const T rho = (T)x[jj];
#pragma unroll
        for (int gt = 0; gt < GT; ++gt)
          if (g0 + gt < D.MT2) T1[gt] = M::mma(rho, vrow[16 * gt], T1[gt]);
      }
    }
#pragma unroll
    for (int mt = 0; mt < MAX_MT; ++mt) {
      if (mt < D.MT1) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T af = V1c[(((size_t)mt * nbt + mb) * 4 + v) * 64 + lane];
#pragma unroll
          for (int gt = 0; gt < GT; ++gt)
            if (g0 + gt < D.MT2) T2a[mt][gt] = M::mma(af, T1[gt][v], T2a[mt][gt]);
        }
      }
    }
  }
  T *out = T2 + ((size_t)p * D.n0 + a) * D.rp1 * D.rp2;
#pragma unroll
  for (int mt = 0; mt < MAX_MT; ++mt) {
    if (mt < D.MT1) {
#pragma unroll
      for (int gt = 0; gt < GT; ++gt) {
        if (g0 + gt < D.MT2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int beta = 16 * mt + drow<T>(lg, v);
            const int gamma = 16 * (g0 + gt) + lr;
            out[(size_t)beta * D.rp2 + gamma] = T2a[mt][gt][v];
          }
        }
      }
    }
  }
  }
}

// proj12, compile-time form: all MT gamma tiles per wavefront (MT = rank
// tiles of every mode), so no per-MFMA guard.  The psi loads run PD c steps
// ahead of their MFMAs in a ring of registers, across the b tiles (slot u
// serves the steps s = u mod PD of the flattened (b tile, c step) order, so
// PD divides the c steps per b tile); addresses are clamped and points past
// the grid are zeroed by a select.  TABS: the shared operands in LDS,
// 2 = V2 and the chained V1 fragments, 1 = V2 only, 0 = neither.
template <typename T, typename Tin, int MT, int TABS, int PD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void k_proj12m(const Tin *__restrict__ psi, Dims D, PairMap pm, int P,
                                                 Tables<T> tb, T *__restrict__ T2) {
  using M = MF<T>;
  using acc = typename M::acc;
  typedef typename std::conditional<sizeof(Tin) == 4, f4, d4>::type V4;
  constexpr int RP = 16 * MT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int nbt = D.nb1 >> 4, nct = D.nc2 >> 4;
  const int S = nbt * nct;
  const T *V2 = tb.V2B, *V1c = tb.V1chain;
  if constexpr (TABS > 0) {
    T *s2 = reinterpret_cast<T *>(smem_raw);
    const int m2 = D.nc2 * RP;
    for (int idx = threadIdx.x; idx < m2; idx += 256) s2[idx] = tb.V2B[idx];
    V2 = s2;
    if constexpr (TABS > 1) {
      T *s1 = s2 + m2;
      const int m1 = MT * nbt * 256;
      for (int idx = threadIdx.x; idx < m1; idx += 256) s1[idx] = tb.V1chain[idx];
      V1c = s1;
    }
    __syncthreads();
  }
  const size_t plane = (size_t)D.n1 * D.n2;
  const long long total = (long long)P * D.n0;
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
    const int a = (int)(item % D.n0);
    const int p = (int)(item / D.n0);
    int i, j;
    pair_ij(pm, p, i, j);
    const Tin *pi = psi + ((size_t)i * D.n0 + a) * plane;
    const Tin *pj = psi + ((size_t)j * D.n0 + a) * plane;
    V4 xq[PD], yq[PD];
    auto issue = [&](int s_, V4 &x, V4 &y) {
      const int mb_ = s_ / nct, J_ = s_ - mb_ * nct;
      const size_t off = (size_t)min(16 * mb_ + lr, D.n1 - 1) * D.n2 + min(16 * J_ + 4 * lg, D.n2 - 4);
      x = *reinterpret_cast<const V4 *>(pi + off);
      y = *reinterpret_cast<const V4 *>(pj + off);
    };
#pragma unroll
    for (int u = 0; u < PD; ++u) issue(min(u, S - 1), xq[u], yq[u]);
    acc T2a[MT][MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int gt = 0; gt < MT; ++gt) T2a[mt][gt] = zero4<acc>();
    for (int mb = 0; mb < nbt; ++mb) {
      acc T1[MT];
#pragma unroll
      for (int gt = 0; gt < MT; ++gt) T1[gt] = zero4<acc>();
      const bool bin = 16 * mb + lr < D.n1;
      for (int J0 = 0; J0 < nct; J0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
          const int J = J0 + u, s = mb * nct + J;
          const int c = 16 * J + 4 * lg;
          const bool in = bin && c < D.n2;
          double x[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) x[q] = in ? (double)xq[u][q] * (double)yq[u][q] : 0.0;
          if (s + PD < S) issue(s + PD, xq[u], yq[u]);
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            const T *vrow = V2 + (size_t)(c + jj) * RP + lr;
            const T rho = (T)x[jj];
#pragma unroll
            for (int gt = 0; gt < MT; ++gt) T1[gt] = M::mma(rho, vrow[16 * gt], T1[gt]);
          }
        }
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T af = V1c[(((size_t)mt * nbt + mb) * 4 + v) * 64 + lane];
#pragma unroll
          for (int gt = 0; gt < MT; ++gt) T2a[mt][gt] = M::mma(af, T1[gt][v], T2a[mt][gt]);
        }
    }
    T *out = T2 + ((size_t)p * D.n0 + a) * RP * RP;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int gt = 0; gt < MT; ++gt)
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(size_t)(16 * mt + drow<T>(lg, v)) * RP + 16 * gt + lr] = T2a[mt][gt][v];
  }
}

// -------------------------------------------------------------------------------------
// proj3: G[p][alpha][f] = sum_a V0[a][alpha] T2[p][a][f], f = (beta, gamma)
// one wavefront per (pair, group of FT f-tiles)
// -------------------------------------------------------------------------------------
template <typename T, int FT, int MT>
__global__ __launch_bounds__(256) void k_proj3(const T *__restrict__ T2, Dims D, int P, Tables<T> tb,
                                               T *__restrict__ G) {
  using M = MF<T>;
  using acc = typename M::acc;
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int NF = (D.rp1 * D.rp2) >> 4;
  const int nfg = (NF + FT - 1) / FT;
  const long long item = (long long)blockIdx.x * 4 + wave;
  if (item >= (long long)P * nfg) return;
  const int fgi = (int)(item % nfg);
  const int p = (int)(item / nfg);
  const int f0 = fgi * FT;
  const size_t F = (size_t)D.rp1 * D.rp2;
  const T *B = T2 + (size_t)p * D.n0 * F;
  // column tiles past the last one read (clamped) tile NF-1 and are not stored
  int fc[FT];
#pragma unroll
  for (int ft = 0; ft < FT; ++ft) fc[ft] = 16 * min(f0 + ft, NF - 1) + lr;

  acc C[MT][FT];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) C[mt][ft] = zero4<acc>();

  // the a loop unrolled by four: the loads of four K = 4 steps are in
  // flight together
#pragma unroll 4
  for (int ka = 0; ka < (D.n0 >> 2); ++ka) {
    const int arow = 4 * ka + lg;
    T bf[FT];
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) bf[ft] = B[(size_t)arow * F + fc[ft]];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const T af = tb.V0K[(size_t)arow * D.rp0 + 16 * mt + lr];
#pragma unroll
      for (int ft = 0; ft < FT; ++ft) C[mt][ft] = M::mma(af, bf[ft], C[mt][ft]);
    }
  }
  T *out = G + (size_t)p * D.rp0 * F;
#pragma unroll
  for (int mt = 0; mt < MT; ++mt) {
#pragma unroll
    for (int ft = 0; ft < FT; ++ft) {
      if (f0 + ft < NF) {
#pragma unroll
        for (int v = 0; v < 4; ++v) out[(size_t)(16 * mt + drow<T>(lg, v)) * F + 16 * (f0 + ft) + lr] = C[mt][ft][v];
      }
    }
  }
}

namespace {

template <typename T, typename Tin, int MT>
void launch_proj12m_mt(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  const unsigned nb = blocks_for((long long)a.P * a.D.n0);
  // the tables in LDS up to 80 KiB (two workgroups per CU), else V2 alone,
  // else neither; the grid is then capped and each workgroup walks several items
  const size_t t2 = (size_t)a.D.nc2 * 16 * MT * sizeof(T);
  const size_t t1 = (size_t)MT * (a.D.nb1 >> 4) * 256 * sizeof(T);
  constexpr size_t LIM = 80 * 1024;
  const unsigned nbl = std::min(nb, (unsigned)a.grid_cap);
  // psi loads two c steps ahead where the c steps per b tile are even
  const bool pd2 = ((a.D.nc2 >> 4) & 1) == 0;
  auto go = [&](auto tabs, size_t lds) {
    constexpr int TB = decltype(tabs)::value;
    if (!pd2) {
      if (lds > 64 * 1024 && hipFuncSetAttribute((const void *)k_proj12m<T, Tin, MT, TB, 1>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
        return;
      hipLaunchKernelGGL((k_proj12m<T, Tin, MT, TB, 1>), dim3(TB ? nbl : nb), dim3(256), lds, s, (const Tin *)a.psi,
                         a.D, a.pm, a.P, tb, a.T2);
      return;
    }
    // above 64 KiB the kernel opts in; a refusal stays the thread's last
    // error, which the caller's launch check reports
    if (lds > 64 * 1024 && hipFuncSetAttribute((const void *)k_proj12m<T, Tin, MT, TB, 2>,
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return;
    hipLaunchKernelGGL((k_proj12m<T, Tin, MT, TB, 2>), dim3(TB ? nbl : nb), dim3(256), lds, s, (const Tin *)a.psi, a.D,
                       a.pm, a.P, tb, a.T2);
  };
  if (t2 + t1 <= LIM) go(std::integral_constant<int, 2>{}, t2 + t1);
  else if (t2 <= LIM) go(std::integral_constant<int, 1>{}, t2);
  else go(std::integral_constant<int, 0>{}, 0);
}

template <typename T, typename Tin>
void launch_proj12m(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  switch (a.D.MT1) {
    case 1: launch_proj12m_mt<T, Tin, 1>(tb, a, s); break;
    case 2: launch_proj12m_mt<T, Tin, 2>(tb, a, s); break;
    case 3: launch_proj12m_mt<T, Tin, 3>(tb, a, s); break;
    case 4: launch_proj12m_mt<T, Tin, 4>(tb, a, s); break;
    default: launch_proj12m_mt<T, Tin, 5>(tb, a, s); break;
  }
}

template <typename T, typename Tin, int GT>
void launch_proj12(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  const int ngg = (a.D.MT2 + GT - 1) / GT;
  const unsigned nb = blocks_for((long long)a.P * a.D.n0 * ngg);
  const size_t tab = ((size_t)a.D.nc2 * a.D.rp2 + (size_t)a.D.MT1 * (a.D.nb1 >> 4) * 256) * sizeof(T);
  if (tab <= 64 * 1024)
    hipLaunchKernelGGL((k_proj12<T, Tin, GT, true>), dim3(std::min(nb, (unsigned)a.grid_cap)), dim3(256), tab, s,
                       (const Tin *)a.psi, a.D, a.pm, a.P, tb, a.T2);
  else
    hipLaunchKernelGGL((k_proj12<T, Tin, GT, false>), dim3(nb), dim3(256), 0, s, (const Tin *)a.psi, a.D, a.pm,
                       a.P, tb, a.T2);
}

// FP64 orbitals rounded to FP32 (two per thread and step)
__global__ __launch_bounds__(256) void k_psi_f32(const double *__restrict__ in, float *__restrict__ out, size_t n) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  typedef float f2 __attribute__((ext_vector_type(2)));
  const size_t n2 = n / 2;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n2; i += (size_t)gridDim.x * 256) {
    const d2 v = reinterpret_cast<const d2 *>(in)[i];
    f2 o;
    o[0] = (float)v[0];
    o[1] = (float)v[1];
    reinterpret_cast<f2 *>(out)[i] = o;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && (n & 1)) out[n - 1] = (float)in[n - 1];
}
template <typename T, typename TinP>
void launch_proj(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  if (a.proj_gt == 4) launch_proj12m<T, TinP>(tb, a, s);
  else if (a.proj_gt == 1) launch_proj12<T, TinP, 1>(tb, a, s);
  else if (a.proj_gt == 3) launch_proj12<T, TinP, 3>(tb, a, s);
  else launch_proj12<T, TinP, 2>(tb, a, s);
}

}  // namespace

template <typename T, typename Tin>
hipError_t launch_projection(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s, Prof *prof) {
  constexpr int FT = 4;
  hipError_t e;
  prof->begin(K_PROJ12, s);
  if constexpr (sizeof(T) == 4 && sizeof(Tin) == 8) {
    if (a.psi32) {
      // the projection reads the FP32 copy (written once per apply, by the
      // first chunk, and counted with its projection)
      if (a.psi32_fill)
        hipLaunchKernelGGL(k_psi_f32, dim3((unsigned)std::min<size_t>((a.psi_elems / 2 + 255) / 256 + 1, 8192)),
                           dim3(256), 0, s, (const double *)a.psi, const_cast<float *>(a.psi32), a.psi_elems);
      ChunkArgs<T> a32 = a;
      a32.psi = a.psi32;
      launch_proj<T, float>(tb, a32, s);
    } else {
      launch_proj<T, Tin>(tb, a, s);
    }
  } else {
    launch_proj<T, Tin>(tb, a, s);
  }
  prof->end(s);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int NF = (a.D.rp1 * a.D.rp2) >> 4;
  const int nfg = (NF + FT - 1) / FT;
  prof->begin(K_PROJ3, s);
  const dim3 g3(blocks_for((long long)a.P * nfg));
  switch (a.D.MT0) {
    case 1: hipLaunchKernelGGL((k_proj3<T, FT, 1>), g3, dim3(256), 0, s, a.T2, a.D, a.P, tb, a.G); break;
    case 2: hipLaunchKernelGGL((k_proj3<T, FT, 2>), g3, dim3(256), 0, s, a.T2, a.D, a.P, tb, a.G); break;
    case 3: hipLaunchKernelGGL((k_proj3<T, FT, 3>), g3, dim3(256), 0, s, a.T2, a.D, a.P, tb, a.G); break;
    case 4: hipLaunchKernelGGL((k_proj3<T, FT, 4>), g3, dim3(256), 0, s, a.T2, a.D, a.P, tb, a.G); break;
    default: hipLaunchKernelGGL((k_proj3<T, FT, 5>), g3, dim3(256), 0, s, a.T2, a.D, a.P, tb, a.G); break;
  }
  prof->end(s);
  return hipGetLastError();
}

template hipError_t launch_projection<double, double>(const Tables<double> &, const ChunkArgs<double> &, hipStream_t,
                                                      Prof *);
template hipError_t launch_projection<float, double>(const Tables<float> &, const ChunkArgs<float> &, hipStream_t,
                                                     Prof *);
template hipError_t launch_projection<float, float>(const Tables<float> &, const ChunkArgs<float> &, hipStream_t,
                                                    Prof *);

}  // namespace txe
