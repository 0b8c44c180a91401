// HIP kernels for gfx950 (MI355X): the per-pair Tucker-tensor exchange path.
//
// One chunk of orbital pairs runs through four kernels:
//   proj12  pair density rho = psi_i psi_j formed on load; T1 = rho x2 V2^T
//           (mode-2 product) chained on the MFMA accumulators into
//           T2 = T1 x1 V1^T (mode-1 product), one a-slab per wavefront
//   proj3   G = T2 x0 V0^T (mode-0 product), batched GEMM
//   core    Phi = sum_k w_k G x0 Chat0_k x1 Chat1_k x2 Chat2_k (the kernel
//           sum in the Tucker core space, eqs. `gauss`, `final`), with
//           e_ij = <G, Phi> and the first back-projection S1 = Phi x0 U0 in
//           its epilogue
//   back    phi = S1 x2 U2 x1 U1 (chained), Vx psi_t -= psi_s phi_ts summed
//           over all sources s in registers (eq. `hadam`), no atomics
// followed by a fixed-order FP64 reduction of the pair energies into E_x.
//
// All products use 16x16x4 MFMA tiles (f64 or f32) with 64-lane wavefronts.
// Fragment layouts of a 16x16x4 MFMA for lane l (lr = l%16, lg = l/16):
//   A[m][k]: m = lr, k = lg        B[k][n]: k = lg, n = lr
//   D[m][n]: n = lr, m = 4*lg + v (f32) or m = 4*v + lg (f64), v = 0..3 the
//            four accumulator entries (measured on gfx950)
// so an accumulator whose rows are the next contraction index feeds the next
// MFMA as its B operand directly, one entry v at a time ("chained").
#include <algorithm>
#include <type_traits>

#include "txe_internal.h"

namespace txe {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct MF;
template <>
struct MF<double> {
  typedef d4 acc;
  static __device__ __forceinline__ acc mma(double a, double b, const acc &c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <>
struct MF<float> {
  typedef f4 acc;
  static __device__ __forceinline__ acc mma(float a, float b, const acc &c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// accumulator row held by entry v of lane group lg
template <typename T>
__device__ __forceinline__ int drow(int lg, int v) {
  return sizeof(T) == 8 ? 4 * v + lg : 4 * lg + v;
}

template <typename A>
__device__ __forceinline__ A zero4() {
  A z;
  z[0] = 0; z[1] = 0; z[2] = 0; z[3] = 0;
  return z;
}

// four consecutive elements (16- or 32-byte aligned)
__device__ __forceinline__ void load4(const double *p, double (&o)[4]) {
  const d4 v = *reinterpret_cast<const d4 *>(p);
  o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
__device__ __forceinline__ void load4(const float *p, double (&o)[4]) {
  const f4 v = *reinterpret_cast<const f4 *>(p);
  o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
}
// the first NL of four consecutive floats (16-byte aligned); the rest are zero
template <int NL>
__device__ __forceinline__ void loadn(const float *p, float (&o)[4]) {
  typedef float f2 __attribute__((ext_vector_type(2)));
  typedef float f3 __attribute__((ext_vector_type(3)));
  o[0] = o[1] = o[2] = o[3] = 0.f;
  if constexpr (NL == 1) {
    o[0] = *p;
  } else if constexpr (NL == 2) {
    const f2 v = *reinterpret_cast<const f2 *>(p);
    o[0] = v[0]; o[1] = v[1];
  } else if constexpr (NL == 3) {
    const f3 v = *reinterpret_cast<const f3 *>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2];
  } else {
    const f4 v = *reinterpret_cast<const f4 *>(p);
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
  }
}

__device__ __forceinline__ long long sym_start(long long i, long long N) { return i * N - i * (i - 1) / 2; }

// a global-memory pointer the caller knows to be the same in every lane,
// moved to scalar registers (loads then take a scalar base and a 32-bit lane
// offset)
template <typename P>
__device__ __forceinline__ const __attribute__((address_space(1))) P *wave_uniform(const P *p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (const __attribute__((address_space(1))) P *)(((unsigned long long)hi << 32) | lo);
}

// Workgroups are handed to the eight XCDs round-robin (block b runs on XCD
// b mod 8), and each XCD has its own L2.  This bijection renumbers the grid
// so that each XCD receives one contiguous range of logical block indices:
// the workgroups of one pair (its beta' tiles and gamma' splits, which all
// read the pair's core tensor G) then share an L2.
__device__ __forceinline__ int xcd_order(int b, int nb) {
  const int x = b & 7, slot = b >> 3, q = nb >> 3, rem = nb & 7;
  return x * q + min(x, rem) + slot;
}

__device__ __forceinline__ void pair_ij(const PairMap &pm, long long pg, int &i, int &j) {
  if (!pm.symmetric) {
    i = pm.i0 + (int)(pg / pm.N);
    j = (int)(pg % pm.N);
    return;
  }
  const double Nd = (double)pm.N;
  const double b = 2.0 * Nd + 1.0;
  long long ii = (long long)floor((b - sqrt(b * b - 8.0 * (double)pg)) * 0.5);
  if (ii < 0) ii = 0;
  if (ii > pm.N - 1) ii = pm.N - 1;
  while (ii > 0 && sym_start(ii, pm.N) > pg) --ii;
  while (ii + 1 < pm.N && sym_start(ii + 1, pm.N) <= pg) ++ii;
  i = (int)ii;
  j = (int)(ii + (pg - sym_start(ii, pm.N)));
}

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
  pair_ij(pm, pm.p0 + p, i, j);
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
// tiles of every mode), so no per-MFMA guard; the psi loads use clamped
// addresses and a select instead of a branch.
template <typename T, typename Tin, int MT, bool LDS_TAB>
__global__ __launch_bounds__(256) void k_proj12m(const Tin *__restrict__ psi, Dims D, PairMap pm, int P,
                                                 Tables<T> tb, T *__restrict__ T2) {
  using M = MF<T>;
  using acc = typename M::acc;
  constexpr int RP = 16 * MT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int nbt = D.nb1 >> 4, nct = D.nc2 >> 4;
  const T *V2 = tb.V2B, *V1c = tb.V1chain;
  if constexpr (LDS_TAB) {
    T *s2 = reinterpret_cast<T *>(smem_raw);
    T *s1 = s2 + (size_t)D.nc2 * RP;
    const int m2 = D.nc2 * RP, m1 = MT * nbt * 256;
    for (int idx = threadIdx.x; idx < m2; idx += 256) s2[idx] = tb.V2B[idx];
    for (int idx = threadIdx.x; idx < m1; idx += 256) s1[idx] = tb.V1chain[idx];
    __syncthreads();
    V2 = s2;
    V1c = s1;
  }
  const size_t plane = (size_t)D.n1 * D.n2;
  const long long total = (long long)P * D.n0;
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
    const int a = (int)(item % D.n0);
    const int p = (int)(item / D.n0);
    int i, j;
    pair_ij(pm, pm.p0 + p, i, j);
    const Tin *pi = psi + ((size_t)i * D.n0 + a) * plane;
    const Tin *pj = psi + ((size_t)j * D.n0 + a) * plane;
    acc T2a[MT][MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
      for (int gt = 0; gt < MT; ++gt) T2a[mt][gt] = zero4<acc>();
    for (int mb = 0; mb < nbt; ++mb) {
      acc T1[MT];
#pragma unroll
      for (int gt = 0; gt < MT; ++gt) T1[gt] = zero4<acc>();
      const int b = 16 * mb + lr;
      const size_t rowoff = (size_t)min(b, D.n1 - 1) * D.n2;
      for (int J = 0; J < nct; ++J) {
        const int c = 16 * J + 4 * lg;
        const bool in = b < D.n1 && c < D.n2;
        const size_t off = rowoff + min(c, D.n2 - 4);
        double x[4], y[4];
        load4(pi + off, x);
        load4(pj + off, y);
#pragma unroll
        for (int q = 0; q < 4; ++q) x[q] = in ? x[q] * y[q] : 0.0;
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const T *vrow = V2 + (size_t)(c + jj) * RP + lr;
          const T rho = (T)x[jj];
#pragma unroll
          for (int gt = 0; gt < MT; ++gt) T1[gt] = M::mma(rho, vrow[16 * gt], T1[gt]);
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

// Epilogue shared by the core kernels: the pair-energy partial
// sum Phi[alpha'][gamma'][beta'] G[alpha'][beta'][gamma'] (FP64, fixed order)
// and the first back-projection S1[a][gamma'][beta'] = sum_alpha' U0[a][alpha'] Phi[alpha'][gamma'][beta'],
// chained on the Phi accumulators.
template <typename T, int MT, int NGW, int NW, bool WRITE_S1>
__device__ __forceinline__ void core_epilogue(typename MF<T>::acc (&Phi)[MT][NGW], const T *__restrict__ Gp, const Dims &D,
                                              int p, int bt, int gs, int NGS, int wg_lo, int wg_hi, int lane, int lr,
                                              int lg, int wave, const Tables<T> &tb, T *__restrict__ S1,
                                              double *__restrict__ epart) {
  using M = MF<T>;
  using acc = typename M::acc;
  constexpr int RP = 16 * MT;
  __shared__ double red[NW];
  double e = 0.0;
  const int bp = 16 * bt + lr;
#pragma unroll
  for (int ng = 0; ng < NGW; ++ng) {
    const int gp = wg_lo + ng;
    if (gp < wg_hi && bp < D.r1) {
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) {
        {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int ap = 16 * mt + drow<T>(lg, v);
            if (ap < D.r0) e += (double)Phi[mt][ng][v] * (double)Gp[((size_t)ap * RP + bp) * RP + gp];
          }
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if (lane == 0) red[wave] = e;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = (red[0] + red[1]) + (red[2] + red[3]);
    if constexpr (NW == 8) t += (red[4] + red[5]) + (red[6] + red[7]);
    epart[((size_t)p * MT + bt) * NGS + gs] = t;
  }

  // ---- S1[p][a][gamma'][beta'] = sum_alpha' U0[a][alpha'] Phi[alpha'][gamma'][beta']
  if (WRITE_S1) {
    const int nat = D.na0 >> 4;
    for (int ma = 0; ma < nat; ++ma) {
      T uf[MT][4];
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          uf[mt][v] = tb.U0chain[(((size_t)ma * MT + mt) * 4 + v) * 64 + lane];
#pragma unroll
      for (int ng = 0; ng < NGW; ++ng) {
        const int gp = wg_lo + ng;
        if (gp < wg_hi) {
          acc S = zero4<acc>();
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) {
            {
#pragma unroll
              for (int v = 0; v < 4; ++v) S = M::mma(uf[mt][v], Phi[mt][ng][v], S);
            }
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = 16 * ma + drow<T>(lg, v);
            if (a < D.n0) S1[(((size_t)p * D.n0 + a) * RP + gp) * RP + bp] = S[v];
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
}

// -------------------------------------------------------------------------------------
// core: per workgroup one pair p, one 16-wide tile bt of beta' and a range of
// gamma' (split gs of NGS).  A step pairs one input slab alpha with one group
// of NW Gaussian terms (wavefront w takes term k = NW*kq + w).  Slab-major
// order (slabs outer, term groups inner) or, where the term fragments fit in
// registers, term-major order (term groups outer, whole slabs streamed
// through LDS); per step:
//   phase A
//     W[gamma][beta']  = sum_beta G[alpha][beta][gamma] Chat1_k[beta'][beta]
//     Z[gamma'][beta'] = sum_gamma Chat2_k[gamma'][gamma] W[gamma][beta']   (chained)
//     Z -> LDS slot w
//   phase B (each wavefront: its own gamma' rows, all alpha')
//     Phi[alpha'][gamma'][beta'] += sum_{k in step} w_k Chat0_k[alpha'][alpha] Z_k[gamma'][beta']
// i.e. the term sum is folded into the reduction of the mode-0 product.  The
// term matrices are shared by every workgroup and come from L2; Z is
// double-buffered in LDS so each step needs one barrier; Phi stays in
// registers for the whole pair.
// Padding: in the last 16-row tile of beta and gamma only the first TL
// four-row chunks are live (TL = 4: all of them); the beta contraction of W
// runs over 4 (MT - 1) + TL K = 4 steps and the gamma contraction of Z skips
// the dead chunks.  A chunk is one accumulator entry v of W across the four
// lane groups;
// FP64 accumulators hold rows 4v + lg, i.e. contiguous chunks already, while
// the FP32 core permutes the slab's gamma rows inside each 16-row tile (row m
// of the A operand is gamma 4(m mod 4) + m / 4) so that its entry v holds
// gamma 4v + lg too.
// -------------------------------------------------------------------------------------
template <typename T, int MT, int NGW, int NW, bool WRITE_S1, int TL>
__global__ __launch_bounds__(64 * NW, 1) void k_core(const T *__restrict__ G, Dims D, int P, int NGS, Tables<T> tb,
                                                 T *__restrict__ S1, double *__restrict__ epart) {
  using M = MF<T>;
  using acc = typename M::acc;
  // the padded core size is the same for all three modes: rp = 16 * MT
  constexpr int RP = 16 * MT;
  constexpr size_t F = (size_t)RP * RP;
  extern __shared__ __align__(16) unsigned char smem_raw[];

  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int bid = xcd_order(blockIdx.x, gridDim.x);
  const int gs = bid % NGS;
  const int tt = bid / NGS;
  const int bt = tt % MT;
  const int p = tt / MT;
  if (p >= P) return;  // whole block leaves together

  const int gper = (D.r2 + NGS - 1) / NGS;
  const int g_lo = gs * gper;
  const int g_hi = min(D.r2, g_lo + gper);
  const int gw = (gper + NW - 1) / NW;            // gamma' rows per wavefront in phase B (<= NGW)
  const int wg_lo = g_lo + wave * gw;
  const int wg_hi = min(g_hi, wg_lo + gw);
  const int nrow = max(0, wg_hi - wg_lo);         // this wavefront's gamma' rows (uniform)
  const T *Gp = G + (size_t)p * RP * F;

  // Register plan per precision and rank tile:
  //   PF     Chat1 / Ahat fragments prefetched one step ahead
  //   C2S    Chat2 fragments loaded whole at the start of the step (else one
  //          gamma' tile at a time inside the Z chain)
  //   HOLD_G the slab's A fragments held in registers for all of its steps
  //          (FP64 at up to two tiles)
  //   LDS_G  the slab in LDS instead (double-buffered; every FP32 form),
  //          each row laid out so a lane reads its fragments with one load
  constexpr bool F32 = sizeof(T) == 4;
  constexpr bool PF = F32 || MT <= 2;
  constexpr bool C2S = F32 ? MT <= 3 : MT <= 2;
  constexpr bool HOLD_G = !F32 && C2S && (NW == 4 || MT <= 2);
  constexpr bool LDS_G = F32 && !HOLD_G;
  //   KM     term-major order (FP32 with Chat2 held): see below
  constexpr bool KM = F32 && LDS_G && C2S;
  // slab gamma row (inside its tile) that this lane feeds to the W chain
  const int lrg = F32 ? ((lr & 3) << 2 | (lr >> 2)) : lr;
  constexpr int NKT = 4 * (MT - 1) + TL;  // K = 4 steps of the beta contraction
  // LDS slab row beta: for each of the 16 lanes of a fragment its MT gamma
  // values (gamma = 16 mg + lane) side by side, padded to LPL, so a lane
  // reads all of its A fragments of one beta row with 16-byte loads
  constexpr int LPL = MT <= 4 ? 4 : 8;
  constexpr int SROW = 16 * LPL;
  constexpr int SLAB = LDS_G ? RP * SROW : 0;
  T *Gs = reinterpret_cast<T *>(smem_raw);        // [2][RP][16][LPL] (LDS_G)
  // Z slots: [2][NW][ZSS].  FP32: row gamma' of slot w at gamma' * ZRS, every
  // padded row has room, so stores need no range test; the 80-byte row
  // stride spreads a store's four lane groups (rows 4 apart) over the banks
  // and the slot stride does the same for phase B's four terms.  FP64 (the
  // faster form there): only the workgroup's gper rows, at (gamma' - g_lo) * 16
  constexpr int ZRS = F32 ? 20 : 16;
  const int ZSS = F32 ? RP * ZRS + 16 : gper * 16;
  T *Zs = Gs + 2 * SLAB;
  const int zsz = NW * ZSS;

  acc Phi[MT][NGW];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ng = 0; ng < NGW; ++ng) Phi[mt][ng] = zero4<acc>();

  // Loops run over the padded size; padded rows and columns of G and of the
  // term matrices are zero.
  constexpr int GK = HOLD_G ? 4 * MT : 1, GM = HOLD_G ? MT : 1;
  constexpr int NTG = NW / 4;  // groups of four terms per step
  const int nkq = (D.K + NW - 1) / NW;
  const int nsteps = D.r0 * nkq;

  // Operands of a step for this wavefront's term k: Chat1_k (16 beta'
  // columns) as B fragments and Ahat[alpha][4kq + lg] (the phase-B column
  // fragments) are prefetched one step ahead; Chat2_k (A fragments in chain
  // order) is loaded at the start of its own step and first used after the
  // W chain.  Loads are issued in the order they are waited for, so the
  // in-order wait counts never wait on a prefetch.
  struct CF {
    T cb[4 * MT];
    T af[NTG][MT];
  };
  // Chat1_k B fragments of every K = 4 step of the W chain (FP32: a lane's
  // four steps of one 16-row group with one load, the live ones only)
  auto load_c1 = [&](int k_, T (&cb)[4 * MT]) {
    if constexpr (F32) {
      const float *C1k = tb.C1f + ((size_t)k_ * MT + bt) * MT * 256 + lane * 4;
#pragma unroll
      for (int kq4 = 0; kq4 < MT; ++kq4) {
        float(&o)[4] = *reinterpret_cast<float(*)[4]>(&cb[4 * kq4]);
        if (kq4 < MT - 1) loadn<4>(C1k + kq4 * 256, o);
        else loadn<TL>(C1k + kq4 * 256, o);
      }
    } else {
      const T *C1k = tb.C1f + (size_t)k_ * F + 16 * bt + lr;
#pragma unroll
      for (int kt = 0; kt < 4 * MT; ++kt) cb[kt] = C1k[(4 * kt + lg) * RP];
    }
  };
  // Chat2_k A fragments [v] of gamma' tile mtp and gamma tile mg
  auto load_c2 = [&](int k_, int mtp, int mg, T (&o)[4]) {
    if constexpr (F32) {
      const float *p_ = tb.C2chain + ((size_t)k_ * MT * MT + mtp * MT + mg) * 256 + lane * 4;
      if (mg < MT - 1) loadn<4>(p_, o);
      else loadn<TL>(p_, o);
    } else {
      const T *p_ = tb.C2chain + ((size_t)k_ * MT * MT + mtp * MT + mg) * 256 + lane;
#pragma unroll
      for (int v = 0; v < 4; ++v) o[v] = p_[v * 64];
    }
  };
  auto load_terms = [&](int alpha_, int kq_, CF &f) {
#pragma unroll
    for (int tg = 0; tg < NTG; ++tg) {
      const T *ah = tb.Ahat + ((size_t)alpha_ * D.Kp + NW * kq_ + 4 * tg + lg) * RP + lr;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) f.af[tg][mt] = ah[16 * mt];
    }
    const int k_ = NW * kq_ + wave;
    if (k_ >= D.K) return;
    load_c1(k_, f.cb);
  };
  // A fragments of slab alpha: G[alpha][beta = 4kt+lg][gamma = 16mg+lr]
  auto load_slab = [&](int alpha_, T (&g)[GK][GM]) {
    const T *Ga_ = Gp + (size_t)alpha_ * F + lrg;
#pragma unroll
    for (int kt = 0; kt < GK; ++kt)
#pragma unroll
      for (int mg = 0; mg < GM; ++mg) g[kt][mg] = Ga_[(4 * kt + lg) * RP + 16 * mg];
  };

  CF ca, cb2;
  T gf[GK][GM];  // held slab fragments
  if constexpr (PF && !KM) load_terms(0, 0, ca);
  const T *Ga = Gp + lrg;
  // LDS slab: the next slab arrives in (about) four chunks of EPT elements
  // per thread, chunk kq during step kq (loaded at the start of the step,
  // stored before the step's barrier); the loads are unconditional (clamped
  // addresses) so every step issues the same loads
  constexpr int CHT = 64 * NW;
  constexpr int EPT = LDS_G ? (int)((F + 4 * CHT - 1) / (4 * CHT)) : 1;
  constexpr int CH = EPT * CHT;
  constexpr int NCH = LDS_G ? (int)((F + CH - 1) / CH) : 0;
  const int tid = threadIdx.x;
  auto slab_load = [&](int c, int a_, T (&v)[EPT]) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) v[j] = Gp[(size_t)a_ * F + min(c * CH + j * CHT + tid, (int)F - 1)];
  };
  auto slab_store = [&](int c, int buf, const T (&v)[EPT]) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = c * CH + j * CHT + tid;
      if (e < (int)F) {
        const int gamma = e % RP;
        const int gl16 = gamma & 15, ln = (gl16 & 3) << 2 | (gl16 >> 2);  // lane that reads it
        Gs[buf * SLAB + (e / RP) * SROW + ln * LPL + (gamma >> 4)] = v[j];
      }
    }
  };
  if constexpr (LDS_G) {
    for (int c = 0; c < NCH; ++c) {
      T v[EPT];
      slab_load(c, 0, v);
      slab_store(c, 0, v);
    }
    __syncthreads();
  }
  if constexpr (KM) {
    // Term-major order: the outer loop walks the groups of NW terms, the
    // inner loop the slabs alpha.  Each wavefront holds its term's Chat1 and
    // Chat2 fragments in registers for all r0 slabs, and one whole slab
    // streams through the LDS double buffer per step, so the term tables are
    // read once per term group instead of once per (slab, term group).  The
    // sums are the same as in slab-major order (phase B adds the same
    // products to the same Phi accumulators, in another order).
    // the next slab in 16-byte pieces (RP is a multiple of 16, so a piece
    // stays inside one beta row): EPS pieces per thread and step
    constexpr int F4 = (int)(F / 4);
    constexpr int EPS = (F4 + CHT - 1) / CHT;
    typedef T AF[NTG][MT];
    auto load_af = [&](int alpha_, int kq_, AF &af) {
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg) {
        const T *ah = tb.Ahat + ((size_t)alpha_ * D.Kp + NW * kq_ + 4 * tg + lg) * RP + lr;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[tg][mt] = ah[16 * mt];
      }
    };
    auto kslab_load = [&](int a_, float4 (&v)[EPS]) {
      const float4 *src = reinterpret_cast<const float4 *>(Gp + (size_t)a_ * F);
#pragma unroll
      for (int j = 0; j < EPS; ++j) v[j] = src[min(j * CHT + tid, F4 - 1)];
    };
    auto kslab_store = [&](int buf, const float4 (&v)[EPS]) {
#pragma unroll
      for (int j = 0; j < EPS; ++j) {
        const int e4 = j * CHT + tid;
        if (e4 < F4) {
          const int beta = (4 * e4) / RP, g0 = (4 * e4) % RP;
          const float x[4] = {v[j].x, v[j].y, v[j].z, v[j].w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int gamma = g0 + q;
            const int gl16 = gamma & 15, ln = (gl16 & 3) << 2 | (gl16 >> 2);
            Gs[buf * SLAB + beta * SROW + ln * LPL + (gamma >> 4)] = x[q];
          }
        }
      }
    };
    T tcb[4 * MT];
    T c2s[MT][MT][4];
    AF afa, afb;
    load_af(0, 0, afa);
    auto kstep = [&](const int kq, const int alpha, const int step, AF &cur, AF &nxt) __attribute__((always_inline)) {
      const int k = NW * kq + wave;
      // the next step's slab (alpha + 1, or alpha 0 of the next term group)
      // and phase-B columns, issued before this step's work
      const bool last_a = alpha + 1 == D.r0;
      const bool more = !last_a || kq + 1 < nkq;  // uniform
      float4 gnext[EPS];
      kslab_load(last_a ? 0 : alpha + 1, gnext);
      if (more) load_af(last_a ? 0 : alpha + 1, last_a ? kq + 1 : kq, nxt);
      T *Zw = Zs + (size_t)(step & 1) * zsz + (size_t)wave * ZSS;
      if (k < D.K) {
        acc W[MT];
#pragma unroll
        for (int mg = 0; mg < MT; ++mg) W[mg] = zero4<acc>();
#pragma unroll
        for (int kt = 0; kt < 4 * MT; ++kt) {
          if (kt >= NKT) break;
          const float4 f =
              *reinterpret_cast<const float4 *>(Gs + (step & 1) * SLAB + (4 * kt + lg) * SROW + lr * LPL);
          const T gl[4] = {f.x, f.y, f.z, f.w};
#pragma unroll
          for (int mg = 0; mg < MT; ++mg) W[mg] = M::mma(gl[mg], tcb[kt], W[mg]);
        }
        acc Z[MT];
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp) Z[mtp] = zero4<acc>();
#pragma unroll
        for (int mg = 0; mg < MT; ++mg)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (mg == MT - 1 && v >= TL) break;
#pragma unroll
            for (int mtp = 0; mtp < MT; ++mtp) Z[mtp] = M::mma(c2s[mtp][mg][v], W[mg][v], Z[mtp]);
          }
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp)
#pragma unroll
          for (int v = 0; v < 4; ++v) Zw[(16 * mtp + drow<T>(lg, v)) * ZRS + lr] = Z[mtp][v];
      } else {
        for (int idx = lane; idx < (g_hi - g_lo) * 16; idx += 64) Zw[(g_lo + (idx >> 4)) * ZRS + (idx & 15)] = (T)0;
      }
      if (more) kslab_store((step + 1) & 1, gnext);
      __syncthreads();
      const T *zb = Zs + (size_t)(step & 1) * zsz + lr;
      T bz[NTG][NGW];
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
        for (int ng = 0; ng < NGW; ++ng) bz[tg][ng] = zb[(4 * tg + lg) * ZSS + min(wg_lo + ng, RP - 1) * ZRS];
#pragma unroll
      for (int ng = 0; ng < NGW; ++ng) {
        if (NW == 8 && ng >= gw) break;
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(cur[tg][mt], bz[tg][ng], Phi[mt][ng]);
      }
    };
    int step = 0;
    for (int kq = 0; kq < nkq; ++kq) {
      const int k = NW * kq + wave;
      if (k < D.K) {
        load_c1(k, tcb);
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp)
#pragma unroll
          for (int mg = 0; mg < MT; ++mg) load_c2(k, mtp, mg, c2s[mtp][mg]);
      }
      int alpha = 0;
      for (; alpha + 1 < D.r0; alpha += 2, step += 2) {
        kstep(kq, alpha, step, afa, afb);
        kstep(kq, alpha + 1, step + 1, afb, afa);
      }
      if (alpha < D.r0) {  // odd r0: the tail step leaves the next columns in afb
        kstep(kq, alpha, step, afa, afb);
        ++step;
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) afa[tg][mt] = afb[tg][mt];
      }
    }
  } else {
  // one step: uses cur, prefetches the next step's operands into nxt
  auto step_body = [&](const int step, CF &cur, CF &nxt) __attribute__((always_inline)) {
    const int alpha = step / nkq;
    const int kq = step - alpha * nkq;
    const int k = NW * kq + wave;
    if (kq == 0) {
      Ga = Gp + (size_t)alpha * F + lrg;
      if constexpr (HOLD_G) {
        load_slab(alpha, gf);
        // settle the slab (and this step's prefetched terms) here, once per
        // slab: later steps then wait only on their own operands, never on
        // the prefetch they issue
        if constexpr (PF) __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
      }
    }
    T gnext[EPT];
    if constexpr (LDS_G) slab_load(min(kq, NCH - 1), min(alpha + 1, D.r0 - 1), gnext);
    T c2s[C2S ? MT : 1][C2S ? MT : 1][4];
    if constexpr (C2S) {
      if (k < D.K) {
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp)
#pragma unroll
          for (int mg = 0; mg < MT; ++mg) load_c2(k, mtp, mg, c2s[mtp][mg]);
      }
    }
    if constexpr (PF) {
      const bool wrap = kq + 1 == nkq;
      if (step + 1 < nsteps) load_terms(wrap ? alpha + 1 : alpha, wrap ? 0 : kq + 1, nxt);
    }
    if constexpr (!PF) {
      if (k < D.K) load_c1(k, cur.cb);
    }
    T *Zw = Zs + (size_t)(step & 1) * zsz + (size_t)wave * ZSS;
    // ---- phase A
    if (k < D.K) {
      acc W[MT];
#pragma unroll
      for (int mg = 0; mg < MT; ++mg) W[mg] = zero4<acc>();
#pragma unroll
      for (int kt = 0; kt < 4 * MT; ++kt) {
        if (kt >= NKT) break;
        T gl[LDS_G ? LPL : 1];
        if constexpr (LDS_G) {
          const float4 *src =
              reinterpret_cast<const float4 *>(Gs + (alpha & 1) * SLAB + (4 * kt + lg) * SROW + lr * LPL);
#pragma unroll
          for (int q = 0; q < LPL / 4; ++q) {
            const float4 f = src[q];
            gl[4 * q] = f.x;
            gl[4 * q + 1] = f.y;
            gl[4 * q + 2] = f.z;
            gl[4 * q + 3] = f.w;
          }
        }
#pragma unroll
        for (int mg = 0; mg < MT; ++mg) {
          T g;
          if constexpr (HOLD_G) g = gf[kt][mg];
          else if constexpr (LDS_G) g = gl[mg];
          else g = Ga[(4 * kt + lg) * RP + 16 * mg];
          W[mg] = M::mma(g, cur.cb[kt], W[mg]);
        }
      }
      // With Chat2 loaded whole (small ranks, FP32) the tiles' chains are
      // interleaved (short MFMA latency, cheap accumulators); otherwise one
      // tile at a time, skipping tiles outside this workgroup's gamma' rows
      // and loading each tile's Chat2 fragments in turn (keeps registers
      // for Phi).  Rows outside the range are stored and never read.
      auto store_z = [&](int mtp, const acc &Zt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gp = 16 * mtp + drow<T>(lg, v);
          if constexpr (F32) Zw[gp * ZRS + lr] = Zt[v];
          else if (gp >= g_lo && gp < g_hi) Zw[(gp - g_lo) * 16 + lr] = Zt[v];
        }
      };
      if constexpr (F32 && C2S) {
        acc Z[MT];
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp) Z[mtp] = zero4<acc>();
#pragma unroll
        for (int mg = 0; mg < MT; ++mg)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (mg == MT - 1 && v >= TL) break;
#pragma unroll
            for (int mtp = 0; mtp < MT; ++mtp) Z[mtp] = M::mma(c2s[mtp][mg][v], W[mg][v], Z[mtp]);
          }
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp) store_z(mtp, Z[mtp]);
      } else {
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp) {
          // only the gamma' tiles that meet this workgroup's rows (uniform);
          // at five FP32 tiles the branch costs registers (spills) and more
          // time than the skipped tiles save
          if constexpr (!(F32 && MT == 5))
            if (16 * mtp >= g_hi || 16 * mtp + 16 <= g_lo) continue;
          T c2[MT][4];
          if constexpr (C2S) {
#pragma unroll
            for (int mg = 0; mg < MT; ++mg)
#pragma unroll
              for (int v = 0; v < 4; ++v) c2[mg][v] = c2s[mtp][mg][v];
          } else {
#pragma unroll
            for (int mg = 0; mg < MT; ++mg) load_c2(k, mtp, mg, c2[mg]);
          }
          acc Z = zero4<acc>();
#pragma unroll
          for (int mg = 0; mg < MT; ++mg)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              if (mg == MT - 1 && v >= TL) break;
              Z = M::mma(c2[mg][v], W[mg][v], Z);
            }
          store_z(mtp, Z);
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    } else {
      if constexpr (F32)
        for (int idx = lane; idx < (g_hi - g_lo) * 16; idx += 64) Zw[(g_lo + (idx >> 4)) * ZRS + (idx & 15)] = (T)0;
      else
        for (int idx = lane; idx < gper * 16; idx += 64) Zw[idx] = (T)0;
    }
    if constexpr (LDS_G) {
      if (alpha + 1 < D.r0) {
        if (kq < NCH) slab_store(kq, (alpha + 1) & 1, gnext);
        if (kq + 1 == nkq)  // fewer steps than chunks: the rest now
          for (int c = nkq; c < NCH; ++c) {
            T v[EPT];
            slab_load(c, alpha + 1, v);
            slab_store(c, (alpha + 1) & 1, v);
          }
      }
    }
    __syncthreads();
    // ---- phase B: reduction over the step's terms, four at a time (slot lg
    // of group tg); rows past this wavefront's range read a valid LDS row
    // and are never stored, and with eight wavefronts a uniform bound skips
    // the spare rows' MFMAs
    const T *zb = Zs + (size_t)(step & 1) * zsz + lr;
    if constexpr (F32) {
      // all Z rows read before the first MFMA
      T bz[NTG][NGW];
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
        for (int ng = 0; ng < NGW; ++ng) bz[tg][ng] = zb[(4 * tg + lg) * ZSS + min(wg_lo + ng, RP - 1) * ZRS];
#pragma unroll
      for (int ng = 0; ng < NGW; ++ng) {
        if (NW == 8 && ng >= gw) break;
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(cur.af[tg][mt], bz[tg][ng], Phi[mt][ng]);
      }
    } else {
      // FP64 (four wavefronts, up to ten rows): each row's read next to its
      // MFMAs keeps the register file for the Phi accumulators
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg) {
        T af[MT];
        if constexpr (PF) {
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) af[mt] = cur.af[tg][mt];
        } else {
          const T *ah = tb.Ahat + ((size_t)alpha * D.Kp + NW * kq + 4 * tg + lg) * RP + lr;
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) af[mt] = ah[16 * mt];
        }
        const T *zrow = zb + (size_t)(4 * tg + lg) * ZSS;
#pragma unroll
        for (int ng = 0; ng < NGW; ++ng) {
          if (NW == 8 && ng >= gw) break;
          const T bz = zrow[min(wg_lo - g_lo + ng, gper - 1) * 16];
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(af[mt], bz, Phi[mt][ng]);
        }
      }
    }
  };
  // two steps per iteration with the operand buffers swapping roles, so the
  // prefetched registers are never copied (a copy would wait for the loads)
  int step = 0;
  if constexpr (PF) {
    for (; step + 1 < nsteps; step += 2) {
      step_body(step, ca, cb2);
      step_body(step + 1, cb2, ca);
    }
  }
  for (; step < nsteps; ++step) step_body(step, ca, cb2);
  }

  core_epilogue<T, MT, NGW, NW, WRITE_S1>(Phi, Gp, D, p, bt, gs, NGS, wg_lo, wg_hi, lane, lr, lg, wave, tb, S1,
                                          epart);
}

// -------------------------------------------------------------------------------------
// split-bf16 helpers: every operand x of the two chained contractions of
// phase A is taken as p0 + p1 (+ p2) in bf16 and a product keeps the terms
// p_i q_j with i + j < NS (bf16 MFMA 16x16x32, FP32 accumulation)
// -------------------------------------------------------------------------------------
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

template <int NS>
__device__ __forceinline__ void split8(const float (&x)[8], bf8 (&o)[NS]) {
  float r[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) r[i] = x[i];
#pragma unroll
  for (int sp = 0; sp < NS; ++sp) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const __bf16 h = (__bf16)r[i];
      o[sp][i] = h;
      if (sp + 1 < NS) r[i] -= (float)h;
    }
  }
}

template <int NS>
__device__ __forceinline__ f4 mma_split(const bf8 (&a)[NS], const bf8 (&b)[NS], f4 c) {
#pragma unroll
  for (int i = 0; i < NS; ++i)
#pragma unroll
    for (int j = 0; j < NS - i; ++j) c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], c, 0, 0, 0);
  return c;
}

__device__ __forceinline__ bf8 ld_bf8(const unsigned short *p) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 v = *reinterpret_cast<const u4 *>(p);
  bf8 r;
  __builtin_memcpy(&r, &v, 16);
  return r;
}


// -------------------------------------------------------------------------------------
// core, split-bf16 form with the slab in LDS: the same loop as k_core<float>
// (NW wavefronts, one term each per step, Z double-buffered in LDS, phase B
// in FP32 MFMA), with the two chained contractions of phase A on bf16 MFMA
// 16x16x32 over split operands.  The slab is split once per slab by the
// workgroup while it arrives (chunked over the steps) and kept in LDS as
// bf16 A fragments [part][gamma tile][beta chunk][lane][8]; each step reads
// its fragments with 16-byte LDS loads.  Chat1 fragments and the phase-B
// Ahat columns of the next step are prefetched.
// -------------------------------------------------------------------------------------
template <int MT, int NGW, int NS, int NW, bool WRITE_S1>
__global__ __launch_bounds__(64 * NW, 1) void k_core_bf2(const float *__restrict__ G, Dims D, int P, int NGS,
                                                         Tables<float> tb, BfTables bft, float *__restrict__ S1,
                                                         double *__restrict__ epart) {
  using M = MF<float>;
  using acc = f4;
  constexpr int RP = 16 * MT;
  constexpr size_t F = (size_t)RP * RP;
  constexpr int NC = (RP + 31) / 32;              // K = 32 chunks of the core size
  constexpr int FRAG = NS * MT * NC * 64 * 8;      // bf16 values of one split slab
  extern __shared__ __align__(16) unsigned char smem_raw[];

  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int bid = xcd_order(blockIdx.x, gridDim.x);
  const int gs = bid % NGS;
  const int tt = bid / NGS;
  const int bt = tt % MT;
  const int p = tt / MT;
  if (p >= P) return;

  const int gper = (D.r2 + NGS - 1) / NGS;
  const int g_lo = gs * gper;
  const int g_hi = min(D.r2, g_lo + gper);
  const int gw = (gper + NW - 1) / NW;
  const int wg_lo = g_lo + wave * gw;
  const int wg_hi = min(g_hi, wg_lo + gw);
  const float *Gp = G + (size_t)p * RP * F;
  unsigned short *Gs = reinterpret_cast<unsigned short *>(smem_raw);   // [2][FRAG]
  // Z slots with room for every padded row (as in k_core<float>)
  constexpr int ZRS = 20, ZSS = RP * ZRS + 16;
  float *Zs = reinterpret_cast<float *>(smem_raw + 2 * FRAG * sizeof(unsigned short));
  constexpr int zsz = NW * ZSS;
  constexpr int NTG = NW / 4;
  const int nkq = (D.K + NW - 1) / NW;
  const int nsteps = D.r0 * nkq;

  acc Phi[MT][NGW];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int ng = 0; ng < NGW; ++ng) Phi[mt][ng] = zero4<acc>();

  // slab chunks: EPT elements per thread, about four chunks per slab
  constexpr int CHT = 64 * NW;
  constexpr int EPT = (int)((F + 4 * CHT - 1) / (4 * CHT));
  constexpr int CH = EPT * CHT;
  constexpr int NCH = (int)((F + CH - 1) / CH);
  const int tid = threadIdx.x;
  auto slab_load = [&](int c, int a_, float (&v)[EPT]) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) v[j] = Gp[(size_t)a_ * F + min(c * CH + j * CHT + tid, (int)F - 1)];
  };
  // element (beta, gamma) -> split parts at A fragment (gamma tile, beta chunk, lane, i)
  auto slab_store = [&](int c, int buf, const float (&v)[EPT]) {
#pragma unroll
    for (int j = 0; j < EPT; ++j) {
      const int e = c * CH + j * CHT + tid;
      if (e < (int)F) {
        const int beta = e / RP, gamma = e % RP;
        const int ln = ((beta >> 3) & 3) * 16 + (gamma & 15);
        const int base = ((((gamma >> 4) * NC + (beta >> 5)) * 64 + ln) * 8) + (beta & 7);
        float r = v[j];
#pragma unroll
        for (int sp = 0; sp < NS; ++sp) {
          const __bf16 h = (__bf16)r;
          Gs[buf * FRAG + sp * (MT * NC * 512) + base] = __builtin_bit_cast(unsigned short, h);
          if (sp + 1 < NS) r -= (float)h;
        }
      }
    }
  };
  // zero both buffers (beta rows past RP inside the last chunk stay zero),
  // then slab 0
  for (int idx = tid; idx < FRAG; idx += CHT) {
    Gs[idx] = 0;
    Gs[FRAG + idx] = 0;
  }
  __syncthreads();
  for (int c = 0; c < NCH; ++c) {
    float v[EPT];
    slab_load(c, 0, v);
    slab_store(c, 0, v);
  }
  __syncthreads();

  struct CF {
    bf8 cb[NC][NS];
    float af[NTG][MT];
  };
  auto load_terms = [&](int alpha_, int kq_, CF &f) {
#pragma unroll
    for (int tg = 0; tg < NTG; ++tg) {
      const float *ah = tb.Ahat + ((size_t)alpha_ * D.Kp + NW * kq_ + 4 * tg + lg) * RP + lr;
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) f.af[tg][mt] = ah[16 * mt];
    }
    const int k_ = NW * kq_ + wave;
    if (k_ >= D.K) return;
    const unsigned short *c1 = bft.C1 + (((size_t)k_ * MT + bt) * 3) * NC * 512 + lane * 8;
#pragma unroll
    for (int sp = 0; sp < NS; ++sp)
#pragma unroll
      for (int c = 0; c < NC; ++c) f.cb[c][sp] = ld_bf8(c1 + ((size_t)sp * NC + c) * 512);
  };

  // eight wavefronts (two-part splits): term-major order as in the FP32 core,
  // the term's split Chat1/Chat2 fragments held for all slabs
  constexpr bool KM = NW == 8;
  if constexpr (KM) {
    constexpr int EPS = (int)((F + CHT - 1) / CHT);  // slab elements per thread and step
    typedef float AF[NTG][MT];
    auto load_af = [&](int alpha_, int kq_, AF &af) {
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg) {
        const float *ah = tb.Ahat + ((size_t)alpha_ * D.Kp + NW * kq_ + 4 * tg + lg) * RP + lr;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[tg][mt] = ah[16 * mt];
      }
    };
    auto kslab_load = [&](int a_, float (&v)[EPS]) {
#pragma unroll
      for (int j = 0; j < EPS; ++j) v[j] = Gp[(size_t)a_ * F + min(j * CHT + tid, (int)F - 1)];
    };
    auto kslab_store = [&](int buf, const float (&v)[EPS]) {
#pragma unroll
      for (int j = 0; j < EPS; ++j) {
        const int e = j * CHT + tid;
        if (e < (int)F) {
          const int beta = e / RP, gamma = e % RP;
          const int ln = ((beta >> 3) & 3) * 16 + (gamma & 15);
          const int base = ((((gamma >> 4) * NC + (beta >> 5)) * 64 + ln) * 8) + (beta & 7);
          float r = v[j];
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) {
            const __bf16 h = (__bf16)r;
            Gs[buf * FRAG + sp * (MT * NC * 512) + base] = __builtin_bit_cast(unsigned short, h);
            if (sp + 1 < NS) r -= (float)h;
          }
        }
      }
    };
    bf8 hcb[NC][NS];
    bf8 hc2[MT][NC][NS];
    AF afa, afb;
    load_af(0, 0, afa);
    auto kstep = [&](const int kq, const int alpha, const int step, AF &cur, AF &nxt) __attribute__((always_inline)) {
      const int k = NW * kq + wave;
      const bool last_a = alpha + 1 == D.r0;
      const bool more = !last_a || kq + 1 < nkq;  // uniform
      float gnext[EPS];
      kslab_load(last_a ? 0 : alpha + 1, gnext);
      if (more) load_af(last_a ? 0 : alpha + 1, last_a ? kq + 1 : kq, nxt);
      float *Zw = Zs + (size_t)(step & 1) * zsz + (size_t)wave * ZSS;
      if (k < D.K) {
        const unsigned short *gl = Gs + (step & 1) * FRAG + lane * 8;
        acc W[MT];
#pragma unroll
        for (int mg = 0; mg < MT; ++mg) W[mg] = zero4<acc>();
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
          for (int mg = 0; mg < MT; ++mg) {
            bf8 g[NS];
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) g[sp] = ld_bf8(gl + ((sp * MT + mg) * NC + c) * 512);
            W[mg] = mma_split<NS>(g, hcb[c], W[mg]);
          }
        bf8 wsp[NC][NS];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          float x[8];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            x[i] = W[2 * c][i];
            x[4 + i] = (2 * c + 1 < MT) ? W[(2 * c + 1 < MT) ? 2 * c + 1 : 0][i] : 0.f;
          }
          split8<NS>(x, wsp[c]);
        }
#pragma unroll
        for (int mtp = 0; mtp < MT; ++mtp) {
          if (16 * mtp >= g_hi || 16 * mtp + 16 <= g_lo) continue;  // uniform: tile outside the split
          acc Z = zero4<acc>();
#pragma unroll
          for (int c = 0; c < NC; ++c) Z = mma_split<NS>(hc2[mtp][c], wsp[c], Z);
#pragma unroll
          for (int v = 0; v < 4; ++v) Zw[(16 * mtp + 4 * lg + v) * ZRS + lr] = Z[v];
        }
      } else {
        for (int idx = lane; idx < (g_hi - g_lo) * 16; idx += 64) Zw[(g_lo + (idx >> 4)) * ZRS + (idx & 15)] = 0.f;
      }
      if (more) kslab_store((step + 1) & 1, gnext);
      __syncthreads();
      const float *zb = Zs + (size_t)(step & 1) * zsz + lr;
      float bz[NTG][NGW];
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
        for (int ng = 0; ng < NGW; ++ng) bz[tg][ng] = zb[(4 * tg + lg) * ZSS + min(wg_lo + ng, RP - 1) * ZRS];
#pragma unroll
      for (int ng = 0; ng < NGW; ++ng) {
        if (ng >= gw) break;
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(cur[tg][mt], bz[tg][ng], Phi[mt][ng]);
      }
    };
    int step = 0;
    for (int kq = 0; kq < nkq; ++kq) {
      const int k = NW * kq + wave;
      if (k < D.K) {
        const unsigned short *c1 = bft.C1 + (((size_t)k * MT + bt) * 3) * NC * 512 + lane * 8;
        const unsigned short *c2 = bft.C2 + (size_t)k * 3 * MT * NC * 512 + lane * 8;
#pragma unroll
        for (int sp = 0; sp < NS; ++sp)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            hcb[c][sp] = ld_bf8(c1 + ((size_t)sp * NC + c) * 512);
#pragma unroll
            for (int mtp = 0; mtp < MT; ++mtp) hc2[mtp][c][sp] = ld_bf8(c2 + (((size_t)sp * MT + mtp) * NC + c) * 512);
          }
      }
      int alpha = 0;
      for (; alpha + 1 < D.r0; alpha += 2, step += 2) {
        kstep(kq, alpha, step, afa, afb);
        kstep(kq, alpha + 1, step + 1, afb, afa);
      }
      if (alpha < D.r0) {  // odd r0: the tail step leaves the next columns in afb
        kstep(kq, alpha, step, afa, afb);
        ++step;
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) afa[tg][mt] = afb[tg][mt];
      }
    }
  } else {
  CF ca, cb2;
  load_terms(0, 0, ca);
  auto step_body = [&](const int step, CF &cur, CF &nxt) __attribute__((always_inline)) {
    const int alpha = step / nkq;
    const int kq = step - alpha * nkq;
    const int k = NW * kq + wave;
    float gnext[EPT];
    slab_load(min(kq, NCH - 1), min(alpha + 1, D.r0 - 1), gnext);
    {
      const bool wrap = kq + 1 == nkq;
      if (step + 1 < nsteps) load_terms(wrap ? alpha + 1 : alpha, wrap ? 0 : kq + 1, nxt);
    }
    float *Zw = Zs + (size_t)(step & 1) * zsz + (size_t)wave * ZSS;
    if (k < D.K) {
      // ---- W[gamma][beta'] = sum_beta G[alpha][beta][gamma] Chat1_k[beta'][beta]
      const unsigned short *gl = Gs + (alpha & 1) * FRAG + lane * 8;
      acc W[MT];
#pragma unroll
      for (int mg = 0; mg < MT; ++mg) W[mg] = zero4<acc>();
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int mg = 0; mg < MT; ++mg) {
          bf8 g[NS];
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) g[sp] = ld_bf8(gl + ((sp * MT + mg) * NC + c) * 512);
          W[mg] = mma_split<NS>(g, cur.cb[c], W[mg]);
        }
      // ---- Z[gamma'][beta'] = sum_gamma Chat2_k[gamma'][gamma] W[gamma][beta'], two W tiles per K = 32
      bf8 wsp[NC][NS];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        float x[8];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x[i] = W[2 * c][i];
          x[4 + i] = (2 * c + 1 < MT) ? W[(2 * c + 1 < MT) ? 2 * c + 1 : 0][i] : 0.f;
        }
        split8<NS>(x, wsp[c]);
      }
      const unsigned short *c2 = bft.C2 + (size_t)k * 3 * MT * NC * 512 + lane * 8;
#pragma unroll
      for (int mtp = 0; mtp < MT; ++mtp) {
        if (16 * mtp >= g_hi || 16 * mtp + 16 <= g_lo) continue;  // uniform: tile outside the split
        acc Z = zero4<acc>();
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          bf8 a[NS];
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) a[sp] = ld_bf8(c2 + (((size_t)sp * MT + mtp) * NC + c) * 512);
          Z = mma_split<NS>(a, wsp[c], Z);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gp = 16 * mtp + 4 * lg + v;
          Zw[gp * ZRS + lr] = Z[v];
        }
      }
    } else {
      for (int idx = lane; idx < (g_hi - g_lo) * 16; idx += 64) Zw[(g_lo + (idx >> 4)) * ZRS + (idx & 15)] = 0.f;
    }
    // the next slab's chunk (split) before the barrier
    if (alpha + 1 < D.r0) {
      if (kq < NCH) slab_store(kq, (alpha + 1) & 1, gnext);
      if (kq + 1 == nkq)
        for (int c = nkq; c < NCH; ++c) {
          float v[EPT];
          slab_load(c, alpha + 1, v);
          slab_store(c, (alpha + 1) & 1, v);
        }
    }
    __syncthreads();
    // ---- phase B (FP32 MFMA): Phi += sum_{k in step} w_k Chat0_k[alpha'][alpha] Z_k,
    // all Z rows read before the first MFMA
    {
      const float *zb = Zs + (size_t)(step & 1) * zsz + lr;
      float bz[NTG][NGW];
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
        for (int ng = 0; ng < NGW; ++ng) bz[tg][ng] = zb[(4 * tg + lg) * ZSS + min(wg_lo + ng, RP - 1) * ZRS];
#pragma unroll
      for (int ng = 0; ng < NGW; ++ng) {
        if (NW == 8 && ng >= gw) break;
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg)
#pragma unroll
          for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(cur.af[tg][mt], bz[tg][ng], Phi[mt][ng]);
      }
    }
  };
  int step = 0;
  for (; step + 1 < nsteps; step += 2) {
    step_body(step, ca, cb2);
    step_body(step + 1, cb2, ca);
  }
  for (; step < nsteps; ++step) step_body(step, ca, cb2);
  }
  core_epilogue<float, MT, NGW, NW, WRITE_S1>(Phi, Gp, D, p, bt, gs, NGS, wg_lo, wg_hi, lane, lr, lg, wave, tb, S1,
                                              epart);
}


// -------------------------------------------------------------------------------------
// back: for target t, slab a and a group of NCG c-tiles, over all sources s:
//   X[beta][c]  = sum_gamma S1[p(t,s)][a][gamma][beta] U2[c][gamma]
//   phi[b][c]   = sum_beta U1[b][beta] X[beta][c]                      (chained)
//   acc[b][c]  += psi_s[a][b][c] phi[b][c]
// then Vx psi_t[a][b][c] = -scale * acc (times w(r) when weighted).  Two
// forms of the same sum:
//   k_back_s  streaming: runtime rank loops, loads next to their MFMA; small
//             register footprint, so many wavefronts per SIMD hide latency
//   k_back_b  batched: compile-time rank tiles, the source-independent U2
//             fragments hoisted out of the source loop, each source's S1
//             rows loaded in batches ahead of their MFMAs (clamped addresses
//             and selects instead of branches); fewer, busier wavefronts
// -------------------------------------------------------------------------------------
template <typename T, typename Tin, int NBT, int NCG, bool LDS_TAB>
__global__ __launch_bounds__(256) void k_back_s(const T *__restrict__ S1, const Tin *__restrict__ psi, Dims D,
                                              PairMap pm, int N, int t_begin, int t_count, Tables<T> tb,
                                              Tin *__restrict__ vx, const double *__restrict__ out_scale,
                                              int weighted, const double *__restrict__ q0,
                                              const double *__restrict__ q1, const double *__restrict__ q2) {
  using M = MF<T>;
  using acc = typename M::acc;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int nct = D.nc2 >> 4, nbt = D.nb1 >> 4;
  const int ncg = (nct + NCG - 1) / NCG;
  // shared operands (U2^T and the chained U1 fragments) staged once per workgroup
  const T *U2t = tb.U2T, *U1c = tb.U1chain;
  if constexpr (LDS_TAB) {
    T *s2 = reinterpret_cast<T *>(smem_raw);
    T *s1 = s2 + (size_t)D.rp2 * D.nc2;
    const int m2 = D.rp2 * D.nc2, m1 = nbt * D.MT1 * 256;
    for (int idx = threadIdx.x; idx < m2; idx += 256) s2[idx] = tb.U2T[idx];
    for (int idx = threadIdx.x; idx < m1; idx += 256) s1[idx] = tb.U1chain[idx];
    __syncthreads();
    U2t = s2;
    U1c = s1;
  }
  const long long total = (long long)t_count * D.n0 * ncg;
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
  const int cgi = (int)(item % ncg);
  const long long rest = item / ncg;
  const int a = (int)(rest % D.n0);
  const int t = t_begin + (int)(rest / D.n0);          // local target index
  const int tglob = pm.symmetric ? t : pm.i0 + t;      // orbital index of the target
  const int c0 = cgi * NCG;
  const size_t plane = (size_t)D.n1 * D.n2;
  const size_t S1pair = (size_t)D.n0 * D.rp2 * D.rp1;

  acc Acc[NBT][NCG];
#pragma unroll
  for (int mb = 0; mb < NBT; ++mb)
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) Acc[mb][cg] = zero4<acc>();

  for (int s = 0; s < N; ++s) {
    long long pg;
    if (pm.symmetric) {
      const int i = min(tglob, s), j = max(tglob, s);
      pg = sym_start(i, pm.N) + (j - i);
    } else {
      pg = (long long)t * pm.N + s;
    }
    const T *S = S1 + (size_t)(pg - pm.p0) * S1pair + (size_t)a * D.rp2 * D.rp1 + lr;
    acc X[MAX_MT][NCG];
#pragma unroll
    for (int mb = 0; mb < MAX_MT; ++mb)
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) X[mb][cg] = zero4<acc>();
    for (int kt = 0; kt < (D.r2k >> 2); ++kt) {
      const int gam = 4 * kt + lg;
      const bool gv = gam < D.r2;
      T bu[NCG];
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg)
        bu[cg] = (gv && c0 + cg < nct) ? U2t[(size_t)gam * D.nc2 + 16 * (c0 + cg) + lr] : (T)0;
      const T *srow = S + (size_t)gam * D.rp1;
#pragma unroll
      for (int mb = 0; mb < MAX_MT; ++mb) {
        if (mb < D.MT1) {
          const T af = gv ? srow[16 * mb] : (T)0;
#pragma unroll
          for (int cg = 0; cg < NCG; ++cg) X[mb][cg] = M::mma(af, bu[cg], X[mb][cg]);
        }
      }
    }
    const Tin *ps = psi + (size_t)s * D.n0 * plane + (size_t)a * plane;
#pragma unroll
    for (int mbb = 0; mbb < NBT; ++mbb) {
      if (mbb < nbt) {
        acc ph[NCG];
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) ph[cg] = zero4<acc>();
#pragma unroll
        for (int mbe = 0; mbe < MAX_MT; ++mbe) {
          if (mbe < D.MT1) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const T af = U1c[(((size_t)mbb * D.MT1 + mbe) * 4 + v) * 64 + lane];
#pragma unroll
              for (int cg = 0; cg < NCG; ++cg) ph[cg] = M::mma(af, X[mbe][cg][v], ph[cg]);
            }
          }
        }
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          const int c = 16 * (c0 + cg) + lr;
          if (c0 + cg < nct && c < D.n2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int b = 16 * mbb + drow<T>(lg, v);
              if (b < D.n1) Acc[mbb][cg][v] += (T)ps[(size_t)b * D.n2 + c] * ph[cg][v];
            }
          }
        }
      }
    }
  }
  const double scale = out_scale ? *out_scale : 1.0;
  Tin *out = vx + (size_t)t * D.n0 * plane + (size_t)a * plane;
#pragma unroll
  for (int mbb = 0; mbb < NBT; ++mbb) {
    if (mbb < nbt) {
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) {
        const int c = 16 * (c0 + cg) + lr;
        if (c0 + cg < nct && c < D.n2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int b = 16 * mbb + drow<T>(lg, v);
            if (b < D.n1) {
              double val = -scale * (double)Acc[mbb][cg][v];
              if (weighted) val *= q0[a] * q1[b] * q2[c];
              out[(size_t)b * D.n2 + c] = (Tin)val;
            }
          }
        }
      }
    }
  }
  }
}

template <typename T, typename Tin, typename Tps, int MT, int NBT, int NCG, bool LDS_TAB>
__global__ __launch_bounds__(256) void k_back_b(const T *__restrict__ S1, const Tps *__restrict__ psi, Dims D,
                                                PairMap pm, int N, int t_begin, int t_count, Tables<T> tb,
                                                Tin *__restrict__ vx, const double *__restrict__ out_scale,
                                                int weighted, const double *__restrict__ q0,
                                                const double *__restrict__ q1, const double *__restrict__ q2,
                                                int mb0) {
  using M = MF<T>;
  using acc = typename M::acc;
  constexpr int RP = 16 * MT;
  // S1 rows (gamma') per batch of loads: all of them while registers allow
  constexpr int KTB = sizeof(T) == 4 ? 2 : 4;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int nct = D.nc2 >> 4, nbt = D.nb1 >> 4;
  const int ncg = (nct + NCG - 1) / NCG;
  const int nkt = (D.r2 + 3) >> 2;  // gamma' rows in use, in fours
  // shared operands (U2^T and the chained U1 fragments), staged once per
  // workgroup in LDS when they fit (the choice is compile-time, so the
  // reads are LDS or global loads, never generic ones)
  T *s2 = reinterpret_cast<T *>(smem_raw);
  T *s1 = s2 + (size_t)RP * D.nc2;
  if constexpr (LDS_TAB) {
    const int m2 = RP * D.nc2, m1 = nbt * MT * 256;
    for (int idx = threadIdx.x; idx < m2; idx += 256) s2[idx] = tb.U2T[idx];
    for (int idx = threadIdx.x; idx < m1; idx += 256) s1[idx] = tb.U1chain[idx];
    __syncthreads();
  }
  const T *U2t = LDS_TAB ? s2 : tb.U2T;
  const T *U1c = LDS_TAB ? s1 : tb.U1chain;
  const size_t plane = (size_t)D.n1 * D.n2;
  const size_t S1pair = (size_t)D.n0 * RP * RP;
  const long long total = (long long)t_count * D.n0 * ncg;
  // per-lane offsets are 32-bit and unsigned, added to wave-uniform bases
  const unsigned soff = (unsigned)(lg * RP + lr);  // S1 fragment element of this lane
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
    const int cgi = (int)(item % ncg);
    const long long rest = item / ncg;
    const int a = (int)(rest % D.n0);
    const int t = t_begin + (int)(rest / D.n0);          // local target index
    const int tglob = pm.symmetric ? t : pm.i0 + t;      // orbital index of the target
    // c tiles of this wavefront (a phantom tile past the last one repeats it
    // and is never stored)
    int ct[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) ct[cg] = min(cgi * NCG + cg, nct - 1);
    // U2 fragments do not depend on the source: B[gamma'][c]
    T bu[4 * MT][NCG];
#pragma unroll
    for (int kt = 0; kt < 4 * MT; ++kt)
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) bu[kt][cg] = U2t[(unsigned)((4 * kt + lg) * D.nc2 + 16 * ct[cg] + lr)];
    // psi_j values of this wavefront's output points, clamped into the grid
    // (points past the edge are computed and never stored)
    unsigned poff[NBT][4];  // within one plane (n1 n2 < 2^31)
#pragma unroll
    for (int mbb = 0; mbb < NBT; ++mbb)
#pragma unroll
      for (int v = 0; v < 4; ++v) poff[mbb][v] = (unsigned)(min(16 * (mb0 + mbb) + drow<T>(lg, v), D.n1 - 1) * D.n2);
    unsigned pc[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) pc[cg] = (unsigned)min(16 * ct[cg] + lr, D.n2 - 1);

    acc Acc[NBT][NCG];
#pragma unroll
    for (int mb = 0; mb < NBT; ++mb)
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) Acc[mb][cg] = zero4<acc>();

    for (int s = 0; s < N; ++s) {
      long long pg;
      if (pm.symmetric) {
        const int i = min(tglob, s), j = max(tglob, s);
        pg = sym_start(i, pm.N) + (j - i);
      } else {
        pg = (long long)t * pm.N + s;
      }
      const auto *S = wave_uniform(S1 + (size_t)(pg - pm.p0) * S1pair + (size_t)a * RP * RP);
      const auto *ps = wave_uniform(psi + (size_t)s * D.n0 * plane + (size_t)a * plane);
      // the U1 fragments do not depend on the source, but holding all of
      // them across the source loop costs NBT * MT * 4 registers: an offset
      // made opaque per source by an empty asm makes them reload
      unsigned u1o = (unsigned)(mb0 * MT * 256 + lane);
      asm volatile("" : "+v"(u1o));
      // X[beta'][c] = sum_gamma' S1[gamma'][beta'] U2[c][gamma']
      acc X[MT][NCG];
#pragma unroll
      for (int mb = 0; mb < MT; ++mb)
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) X[mb][cg] = zero4<acc>();
#pragma unroll
      for (int kb = 0; kb < 4 * MT; kb += KTB) {
        if (kb >= nkt) break;  // uniform: padded gamma' rows only
        T sf[KTB][MT];
#pragma unroll
        for (int k = 0; k < KTB; ++k) {
          const int gam = 4 * (kb + k) + lg;
#pragma unroll
          for (int mb = 0; mb < MT; ++mb) {
            const T x = S[soff + (unsigned)(4 * (kb + k) * RP + 16 * mb)];
            sf[k][mb] = gam < D.r2 ? x : (T)0;  // rows past r2 are not written by the core kernel
          }
        }
#pragma unroll
        for (int k = 0; k < KTB; ++k)
#pragma unroll
          for (int mb = 0; mb < MT; ++mb)
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg) X[mb][cg] = M::mma(sf[k][mb], bu[kb + k][cg], X[mb][cg]);
      }
      // phi[b][c] = sum_beta' U1[b][beta'] X[beta'][c] (chained), then Acc += psi_j phi
#pragma unroll
      for (int mbb = 0; mbb < NBT; ++mbb) {
        if (mb0 + mbb >= nbt) break;  // uniform
        // one b tile at a time: keeps the U1 fragments and psi values of the
        // other tiles out of registers
        __builtin_amdgcn_sched_barrier(0);
        // psi_j at this b tile's points, loaded ahead of the chain that needs them
        Tps pv[NCG][4];
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
          for (int v = 0; v < 4; ++v) pv[cg][v] = ps[poff[mbb][v] + pc[cg]];
        acc ph[NCG];
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) ph[cg] = zero4<acc>();
#pragma unroll
        for (int mbe = 0; mbe < MT; ++mbe)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T af = U1c[u1o + (unsigned)(((mbb * MT + mbe) * 4 + v) * 64)];
#pragma unroll
            for (int cg = 0; cg < NCG; ++cg) ph[cg] = M::mma(af, X[mbe][cg][v], ph[cg]);
          }
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
          for (int v = 0; v < 4; ++v) Acc[mbb][cg][v] += (T)pv[cg][v] * ph[cg][v];
      }
    }
    const double scale = out_scale ? *out_scale : 1.0;
    Tin *out = vx + (size_t)t * D.n0 * plane + (size_t)a * plane;
#pragma unroll
    for (int mbb = 0; mbb < NBT; ++mbb) {
      if (mb0 + mbb >= nbt) break;
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) {
        const int c = 16 * (cgi * NCG + cg) + lr;
        if (cgi * NCG + cg < nct && c < D.n2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int b = 16 * (mb0 + mbb) + drow<T>(lg, v);
            if (b < D.n1) {
              double val = -scale * (double)Acc[mbb][cg][v];
              if (weighted) val *= q0[a] * q1[b] * q2[c];
              out[(size_t)b * D.n2 + c] = (Tin)val;
            }
          }
        }
      }
    }
  }
}

// -------------------------------------------------------------------------------------
// pair energies: e_pair[p0 + p] = sum of the core kernel's partials (fixed order)
// -------------------------------------------------------------------------------------
__global__ void k_epair(const double *__restrict__ epart, int P, int parts, long long p0, double *__restrict__ epair) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int q = 0; q < parts; ++q) s += epart[(size_t)p * parts + q];
  epair[p0 + p] = s;
}

// E_x = sum_p c_p e_pair[p]; c_p = -1/2 for ordered pairs (block mode) and
// for diagonal unique pairs, -1 for off-diagonal unique pairs.  One block,
// fixed summation order.
__global__ __launch_bounds__(256) void k_energy(const double *__restrict__ epair, long long np, int symmetric, int N,
                                                double *__restrict__ ex, double *__restrict__ e_out) {
  __shared__ double part[256];
  double s = 0.0;
  for (long long pg = threadIdx.x; pg < np; pg += 256) {
    const double e = epair[pg];
    if (e_out) e_out[pg] = e;
    double c = -0.5;
    if (symmetric) {
      // pair pg is diagonal when it is the first pair of its row
      const double Nd = (double)N;
      const double b = 2.0 * Nd + 1.0;
      long long ii = (long long)floor((b - sqrt(b * b - 8.0 * (double)pg)) * 0.5);
      if (ii < 0) ii = 0;
      if (ii > N - 1) ii = N - 1;
      while (ii > 0 && sym_start(ii, N) > pg) --ii;
      while (ii + 1 < N && sym_start(ii + 1, N) <= pg) ++ii;
      c = (sym_start(ii, N) == pg) ? -0.5 : -1.0;
    }
    s += c * e;
  }
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0 && ex) *ex = part[0];
}

// -------------------------------------------------------------------------------------
// host launchers
// -------------------------------------------------------------------------------------
namespace {

inline unsigned blocks_for(long long waves) { return (unsigned)((waves + 3) / 4); }

template <typename T, int MT, int NGW, int NW, int TL>
hipError_t launch_core_mt(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s) {
  const int gper = (a.D.r2 + a.NGS - 1) / a.NGS;
  if ((gper + NW - 1) / NW > NGW) return hipErrorInvalidValue;  // the plan gives every wavefront <= NGW rows
  constexpr int RP = 16 * MT;
  constexpr bool lds_g = sizeof(T) == 4;  // the slab-in-LDS forms of k_core (every FP32 one)
  constexpr size_t slab = lds_g ? (size_t)RP * 16 * (MT <= 4 ? 4 : 8) : 0;
  const size_t zslot = sizeof(T) == 4 ? (size_t)RP * 20 + 16 : (size_t)gper * 16;  // k_core's Z slot
  const size_t lds = (2 * slab + 2 * NW * zslot) * sizeof(T);
  const unsigned nb = (unsigned)((size_t)a.P * a.D.MT1 * a.NGS);
  if (lds > 64 * 1024) {  // opt in to more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per CU)
    const void *fn =
        want_vx ? (const void *)k_core<T, MT, NGW, NW, true, TL> : (const void *)k_core<T, MT, NGW, NW, false, TL>;
    const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  if (want_vx)
    hipLaunchKernelGGL((k_core<T, MT, NGW, NW, true, TL>), dim3(nb), dim3(64 * NW), lds, s, a.G, a.D, a.P, a.NGS, tb,
                       a.S1, a.epart);
  else
    hipLaunchKernelGGL((k_core<T, MT, NGW, NW, false, TL>), dim3(nb), dim3(64 * NW), lds, s, a.G, a.D, a.P, a.NGS, tb,
                       a.S1, a.epart);
  return hipGetLastError();
}

// register budget of the Phi accumulators: MT * NGW * 4 values per lane
constexpr int NGW64[MAX_MT + 1] = {0, 4, 8, 10, 8, 6};
constexpr int NGW32[MAX_MT + 1] = {0, 4, 8, 10, 12, 10};
// FP32 core at small ranks: eight wavefronts per workgroup (two per SIMD, so
// one hides the other's latencies), each with fewer Phi rows
constexpr int NW32[MAX_MT + 1] = {0, 8, 8, 8, 4, 4};
constexpr int NGW32x8[MAX_MT + 1] = {0, 2, 4, 6, 0, 0};

// FP32: one core per count of live chunks in the last tile of modes 1 and 2
template <int MT, int NGW, int NW>
hipError_t launch_core_f32_tl(const Tables<float> &tb, const ChunkArgs<float> &a, bool want_vx, hipStream_t s) {
  const int rt = max(a.D.r1, a.D.r2) - 16 * (MT - 1);
  switch (min(4, max(1, (rt + 3) / 4))) {
    case 1: return launch_core_mt<float, MT, NGW, NW, 1>(tb, a, want_vx, s);
    case 2: return launch_core_mt<float, MT, NGW, NW, 2>(tb, a, want_vx, s);
    case 3: return launch_core_mt<float, MT, NGW, NW, 3>(tb, a, want_vx, s);
    default: return launch_core_mt<float, MT, NGW, NW, 4>(tb, a, want_vx, s);
  }
}

template <typename T>
hipError_t launch_core(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s) {
  const int mt = max(a.D.MT0, max(a.D.MT1, a.D.MT2));
  if constexpr (sizeof(T) == 8) {
    switch (mt) {
      case 1: return launch_core_mt<T, 1, NGW64[1], 4, 4>(tb, a, want_vx, s);
      case 2: return launch_core_mt<T, 2, NGW64[2], 4, 4>(tb, a, want_vx, s);
      case 3: return launch_core_mt<T, 3, NGW64[3], 4, 4>(tb, a, want_vx, s);
      case 4: return launch_core_mt<T, 4, NGW64[4], 4, 4>(tb, a, want_vx, s);
      case 5: return launch_core_mt<T, 5, NGW64[5], 4, 4>(tb, a, want_vx, s);
    }
  } else {
    switch (mt) {
      case 1: return launch_core_f32_tl<1, NGW32x8[1], 8>(tb, a, want_vx, s);
      case 2: return launch_core_f32_tl<2, NGW32x8[2], 8>(tb, a, want_vx, s);
      case 3: return launch_core_f32_tl<3, NGW32x8[3], 8>(tb, a, want_vx, s);
      case 4: return launch_core_f32_tl<4, NGW32[4], 4>(tb, a, want_vx, s);
      case 5: return launch_core_f32_tl<5, NGW32[5], 4>(tb, a, want_vx, s);
    }
  }
  return hipErrorInvalidValue;
}

template <int MT, int NGW, int NS, int NW>
hipError_t launch_core_bf2_mt(const Tables<float> &tb, const BfTables &bft, const ChunkArgs<float> &a, bool want_vx,
                              hipStream_t s) {
  const int gper = (a.D.r2 + a.NGS - 1) / a.NGS;
  if ((gper + NW - 1) / NW > NGW) return hipErrorInvalidValue;
  constexpr int RP = 16 * MT, NC = (RP + 31) / 32;
  constexpr size_t frag = (size_t)NS * MT * NC * 512;
  const size_t lds = 2 * frag * sizeof(unsigned short) + (2 * NW * ((size_t)RP * 20 + 16)) * sizeof(float);
  const unsigned nb = (unsigned)((size_t)a.P * a.D.MT1 * a.NGS);
  if (lds > 64 * 1024) {
    const void *fn = want_vx ? (const void *)k_core_bf2<MT, NGW, NS, NW, true>
                             : (const void *)k_core_bf2<MT, NGW, NS, NW, false>;
    const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  if (want_vx)
    hipLaunchKernelGGL((k_core_bf2<MT, NGW, NS, NW, true>), dim3(nb), dim3(64 * NW), lds, s, (const float *)a.G, a.D,
                       a.P, a.NGS, tb, bft, a.S1, a.epart);
  else
    hipLaunchKernelGGL((k_core_bf2<MT, NGW, NS, NW, false>), dim3(nb), dim3(64 * NW), lds, s, (const float *)a.G,
                       a.D, a.P, a.NGS, tb, bft, a.S1, a.epart);
  return hipGetLastError();
}

template <int NS>
hipError_t launch_core_bf(const Tables<float> &tb, const BfTables &bft, const ChunkArgs<float> &a, bool want_vx,
                          hipStream_t s) {
  switch (a.D.MT0) {
    // two-part splits at small ranks: eight wavefronts; otherwise four
    case 1:
      if constexpr (NS == 2) return launch_core_bf2_mt<1, NGW32x8[1], NS, 8>(tb, bft, a, want_vx, s);
      else return launch_core_bf2_mt<1, NGW32[1], NS, 4>(tb, bft, a, want_vx, s);
    case 2:
      if constexpr (NS == 2) return launch_core_bf2_mt<2, NGW32x8[2], NS, 8>(tb, bft, a, want_vx, s);
      else return launch_core_bf2_mt<2, NGW32[2], NS, 4>(tb, bft, a, want_vx, s);
    case 3:
      if constexpr (NS == 2) return launch_core_bf2_mt<3, NGW32x8[3], NS, 8>(tb, bft, a, want_vx, s);
      else return launch_core_bf2_mt<3, NGW32[3], NS, 4>(tb, bft, a, want_vx, s);
    case 4: return launch_core_bf2_mt<4, NGW32[4], NS, 4>(tb, bft, a, want_vx, s);
    case 5: return launch_core_bf2_mt<5, NGW32[5], NS, 4>(tb, bft, a, want_vx, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename Tin, int NCG>
hipError_t launch_back_s_ncg(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  const int nct = a.D.nc2 >> 4, nbt = a.D.nb1 >> 4;
  const long long waves = (long long)a.t_count * a.D.n0 * ((nct + NCG - 1) / NCG);
  const unsigned nb = blocks_for(waves);
  const Tin *psi = (const Tin *)a.psi;
  Tin *vx = (Tin *)a.vx;
  // shared operands in LDS when they fit in 64 KiB; the grid is then capped
  // and each workgroup walks several items
  const size_t tab = ((size_t)a.D.rp2 * a.D.nc2 + (size_t)nbt * a.D.MT1 * 256) * sizeof(T);
  const bool lds_tab = tab <= 64 * 1024;
  const unsigned nbl = lds_tab ? std::min(nb, (unsigned)a.grid_cap) : nb;
#define TXE_BACK(NBTV)                                                                                         \
  if (lds_tab)                                                                                                   \
    hipLaunchKernelGGL((k_back_s<T, Tin, NBTV, NCG, true>), dim3(nbl), dim3(256), tab, s, a.S1, psi, a.D, a.pm,  \
                       a.N, a.t_begin, a.t_count, tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1],         \
                       a.qdev[2]);                                                                               \
  else                                                                                                           \
    hipLaunchKernelGGL((k_back_s<T, Tin, NBTV, NCG, false>), dim3(nb), dim3(256), 0, s, a.S1, psi, a.D, a.pm,    \
                       a.N, a.t_begin, a.t_count, tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1],         \
                       a.qdev[2])
  if (nbt <= 2) TXE_BACK(2);
  else if (nbt <= 4) TXE_BACK(4);
  else if (nbt <= 6) TXE_BACK(6);
  else if (nbt <= 8) TXE_BACK(8);
  else return hipErrorInvalidValue;
#undef TXE_BACK
  return hipGetLastError();
}

template <typename T, typename Tin, typename Tps, int MT, int NCG>
hipError_t launch_back_b_mt(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  const int nct = a.D.nc2 >> 4, nbt = a.D.nb1 >> 4;
  const long long waves = (long long)a.t_count * a.D.n0 * ((nct + NCG - 1) / NCG);
  const unsigned nb = blocks_for(waves);
  // psi_j as read: the orbitals, or their FP32 copy (the values the FP32
  // kernel rounds them to anyway)
  const Tps *psi = std::is_same<Tps, Tin>::value ? (const Tps *)a.psi : (const Tps *)a.psi32;
  Tin *vx = (Tin *)a.vx;
  // shared operands in LDS when they fit in 64 KiB; the grid is then capped
  // and each workgroup walks several items
  const size_t tab = ((size_t)16 * MT * a.D.nc2 + (size_t)nbt * MT * 256) * sizeof(T);
  const int lds_tab = tab <= 64 * 1024 ? 1 : 0;
  const unsigned nbl = lds_tab ? std::min(nb, (unsigned)a.grid_cap) : nb;
  const size_t lds = lds_tab ? tab : 0;
  // all b tiles in one launch up to six tiles (X computed once per source);
  // FP64 up to eight.  FP32 beyond six: launches over disjoint ranges of
  // four b tiles, each recomputing X for its sources (registers)
  if (nbt > 8) return hipErrorInvalidValue;
#define TXE_BACK(NBTV, MB0)                                                                                      \
  do {                                                                                                           \
    if (lds_tab)                                                                                                 \
      hipLaunchKernelGGL((k_back_b<T, Tin, Tps, MT, NBTV, NCG, true>), dim3(nbl), dim3(256), lds, s, a.S1, psi, a.D,  \
                         a.pm, a.N, a.t_begin, a.t_count, tb, vx, a.out_scale, a.weighted, a.qdev[0],           \
                         a.qdev[1], a.qdev[2], MB0);                                                             \
    else                                                                                                         \
      hipLaunchKernelGGL((k_back_b<T, Tin, Tps, MT, NBTV, NCG, false>), dim3(nbl), dim3(256), 0, s, a.S1, psi, a.D,   \
                         a.pm, a.N, a.t_begin, a.t_count, tb, vx, a.out_scale, a.weighted, a.qdev[0],           \
                         a.qdev[1], a.qdev[2], MB0);                                                             \
  } while (0)
  if (nbt <= 2) {
    TXE_BACK(2, 0);
  } else if (nbt <= 4) {
    TXE_BACK(4, 0);
  } else if (nbt <= 6) {
    TXE_BACK(6, 0);
  } else if constexpr (sizeof(T) == 8) {
    TXE_BACK(8, 0);
  } else {
    for (int mb0 = 0; mb0 < nbt; mb0 += 4) TXE_BACK(4, mb0);
  }
#undef TXE_BACK
  return hipGetLastError();
}

template <typename T, typename Tin, typename Tps, int NCG>
hipError_t launch_back_b_tps(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  switch (a.D.MT1) {
    case 1: return launch_back_b_mt<T, Tin, Tps, 1, NCG>(tb, a, s);
    case 2: return launch_back_b_mt<T, Tin, Tps, 2, NCG>(tb, a, s);
    case 3: return launch_back_b_mt<T, Tin, Tps, 3, NCG>(tb, a, s);
    case 4: return launch_back_b_mt<T, Tin, Tps, 4, NCG>(tb, a, s);
    case 5: return launch_back_b_mt<T, Tin, Tps, 5, NCG>(tb, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename Tin, int NCG>
hipError_t launch_back_b_ncg(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  if constexpr (sizeof(T) == 4 && sizeof(Tin) == 8)
    if (a.psi32) return launch_back_b_tps<T, Tin, float, NCG>(tb, a, s);
  return launch_back_b_tps<T, Tin, Tin, NCG>(tb, a, s);
}

template <typename T, typename Tin>
hipError_t launch_back(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  // form: streaming (k_back_s, runtime rank loops, high occupancy) or
  // batched (k_back_b, compile-time rank tiles, loads issued per source in
  // batches).  Default: batched, which measured fastest on the 64^3 and
  // 80^3 workloads in both precisions
  const bool batched = a.back_form ? a.back_form == 2 : true;
  // two c-tiles per wavefront while the b-tile accumulators are few
  const int ncg = a.back_ncg ? a.back_ncg : ((a.D.nb1 >> 4) <= 4 ? 2 : 1);
  if (batched) return ncg == 2 ? launch_back_b_ncg<T, Tin, 2>(tb, a, s) : launch_back_b_ncg<T, Tin, 1>(tb, a, s);
  return ncg == 2 ? launch_back_s_ncg<T, Tin, 2>(tb, a, s) : launch_back_s_ncg<T, Tin, 1>(tb, a, s);
}

template <typename T, typename Tin, int MT>
void launch_proj12m_mt(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s) {
  const unsigned nb = blocks_for((long long)a.P * a.D.n0);
  const size_t tab = ((size_t)a.D.nc2 * 16 * MT + (size_t)MT * (a.D.nb1 >> 4) * 256) * sizeof(T);
  if (tab <= 64 * 1024)
    hipLaunchKernelGGL((k_proj12m<T, Tin, MT, true>), dim3(std::min(nb, (unsigned)a.grid_cap)), dim3(256), tab, s,
                       (const Tin *)a.psi, a.D, a.pm, a.P, tb, a.T2);
  else
    hipLaunchKernelGGL((k_proj12m<T, Tin, MT, false>), dim3(nb), dim3(256), 0, s, (const Tin *)a.psi, a.D, a.pm,
                       a.P, tb, a.T2);
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

template <typename T, typename Tin>
hipError_t run_chunk_t(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s, Prof *prof,
                       const BfTables *bft = nullptr, int nsplit = 0) {
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
  {
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
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  prof->begin(K_CORE, s);
  if constexpr (sizeof(T) == 4) {
    if (nsplit == 2) e = launch_core_bf<2>(tb, *bft, a, want_vx, s);
    else if (nsplit == 3) e = launch_core_bf<3>(tb, *bft, a, want_vx, s);
    else e = launch_core<T>(tb, a, want_vx, s);
  } else {
    e = launch_core<T>(tb, a, want_vx, s);
  }
  prof->end(s);
  if (e != hipSuccess) return e;
  {
    const int parts = a.D.MT1 * a.NGS;
    prof->begin(K_EPAIR, s);
    hipLaunchKernelGGL(k_epair, dim3((a.P + 255) / 256), dim3(256), 0, s, a.epart, a.P, parts, a.pm.p0, a.epair);
    prof->end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (want_vx) {
    prof->begin(K_BACK, s);
    e = launch_back<T, Tin>(tb, a, s);
    prof->end(s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

int core_rows(bool f64, int nsplit, int mt) {
  if (f64) return 4 * NGW64[mt];
  if (nsplit == 3 || NW32[mt] == 4) return 4 * NGW32[mt];
  return 8 * NGW32x8[mt];  // FP32 and two-part bf16 at up to three tiles
}

hipError_t run_chunk_f64(const Tables<double> &tb, const ChunkArgs<double> &a, bool want_vx, hipStream_t s,
                         Prof *prof) {
  return run_chunk_t<double, double>(tb, a, want_vx, s, prof);
}

hipError_t run_chunk_f32(const Tables<float> &tb, const ChunkArgs<float> &a, bool psi_f64, bool want_vx,
                         hipStream_t s, Prof *prof) {
  if (psi_f64) return run_chunk_t<float, double>(tb, a, want_vx, s, prof);
  return run_chunk_t<float, float>(tb, a, want_vx, s, prof);
}

hipError_t run_chunk_bf16(const Tables<float> &tb, const BfTables &bft, int nsplit, const ChunkArgs<float> &a,
                          bool psi_f64, bool want_vx, hipStream_t s, Prof *prof) {
  if (psi_f64) return run_chunk_t<float, double>(tb, a, want_vx, s, prof, &bft, nsplit);
  return run_chunk_t<float, float>(tb, a, want_vx, s, prof, &bft, nsplit);
}

hipError_t run_energy(const double *epair, long long npairs, int symmetric, int N, double *ex, double *e_out,
                      hipStream_t s, Prof *prof) {
  prof->begin(K_ENERGY, s);
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, s, epair, npairs, symmetric, N, ex, e_out);
  prof->end(s);
  return hipGetLastError();
}

}  // namespace txe
