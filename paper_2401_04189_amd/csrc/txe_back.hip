// Back-projection, product with psi_j and the sum over sources (eq.
// `hadam`), accumulated in registers without atomics.
#include "txe_dev.h"

namespace txe {

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
//   k_back_l  LDS-staged: the four wavefronts of a workgroup share the
//             target and slab a and take four c-tile groups; each source's
//             S1 slab is loaded once per workgroup in 16-byte pieces one
//             source ahead and read from LDS, the chained U1 fragments are
//             staged in LDS once per workgroup, and every b tile is done in
//             one pass, so X is computed once per source (FP32: two
//             workgroups per CU; FP64: one, its LDS up to 160 KiB).  Same
//             products in the same order as k_back_b.
// -------------------------------------------------------------------------------------
template <typename T, typename Tin, int NBT, int NCG, bool LDS_TAB>
__global__ __launch_bounds__(256) void k_back_s(const T *__restrict__ S1, const Tin *__restrict__ psi, Dims D,
                                              PairMap pm, BackRange br, Tables<T> tb,
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
  const long long total = (long long)br.nt * D.n0 * ncg;
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
  const int cgi = (int)(item % ncg);
  const long long rest = item / ncg;
  const int a = (int)(rest % D.n0);
  const int tglob = br.t0 + (int)(rest / D.n0);       // orbital index of the target
  const int c0 = cgi * NCG;
  const size_t plane = (size_t)D.n1 * D.n2;
  const size_t S1pair = (size_t)D.n0 * D.rp2 * D.rp1;

  Tin *out = vx + (size_t)(tglob - br.out0) * D.n0 * plane + (size_t)a * plane;
  acc Acc[NBT][NCG];
#pragma unroll
  for (int mb = 0; mb < NBT; ++mb)
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) {
      Acc[mb][cg] = zero4<acc>();
      // raw sums of the target's earlier sources (an earlier chunk)
      const int c = 16 * (c0 + cg) + lr;
      if (br.acc_in && mb < nbt && c0 + cg < nct && c < D.n2) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int b = 16 * mb + drow<T>(lg, v);
          if (b < D.n1) Acc[mb][cg][v] = (T)out[(size_t)b * D.n2 + c];
        }
      }
    }

  for (int s = br.s0; s < br.s0 + br.ns; ++s) {
    const long long pl = local_pair(pm, br, tglob, s);
    const T *S = S1 + (size_t)pl * S1pair + (size_t)a * D.rp2 * D.rp1 + lr;
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
              if (br.finish) {
                double val = -scale * (double)Acc[mbb][cg][v];
                if (weighted) val *= q0[a] * q1[b] * q2[c];
                out[(size_t)b * D.n2 + c] = (Tin)val;
              } else {
                out[(size_t)b * D.n2 + c] = (Tin)Acc[mbb][cg][v];  // raw sum, exact in Tin
              }
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
                                                PairMap pm, BackRange br, Tables<T> tb,
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
  const long long total = (long long)br.nt * D.n0 * ncg;
  // per-lane offsets are 32-bit and unsigned, added to wave-uniform bases
  const unsigned soff = (unsigned)(lg * RP + lr);  // S1 fragment element of this lane
  for (long long item = (long long)blockIdx.x * 4 + wave; item < total; item += (long long)gridDim.x * 4) {
    const int cgi = (int)(item % ncg);
    const long long rest = item / ncg;
    const int a = (int)(rest % D.n0);
    const int tglob = br.t0 + (int)(rest / D.n0);       // orbital index of the target
    Tin *out = vx + (size_t)(tglob - br.out0) * D.n0 * plane + (size_t)a * plane;
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
    // (b tile mbb adds 16 mbb rows to the first tile's rows; the last row
    // clamps every offset into the plane)
    unsigned poff0[4];  // within one plane (n1 n2 < 2^31)
#pragma unroll
    for (int v = 0; v < 4; ++v) poff0[v] = (unsigned)((16 * mb0 + drow<T>(lg, v)) * D.n2);
    const unsigned plast = (unsigned)((D.n1 - 1) * D.n2), prow16 = (unsigned)(16 * D.n2);
    unsigned pc[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) pc[cg] = (unsigned)min(16 * ct[cg] + lr, D.n2 - 1);

    acc Acc[NBT][NCG];
#pragma unroll
    for (int mb = 0; mb < NBT; ++mb)
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) Acc[mb][cg] = zero4<acc>();
    if (br.acc_in) {
      // raw sums of the target's earlier sources (an earlier chunk)
#pragma unroll
      for (int mbb = 0; mbb < NBT; ++mbb) {
        if (mb0 + mbb >= nbt) break;  // uniform
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          const int c = 16 * (cgi * NCG + cg) + lr;
          if (cgi * NCG + cg < nct && c < D.n2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int b = 16 * (mb0 + mbb) + drow<T>(lg, v);
              if (b < D.n1) Acc[mbb][cg][v] = (T)out[(size_t)b * D.n2 + c];
            }
          }
        }
      }
    }

    for (int s = br.s0; s < br.s0 + br.ns; ++s) {
      const long long pl = local_pair(pm, br, tglob, s);
      const auto *S = wave_uniform(S1 + (size_t)pl * S1pair + (size_t)a * RP * RP);
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
          for (int v = 0; v < 4; ++v) pv[cg][v] = ps[min(poff0[v] + (unsigned)mbb * prow16, plast) + pc[cg]];
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
              if (br.finish) {
                double val = -scale * (double)Acc[mbb][cg][v];
                if (weighted) val *= q0[a] * q1[b] * q2[c];
                out[(size_t)b * D.n2 + c] = (Tin)val;
              } else {
                out[(size_t)b * D.n2 + c] = (Tin)Acc[mbb][cg][v];  // raw sum, exact in Tin
              }
            }
          }
        }
      }
    }
  }
}

// row stride of the staged S1 slab: four rows 4 apart start in four
// different quarters of the 64 LDS banks, so a fragment read (16 lanes per
// row) is conflict-free
__host__ __device__ constexpr int back_srs(int rp) { return rp % 32 == 16 ? rp : rp + 16; }

template <typename T, typename Tin, typename Tps, int MT, int NBT, int NCG>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 2 : 1))) void k_back_l(const T *__restrict__ S1, const Tps *__restrict__ psi, Dims D,
                                                PairMap pm, BackRange br, Tables<T> tb,
                                                Tin *__restrict__ vx, const double *__restrict__ out_scale,
                                                int weighted, const double *__restrict__ q0,
                                                const double *__restrict__ q1, const double *__restrict__ q2) {
  using M = MF<T>;
  using acc = typename M::acc;
  typedef T V16 __attribute__((ext_vector_type(16 / sizeof(T))));
  constexpr int RP = 16 * MT;
  constexpr int SRS = back_srs(RP);
  constexpr int PE = 16 / (int)sizeof(T);  // values per 16-byte piece
  constexpr int NPC = RP * RP / PE;        // pieces per slab
  constexpr int EPT = (NPC + 255) / 256;   // pieces per thread
  constexpr int KTB = 2;                   // S1 rows (gamma') per batch of LDS reads
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int lane = threadIdx.x & 63, lr = lane & 15, lg = lane >> 4;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform per wavefront
  const int tid = threadIdx.x;
  const int nct = D.nc2 >> 4, nbt = D.nb1 >> 4;
  const int ncq = (nct + 4 * NCG - 1) / (4 * NCG);
  const int nkt = (D.r2 + 3) >> 2;  // gamma' rows in use, in fours
  T *Ss = reinterpret_cast<T *>(smem_raw);  // [RP][SRS]: the source's S1 slab, S1[gamma'][beta']
  T *U1c = Ss + RP * SRS;                   // chained U1 fragments [nbt][MT][4][64]
  for (int idx = tid; idx < nbt * MT * 256; idx += 256) U1c[idx] = tb.U1chain[idx];
  // (visible after the first source's barriers)
  const size_t plane = (size_t)D.n1 * D.n2;
  const size_t S1pair = (size_t)D.n0 * RP * RP;
  const long long total = (long long)br.nt * D.n0 * ncq;
  const unsigned soff = (unsigned)(lg * SRS + lr);  // S1 fragment element of this lane
  for (long long item = blockIdx.x; item < total; item += gridDim.x) {  // uniform per workgroup
    const int cq = (int)(item % ncq);
    const long long rest = item / ncq;
    const int a = (int)(rest % D.n0);
    const int tglob = br.t0 + (int)(rest / D.n0);
    Tin *out = vx + (size_t)(tglob - br.out0) * D.n0 * plane + (size_t)a * plane;
    const int c0 = (4 * cq + wave) * NCG;  // first c tile of this wavefront
    // c tiles past the last one repeat it and are never stored
    int ct[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) ct[cg] = min(c0 + cg, nct - 1);
    T bu[4 * MT][NCG];
#pragma unroll
    for (int kt = 0; kt < 4 * MT; ++kt)
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) bu[kt][cg] = tb.U2T[(unsigned)((4 * kt + lg) * D.nc2 + 16 * ct[cg] + lr)];
    unsigned poff0[4];  // within one plane (n1 n2 < 2^31); b tile mbb adds 16 mbb rows, clamped to the last row
#pragma unroll
    for (int v = 0; v < 4; ++v) poff0[v] = (unsigned)(drow<T>(lg, v) * D.n2);
    const unsigned plast = (unsigned)((D.n1 - 1) * D.n2), prow16 = (unsigned)(16 * D.n2);
    unsigned pc[NCG];
#pragma unroll
    for (int cg = 0; cg < NCG; ++cg) pc[cg] = (unsigned)min(16 * ct[cg] + lr, D.n2 - 1);

    acc Acc[NBT][NCG];
#pragma unroll
    for (int mb = 0; mb < NBT; ++mb)
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) Acc[mb][cg] = zero4<acc>();
    if (br.acc_in) {
#pragma unroll
      for (int mbb = 0; mbb < NBT; ++mbb) {
        if (mbb >= nbt) break;  // uniform
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) {
          const int c = 16 * (c0 + cg) + lr;
          if (c0 + cg < nct && c < D.n2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int b = 16 * mbb + drow<T>(lg, v);
              if (b < D.n1) Acc[mbb][cg][v] = (T)out[(size_t)b * D.n2 + c];
            }
          }
        }
      }
    }
    // the next source's slab, in flight during this source's MFMAs
    V16 pre[EPT];
    auto fetch = [&](int s_) {
      const V16 *src = reinterpret_cast<const V16 *>(S1 + (size_t)local_pair(pm, br, tglob, s_) * S1pair +
                                                     (size_t)a * RP * RP);
#pragma unroll
      for (int j = 0; j < EPT; ++j) pre[j] = src[min(j * 256 + tid, NPC - 1)];
    };
    fetch(br.s0);
    for (int s = br.s0; s < br.s0 + br.ns; ++s) {
      __syncthreads();  // every wavefront is done with the previous slab
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        const int e = j * 256 + tid;
        if (e < NPC) *reinterpret_cast<V16 *>(Ss + (PE * e / RP) * SRS + PE * e % RP) = pre[j];
      }
      __syncthreads();
      if (s + 1 < br.s0 + br.ns) fetch(s + 1);
      const auto *ps = wave_uniform(psi + (size_t)s * D.n0 * plane + (size_t)a * plane);
      // the psi row bases, made opaque per source so the per-tile offsets are
      // formed next to their loads instead of held across the source loop
      unsigned pb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        pb[v] = poff0[v];
        asm volatile("" : "+v"(pb[v]));
      }
      // X[beta'][c] = sum_gamma' S1[gamma'][beta'] U2[c][gamma']
      acc X[MT][NCG];
#pragma unroll
      for (int mb = 0; mb < MT; ++mb)
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) X[mb][cg] = zero4<acc>();
#pragma unroll
      for (int kb = 0; kb < 4 * MT; kb += KTB) {
        // uniform: padded gamma' rows only (FP64 skips them instead of leaving
        // the loop: with the exit the compiler left it rolled and moved bu to
        // scratch)
        if constexpr (sizeof(T) == 4) {
          if (kb >= nkt) break;
        } else if (kb >= nkt) {
          continue;
        }
        T sf[KTB][MT];
#pragma unroll
        for (int k = 0; k < KTB; ++k) {
          const int gam = 4 * (kb + k) + lg;
#pragma unroll
          for (int mb = 0; mb < MT; ++mb) {
            const T x = Ss[soff + (unsigned)(4 * (kb + k) * SRS + 16 * mb)];
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
        if (mbb >= nbt) break;  // uniform
        __builtin_amdgcn_sched_barrier(0);
        Tps pv[NCG][4];
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg)
#pragma unroll
          for (int v = 0; v < 4; ++v) pv[cg][v] = ps[min(pb[v] + (unsigned)mbb * prow16, plast) + pc[cg]];
        acc ph[NCG];
#pragma unroll
        for (int cg = 0; cg < NCG; ++cg) ph[cg] = zero4<acc>();
#pragma unroll
        for (int mbe = 0; mbe < MT; ++mbe)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T af = U1c[lane + ((mbb * MT + mbe) * 4 + v) * 64];
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
    // lane indices rebuilt from an opaque copy: the output addresses are then
    // formed here, not shared with the initial read and held across the loop
    int ln = lane;
    asm volatile("" : "+v"(ln));
    const int lre = ln & 15, lge = ln >> 4;
#pragma unroll
    for (int mbb = 0; mbb < NBT; ++mbb) {
      if (mbb >= nbt) break;
#pragma unroll
      for (int cg = 0; cg < NCG; ++cg) {
        const int c = 16 * (c0 + cg) + lre;
        if (c0 + cg < nct && c < D.n2) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int b = 16 * mbb + drow<T>(lge, v);
            if (b < D.n1) {
              if (br.finish) {
                double val = -scale * (double)Acc[mbb][cg][v];
                if (weighted) val *= q0[a] * q1[b] * q2[c];
                out[(size_t)b * D.n2 + c] = (Tin)val;
              } else {
                out[(size_t)b * D.n2 + c] = (Tin)Acc[mbb][cg][v];  // raw sum, exact in Tin
              }
            }
          }
        }
      }
    }
  }
}

// LDS bytes of k_back_l: the staged slab and the chained U1 fragments
inline size_t back_l_lds(int mt, int nbt, size_t elt) {
  return ((size_t)16 * mt * back_srs(16 * mt) + (size_t)nbt * mt * 256) * elt;
}

template <typename T, typename Tin, typename Tps, int MT, int NCG>
hipError_t launch_back_l_mt(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  const int nct = a.D.nc2 >> 4, nbt = a.D.nb1 >> 4;
  const long long items = (long long)br.nt * a.D.n0 * ((nct + 4 * NCG - 1) / (4 * NCG));
  const unsigned nb = (unsigned)std::min<long long>(items, a.grid_cap);
  const Tps *psi = std::is_same<Tps, Tin>::value ? (const Tps *)a.psi : (const Tps *)a.psi32;
  Tin *vx = (Tin *)a.vx;
  const size_t lds = back_l_lds(MT, nbt, sizeof(T));
  if constexpr (NCG == 2)  // two c tiles per wavefront only up to four b tiles (registers)
    if (nbt > 4) return launch_back_l_mt<T, Tin, Tps, MT, 1>(tb, a, br, s);
  auto go = [&](auto nbt_c) -> hipError_t {
    constexpr int NB = decltype(nbt_c)::value;
    if constexpr (NCG == 2 && NB > 4) return hipErrorInvalidValue;  // not reached
    const void *fn = (const void *)k_back_l<T, Tin, Tps, MT, NB, NCG>;
    if (lds > 64 * 1024) {
      const hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_back_l<T, Tin, Tps, MT, NB, NCG>), dim3(nb), dim3(256), lds, s, a.S1, psi, a.D, a.pm, br,
                       tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1], a.qdev[2]);
    return hipGetLastError();
  };
  if (nbt <= 2) return go(std::integral_constant<int, 2>{});
  if (nbt <= 4) return go(std::integral_constant<int, 4>{});
  if (nbt <= 6) return go(std::integral_constant<int, 6>{});
  if (nbt <= 8) return go(std::integral_constant<int, 8>{});
  return hipErrorInvalidValue;
}

template <typename T, typename Tin, typename Tps, int NCG>
hipError_t launch_back_l_tps(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  switch (a.D.MT1) {
    case 1: return launch_back_l_mt<T, Tin, Tps, 1, NCG>(tb, a, br, s);
    case 2: return launch_back_l_mt<T, Tin, Tps, 2, NCG>(tb, a, br, s);
    case 3: return launch_back_l_mt<T, Tin, Tps, 3, NCG>(tb, a, br, s);
    case 4: return launch_back_l_mt<T, Tin, Tps, 4, NCG>(tb, a, br, s);
    case 5: return launch_back_l_mt<T, Tin, Tps, 5, NCG>(tb, a, br, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename Tin, int NCG>
hipError_t launch_back_l_ncg(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  if constexpr (sizeof(T) == 4 && sizeof(Tin) == 8)
    if (a.psi32) return launch_back_l_tps<T, Tin, float, NCG>(tb, a, br, s);
  return launch_back_l_tps<T, Tin, Tin, NCG>(tb, a, br, s);
}

template <typename T, typename Tin, int NCG>
hipError_t launch_back_s_ncg(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  const int nct = a.D.nc2 >> 4, nbt = a.D.nb1 >> 4;
  const long long waves = (long long)br.nt * a.D.n0 * ((nct + NCG - 1) / NCG);
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
                       br, tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1], a.qdev[2]);                    \
  else                                                                                                           \
    hipLaunchKernelGGL((k_back_s<T, Tin, NBTV, NCG, false>), dim3(nb), dim3(256), 0, s, a.S1, psi, a.D, a.pm,    \
                       br, tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1], a.qdev[2])
  if (nbt <= 2) TXE_BACK(2);
  else if (nbt <= 4) TXE_BACK(4);
  else if (nbt <= 6) TXE_BACK(6);
  else if (nbt <= 8) TXE_BACK(8);
  else return hipErrorInvalidValue;
#undef TXE_BACK
  return hipGetLastError();
}

template <typename T, typename Tin, typename Tps, int MT, int NCG>
hipError_t launch_back_b_mt(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  const int nct = a.D.nc2 >> 4, nbt = a.D.nb1 >> 4;
  const long long waves = (long long)br.nt * a.D.n0 * ((nct + NCG - 1) / NCG);
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
  // four b tiles, each recomputing X for its sources: one launch of eight
  // tiles holds one wavefront per SIMD and measured twice as slow at 128^3
  // (the kernel hides its load latency with a second wavefront)
  if (nbt > 8) return hipErrorInvalidValue;
#define TXE_BACK(NBTV, MB0)                                                                                      \
  do {                                                                                                           \
    if (lds_tab)                                                                                                 \
      hipLaunchKernelGGL((k_back_b<T, Tin, Tps, MT, NBTV, NCG, true>), dim3(nbl), dim3(256), lds, s, a.S1, psi, a.D,  \
                         a.pm, br, tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1], a.qdev[2], MB0);      \
    else                                                                                                         \
      hipLaunchKernelGGL((k_back_b<T, Tin, Tps, MT, NBTV, NCG, false>), dim3(nbl), dim3(256), 0, s, a.S1, psi, a.D,   \
                         a.pm, br, tb, vx, a.out_scale, a.weighted, a.qdev[0], a.qdev[1], a.qdev[2], MB0);      \
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
hipError_t launch_back_b_tps(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  switch (a.D.MT1) {
    case 1: return launch_back_b_mt<T, Tin, Tps, 1, NCG>(tb, a, br, s);
    case 2: return launch_back_b_mt<T, Tin, Tps, 2, NCG>(tb, a, br, s);
    case 3: return launch_back_b_mt<T, Tin, Tps, 3, NCG>(tb, a, br, s);
    case 4: return launch_back_b_mt<T, Tin, Tps, 4, NCG>(tb, a, br, s);
    case 5: return launch_back_b_mt<T, Tin, Tps, 5, NCG>(tb, a, br, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename Tin, int NCG>
hipError_t launch_back_b_ncg(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  if constexpr (sizeof(T) == 4 && sizeof(Tin) == 8)
    if (a.psi32) return launch_back_b_tps<T, Tin, float, NCG>(tb, a, br, s);
  return launch_back_b_tps<T, Tin, Tin, NCG>(tb, a, br, s);
}

template <typename T, typename Tin>
hipError_t launch_back(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s) {
  // form: streaming (k_back_s, runtime rank loops, high occupancy), batched
  // (k_back_b, compile-time rank tiles, loads issued per source in batches)
  // or LDS-staged (k_back_l: FP32 while its LDS leaves room for two
  // workgroups per CU, FP64 while it fits one).  Default: LDS-staged where
  // it applies, else batched
  const int nbt = a.D.nb1 >> 4;
  // (FP32 compute reads FP64 orbitals as they are, without an FP32 copy, only
  // up to six b tiles: registers)
  const bool psi64_direct = sizeof(T) == 4 && sizeof(Tin) == 8 && !a.psi32;
  const bool lds_ok = nbt <= (psi64_direct ? 6 : 8) &&
                      back_l_lds(a.D.MT1, nbt, sizeof(T)) <= (sizeof(T) == 4 ? 80 : 160) * 1024;
  const int form = a.back_form == 3 && !lds_ok ? 2 : a.back_form ? a.back_form : (lds_ok ? 3 : 2);
  if (form == 3) {
    const int ncg = a.back_ncg ? a.back_ncg : 1;
    return ncg == 2 ? launch_back_l_ncg<T, Tin, 2>(tb, a, br, s) : launch_back_l_ncg<T, Tin, 1>(tb, a, br, s);
  }
  // two c-tiles per wavefront while the b-tile accumulators are few
  const int ncg = a.back_ncg ? a.back_ncg : (nbt <= 4 ? 2 : 1);
  if (form != 1) return ncg == 2 ? launch_back_b_ncg<T, Tin, 2>(tb, a, br, s) : launch_back_b_ncg<T, Tin, 1>(tb, a, br, s);
  return ncg == 2 ? launch_back_s_ncg<T, Tin, 2>(tb, a, br, s) : launch_back_s_ncg<T, Tin, 1>(tb, a, br, s);
}

template hipError_t launch_back<double, double>(const Tables<double> &, const ChunkArgs<double> &, const BackRange &,
                                                hipStream_t);
template hipError_t launch_back<float, double>(const Tables<float> &, const ChunkArgs<float> &, const BackRange &,
                                               hipStream_t);
template hipError_t launch_back<float, float>(const Tables<float> &, const ChunkArgs<float> &, const BackRange &,
                                              hipStream_t);

}  // namespace txe
