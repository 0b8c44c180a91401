// The core-space Gaussian kernel sum of one pair (eqs. `gauss`, `final`
// restricted to the Tucker core), with the pair energy and the first
// back-projection stage in its epilogue: the kernel template and its
// launcher, instantiated per precision in txe_core_f32.hip / txe_core_f64.hip.
#pragma once

#include "txe_dev.h"

namespace txe {

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
template <typename T, int MT, int NGW, int NW, bool WRITE_S1, int TL, int TZ>
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
  if (tb.ps_c1 | tb.ps_c2 | tb.ps_ah | tb.ps_u0) {  // uniform: this pair's own tables
    tb.C1f += (size_t)p * tb.ps_c1;
    tb.C2chain += (size_t)p * tb.ps_c2;
    tb.Ahat += (size_t)p * tb.ps_ah;
    tb.U0chain += (size_t)p * tb.ps_u0;
  }

  // Register plan per precision and rank tile:
  //   PF     Chat1 / Ahat fragments prefetched one step ahead
  //   C2S    Chat2 fragments loaded whole at the start of the step (else one
  //          gamma' tile at a time inside the Z chain)
  //   HOLD_G the slab's A fragments held in registers for all of its steps
  //          (FP64 at up to two tiles)
  //   LDS_G  the slab in LDS instead (double-buffered; every FP32 form),
  //          each row laid out so a lane reads its fragments with one load
  //   KM     term-major order (see below): every FP32 form and FP64 at up
  //          to three tiles; it holds the term's Chat1 fragments and the
  //          Chat2 fragments of the TZ gamma' tiles this workgroup's split
  //          meets, with the slab in LDS
  constexpr bool F32 = sizeof(T) == 4;
  constexpr bool KM = F32 || MT <= 3 || TZ < MT;
  constexpr bool PF = F32 || MT <= 2;
  constexpr bool C2S = F32 ? MT <= 3 : MT <= 2;
  constexpr bool HOLD_G = !KM && !F32 && C2S && (NW == 4 || MT <= 2);
  constexpr bool LDS_G = KM || (F32 && !HOLD_G);
  // slab gamma row (inside its tile) that this lane feeds to the W chain
  const int lrg = F32 ? ((lr & 3) << 2 | (lr >> 2)) : lr;
  // and the lane that reads slab row gamma (inside its tile) from LDS
  auto lane_of = [](int g16) { return F32 ? ((g16 & 3) << 2 | (g16 >> 2)) : g16; };
  constexpr int NKT = 4 * (MT - 1) + TL;  // K = 4 steps of the beta contraction
  // LDS slab row beta: for each of the 16 lanes of a fragment its MT gamma
  // values (gamma = 16 mg + lane) side by side, padded to LPL, so a lane
  // reads all of its A fragments of one beta row with 16-byte loads (five
  // FP64 values take three 16-byte pieces: LPL = 6 keeps the FP64 slab's
  // double buffer within the LDS)
  constexpr int LPL = MT <= 4 ? 4 : (F32 ? 8 : 6);
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
        Gs[buf * SLAB + (e / RP) * SROW + lane_of(gamma & 15) * LPL + (gamma >> 4)] = v[j];
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
    // inner loop the slabs alpha.  Each wavefront holds its term's Chat1
    // fragments and the Chat2 fragments of the gamma' tiles of this
    // workgroup's split in registers for all r0 slabs, and one whole slab
    // streams through the LDS double buffer per step, so the term tables are
    // read once per term group instead of once per (slab, term group).  The
    // sums are the same as in slab-major order (phase B adds the same
    // products to the same Phi accumulators, in another order).
    // The next slab arrives in 16-byte pieces (RP is a multiple of 16, so a
    // piece stays inside one beta row): EPS pieces per thread and step.
    typedef typename std::conditional<F32, float4, double2>::type V16;
    constexpr int PE = 16 / (int)sizeof(T);       // elements per piece
    constexpr int FP = (int)(F / PE);
    constexpr int EPS = (FP + CHT - 1) / CHT;
    typedef T AF[NTG][MT];
    auto load_af = [&](int alpha_, int kq_, AF &af) {
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg) {
        const T *ah = tb.Ahat + ((size_t)alpha_ * D.Kp + NW * kq_ + 4 * tg + lg) * RP + lr;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[tg][mt] = ah[16 * mt];
      }
    };
    auto kslab_load = [&](int a_, V16 (&v)[EPS]) {
      const V16 *src = reinterpret_cast<const V16 *>(Gp + (size_t)a_ * F);
#pragma unroll
      for (int j = 0; j < EPS; ++j) v[j] = src[min(j * CHT + tid, FP - 1)];
    };
    auto kslab_store = [&](int buf, const V16 (&v)[EPS]) {
      if constexpr (F32) {
        // without a branch: threads past the slab's last piece loaded that
        // piece (clamped) and store it again, the same values
#pragma unroll
        for (int j = 0; j < EPS; ++j) {
          const int e4 = min(j * CHT + tid, FP - 1);
          const int beta = (PE * e4) / RP, g0 = (PE * e4) % RP;
          const T *x = reinterpret_cast<const T *>(&v[j]);
#pragma unroll
          for (int q = 0; q < PE; ++q) {
            const int gamma = g0 + q;
            Gs[buf * SLAB + beta * SROW + lane_of(gamma & 15) * LPL + (gamma >> 4)] = x[q];
          }
        }
        return;
      }
#pragma unroll
      for (int j = 0; j < EPS; ++j) {
        const int e4 = j * CHT + tid;
        if (e4 < FP) {
          const int beta = (PE * e4) / RP, g0 = (PE * e4) % RP;
          const T *x = reinterpret_cast<const T *>(&v[j]);
#pragma unroll
          for (int q = 0; q < PE; ++q) {
            const int gamma = g0 + q;
            Gs[buf * SLAB + beta * SROW + lane_of(gamma & 15) * LPL + (gamma >> 4)] = x[q];
          }
        }
      }
    };
    // the gamma' tiles this workgroup's split meets: mtb .. mtb + nz - 1 (<= TZ);
    // holding all MT tiles, the tile index is compile-time
    constexpr bool ALLT = TZ == MT;
    const int mtb = ALLT ? 0 : g_lo >> 4;
    const int nz = ALLT ? MT : min(TZ, ((max(g_hi, g_lo + 1) - 1) >> 4) - mtb + 1);
    T tcb[4 * MT];
    T c2s[TZ][MT][4];
    AF afa, afb;
    load_af(0, 0, afa);
    auto store_z = [&](T *Zw, int mtp, const acc &Zt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gp = 16 * mtp + drow<T>(lg, v);
        if constexpr (F32) Zw[gp * ZRS + lr] = Zt[v];
        else if (gp >= g_lo && gp < g_hi) Zw[(gp - g_lo) * 16 + lr] = Zt[v];
      }
    };
    // FP64 at four or five tiles (registers): the next slab arrives in two
    // halves (the first during the W chain, the second during the Z chain)
    // and the phase-B columns are loaded in the step that uses them
    constexpr bool SPLIT = !F32 && MT >= 4;
    constexpr int EPS1 = SPLIT ? (EPS + 1) / 2 : EPS;
    auto kslab_load_part = [&](int a_, int j0, V16 (&v)[EPS1]) {
      const V16 *src = reinterpret_cast<const V16 *>(Gp + (size_t)a_ * F);
#pragma unroll
      for (int j = 0; j < EPS1; ++j) v[j] = src[min((j0 + j) * CHT + tid, FP - 1)];
    };
    auto kslab_store_part = [&](int buf, int j0, const V16 (&v)[EPS1]) {
#pragma unroll
      for (int j = 0; j < EPS1; ++j) {
        const int e4 = (j0 + j) * CHT + tid;
        if (j0 + j < EPS && e4 < FP) {
          const int beta = (PE * e4) / RP, g0 = (PE * e4) % RP;
          const T *x = reinterpret_cast<const T *>(&v[j]);
#pragma unroll
          for (int q = 0; q < PE; ++q) {
            const int gamma = g0 + q;
            Gs[buf * SLAB + beta * SROW + lane_of(gamma & 15) * LPL + (gamma >> 4)] = x[q];
          }
        }
      }
    };
    auto kstep = [&](const int kq, const int alpha, const int step, AF &cur, AF &nxt) __attribute__((always_inline)) {
      const int k = NW * kq + wave;
      // the next step's slab (alpha + 1, or alpha 0 of the next term group)
      // and phase-B columns, issued before this step's work
      const bool last_a = alpha + 1 == D.r0;
      const bool more = !last_a || kq + 1 < nkq;  // uniform
      const int a_next = last_a ? 0 : alpha + 1;
      V16 gnext[EPS1];
      if constexpr (SPLIT) kslab_load_part(a_next, 0, gnext);
      else kslab_load(a_next, gnext);
      if constexpr (!SPLIT)
        if (more) load_af(last_a ? 0 : alpha + 1, last_a ? kq + 1 : kq, nxt);
      T *Zw = Zs + (size_t)(step & 1) * zsz + (size_t)wave * ZSS;
      if (k < D.K) {
        acc W[MT];
#pragma unroll
        for (int mg = 0; mg < MT; ++mg) W[mg] = zero4<acc>();
        if constexpr (F32) {
          // the slab fragments of K step kt + 2 are read while the MFMAs of kt
          // run (a ring of three), so the LDS latency stays off the MFMA pipe
          constexpr int NQ = (MT + PE - 1) / PE;
          const V16 *src0 = reinterpret_cast<const V16 *>(Gs + (step & 1) * SLAB + lg * SROW + lr * LPL);
          V16 ring[3][NQ];
          auto rd = [&](int kt_, V16 (&o)[NQ]) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) o[q] = src0[(4 * kt_ * SROW) / PE + q];
          };
          rd(0, ring[0]);
          if (NKT > 1) rd(1, ring[1]);
          __builtin_amdgcn_sched_group_barrier(0x100, NKT > 1 ? 2 * NQ : NQ, 0);  // the first two reads
#pragma unroll
          for (int kt = 0; kt < 4 * MT; ++kt) {
            if (kt >= NKT) break;
            if (kt + 2 < NKT) rd(kt + 2, ring[(kt + 2) % 3]);
            const T *x = reinterpret_cast<const T *>(&ring[kt % 3][0]);
#pragma unroll
            for (int mg = 0; mg < MT; ++mg) W[mg] = M::mma(x[mg], tcb[kt], W[mg]);
            // issue order: the reads of kt + 2, then the MFMAs of kt
            if (kt + 2 < NKT) __builtin_amdgcn_sched_group_barrier(0x100, NQ, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, MT, 0);
          }
        } else {
#pragma unroll
        for (int kt = 0; kt < 4 * MT; ++kt) {
          if (kt >= NKT) break;
          const V16 *src = reinterpret_cast<const V16 *>(Gs + (step & 1) * SLAB + (4 * kt + lg) * SROW + lr * LPL);
          T gl[LPL];
#pragma unroll
          for (int q = 0; q < (MT + PE - 1) / PE; ++q) {
            const V16 f = src[q];
            const T *x = reinterpret_cast<const T *>(&f);
#pragma unroll
            for (int e = 0; e < PE; ++e) gl[PE * q + e] = x[e];
          }
#pragma unroll
          for (int mg = 0; mg < MT; ++mg) W[mg] = M::mma(gl[mg], tcb[kt], W[mg]);
        }
        }
        if constexpr (SPLIT) {  // first half stored, second half issued
          if (more) kslab_store_part((step + 1) & 1, 0, gnext);
          kslab_load_part(a_next, EPS1, gnext);
        }
        // FP32: the next slab goes into the other buffer during the Z chain
        // (that buffer's last reads were before the previous barrier, and its
        // loads had the W chain's time to arrive); its LDS writes are spread
        // between the Z chain's MFMAs.  Written on the last step too, where
        // nothing reads it.
        if constexpr (F32) kslab_store((step + 1) & 1, gnext);
        acc Z[TZ];
#pragma unroll
        for (int z = 0; z < TZ; ++z) Z[z] = zero4<acc>();
#pragma unroll
        for (int mg = 0; mg < MT; ++mg)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            if (mg == MT - 1 && v >= TL) break;
#pragma unroll
            for (int z = 0; z < TZ; ++z) Z[z] = M::mma(c2s[z][mg][v], W[mg][v], Z[z]);
            if constexpr (F32) {
              __builtin_amdgcn_sched_group_barrier(0x008, TZ, 0);
              __builtin_amdgcn_sched_group_barrier(0x200, 2, 0);
            }
          }
#pragma unroll
        for (int z = 0; z < TZ; ++z)
          if (z < nz) store_z(Zw, mtb + z, Z[z]);
      } else {
        if constexpr (F32) {
          kslab_store((step + 1) & 1, gnext);
          for (int idx = lane; idx < (g_hi - g_lo) * 16; idx += 64) Zw[(g_lo + (idx >> 4)) * ZRS + (idx & 15)] = (T)0;
        } else {
          for (int idx = lane; idx < gper * 16; idx += 64) Zw[idx] = (T)0;
        }
        if constexpr (SPLIT) {
          if (more) kslab_store_part((step + 1) & 1, 0, gnext);
          kslab_load_part(a_next, EPS1, gnext);
        }
      }
      if constexpr (SPLIT) {
        if (more) kslab_store_part((step + 1) & 1, EPS1, gnext);
        load_af(alpha, kq, cur);  // this step's phase-B columns, waited for after the barrier
      } else if constexpr (!F32) {
        if (more) kslab_store((step + 1) & 1, gnext);
      }
      __syncthreads();
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
            for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(cur[tg][mt], bz[tg][ng], Phi[mt][ng]);
        }
      } else {
        // FP64: each row's read next to its MFMAs keeps the register file
        // for the Phi accumulators
#pragma unroll
        for (int tg = 0; tg < NTG; ++tg) {
          const T *zrow = zb + (size_t)(4 * tg + lg) * ZSS;
#pragma unroll
          for (int ng = 0; ng < NGW; ++ng) {
            const T bz = zrow[min(wg_lo - g_lo + ng, gper - 1) * 16];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) Phi[mt][ng] = M::mma(cur[tg][mt], bz, Phi[mt][ng]);
          }
        }
      }
    };
    int step = 0;
    for (int kq = 0; kq < nkq; ++kq) {
      const int k = NW * kq + wave;
      if (k < D.K) {
        load_c1(k, tcb);
#pragma unroll
        for (int z = 0; z < TZ; ++z)
#pragma unroll
          for (int mg = 0; mg < MT; ++mg) load_c2(k, ALLT ? z : min(mtb + z, MT - 1), mg, c2s[z][mg]);
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

template <typename T, int MT, int NGW, int NW, int TL, int TZ>
hipError_t launch_core_mt(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s) {
  const int gper = (a.D.r2 + a.NGS - 1) / a.NGS;
  if ((gper + NW - 1) / NW > NGW) return hipErrorInvalidValue;  // the plan gives every wavefront <= NGW rows
  constexpr int RP = 16 * MT;
  constexpr bool km = sizeof(T) == 4 || MT <= 3 || TZ < MT;   // k_core's term-major forms (slab in LDS)
  constexpr bool lds_g = km || sizeof(T) == 4;
  constexpr size_t slab = lds_g ? (size_t)RP * 16 * (MT <= 4 ? 4 : (sizeof(T) == 4 ? 8 : 6)) : 0;
  const size_t zslot = sizeof(T) == 4 ? (size_t)RP * 20 + 16 : (size_t)gper * 16;  // k_core's Z slot
  const size_t lds = (2 * slab + 2 * NW * zslot) * sizeof(T);
  const unsigned nb = (unsigned)((size_t)a.P * a.D.MT1 * a.NGS);
  const void *fn = want_vx ? (const void *)k_core<T, MT, NGW, NW, true, TL, TZ>
                           : (const void *)k_core<T, MT, NGW, NW, false, TL, TZ>;
  if (lds > 64 * 1024) {  // opt in to more than 64 KiB of dynamic LDS (gfx950 has 160 KiB per CU)
    const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  if (want_vx)
    hipLaunchKernelGGL((k_core<T, MT, NGW, NW, true, TL, TZ>), dim3(nb), dim3(64 * NW), lds, s, a.G, a.D, a.P, a.NGS,
                       tb, a.S1, a.epart);
  else
    hipLaunchKernelGGL((k_core<T, MT, NGW, NW, false, TL, TZ>), dim3(nb), dim3(64 * NW), lds, s, a.G, a.D, a.P,
                       a.NGS, tb, a.S1, a.epart);
  return hipGetLastError();
}

// gamma' tiles the widest split of the plan meets
inline int split_tiles(const Dims &D, int NGS) {
  const int gper = (D.r2 + NGS - 1) / NGS;
  int need = 1;
  for (int gs = 0; gs < NGS; ++gs) {
    const int lo = gs * gper, hi = std::min(D.r2, lo + gper);
    if (lo < hi) need = std::max(need, (hi - 1) / 16 - lo / 16 + 1);
  }
  return need;
}

// One rank-tile count: the live chunks TL of the last tile of modes 1 and 2
// and the held gamma' tiles TZ select the instance: the fewest of the
// instance's TZ choices that cover the gamma' tiles the widest split meets,
// else all MT.  Up to three tiles TZ = MT.  FP32 at four tiles: TZ 2 or 3
// (splits of at most 32 rows), at five: 3.  FP64 at four or five tiles:
// splits of at most 16 rows (four per wavefront), TZ 1 or 2 (term-major
// order); TZ = MT (slab-major for FP64) only if a plan ever gave wider splits.
template <typename T, int MT>
hipError_t launch_core_for_mt(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s) {
  constexpr bool f64 = sizeof(T) == 8;
  constexpr int NW = f64 ? 4 : NW32[MT];
  constexpr int NGW = f64 ? NGW64[MT] : (NW == 8 ? NGW32x8[MT] : NGW32[MT]);
  constexpr bool F64W = f64 && MT >= 4;
  constexpr int TZA = F64W ? 1 : (MT <= 3 ? MT : MT == 4 ? 2 : 3);
  constexpr int TZB = F64W ? 2 : (MT == 4 ? 3 : TZA);
  const int st = split_tiles(a.D, a.NGS);
  const int pick = st <= TZA ? 0 : st <= TZB ? 1 : 2;
  const int rt = std::max(a.D.r1, a.D.r2) - 16 * (MT - 1);
  const int tl = std::min(4, std::max(1, (rt + 3) / 4));
#define TXE_CORE_TL(TLV)                                                                  \
  case TLV:                                                                               \
    if (pick == 0) return launch_core_mt<T, MT, NGW, NW, TLV, TZA>(tb, a, want_vx, s);    \
    if constexpr (TZB != TZA)                                                             \
      if (pick == 1) return launch_core_mt<T, MT, NGW, NW, TLV, TZB>(tb, a, want_vx, s);  \
    return launch_core_mt<T, MT, NGW, NW, TLV, MT>(tb, a, want_vx, s);
  switch (tl) {
    TXE_CORE_TL(1)
    TXE_CORE_TL(2)
    TXE_CORE_TL(3)
    TXE_CORE_TL(4)
  }
#undef TXE_CORE_TL
  return hipErrorInvalidValue;
}

}  // namespace txe
