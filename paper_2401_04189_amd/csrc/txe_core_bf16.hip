// The core kernel sum with split-bf16 operands (bf16 MFMA 16x16x32, FP32
// accumulation) for the two chained contractions of each term.
#include "txe_core.h"

namespace txe {

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
// G split into its bf16 parts once per pair, each slab alpha written as the
// term-major core's LDS image: value i of lane ln of (part sp, gamma tile mg,
// beta chunk c) is part sp of G[alpha][32 c + 8 (ln >> 4) + i][16 mg + (ln & 15)]
// (zero for beta past the padded rank).  One thread per (pair, alpha, mg, c, ln).
// -------------------------------------------------------------------------------------
template <int MT, int NS>
__global__ __launch_bounds__(256) void k_split_g(const float *__restrict__ G, int P, unsigned short *__restrict__ Gbf) {
  constexpr int RP = 16 * MT, NC = (RP + 31) / 32;
  constexpr int FRAG = NS * MT * NC * 512;
  const long long total = (long long)P * RP * MT * NC * 64;
  for (long long t = (long long)blockIdx.x * 256 + threadIdx.x; t < total; t += (long long)gridDim.x * 256) {
    const int ln = (int)(t & 63);
    long long r = t >> 6;
    const int c = (int)(r % NC);
    r /= NC;
    const int mg = (int)(r % MT);
    r /= MT;
    const int alpha = (int)(r % RP);
    const long long p = r / RP;
    const int gamma = 16 * mg + (ln & 15), b0 = 32 * c + 8 * (ln >> 4);
    const float *src = G + ((size_t)p * RP + alpha) * RP * RP + gamma;
    float x[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = b0 + i < RP ? src[(size_t)(b0 + i) * RP] : 0.f;
    bf8 o[NS];
    split8<NS>(x, o);
    unsigned short *dst = Gbf + ((size_t)p * RP + alpha) * FRAG + ((size_t)mg * NC + c) * 512 + ln * 8;
#pragma unroll
    for (int sp = 0; sp < NS; ++sp) {
      typedef unsigned int u4 __attribute__((ext_vector_type(4)));
      u4 v;
      __builtin_memcpy(&v, &o[sp], 16);
      *reinterpret_cast<u4 *>(dst + (size_t)sp * MT * NC * 512) = v;
    }
  }
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
template <int MT, int NGW, int NS, int NW, bool WRITE_S1, int TZ>
__global__ __launch_bounds__(64 * NW, 1) void k_core_bf2(const float *__restrict__ G,
                                                         const unsigned short *__restrict__ Gbf, Dims D, int P,
                                                         int NGS, Tables<float> tb, BfTables bft,
                                                         float *__restrict__ S1, double *__restrict__ epart) {
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
  constexpr bool KM = NW == 8 || MT == 4 || (MT == 5 && NS == 2);
  // term-major: slabs arrive as their split images (k_split_g), copied as they are
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  constexpr int NPC = FRAG / 8;  // 16-byte pieces of a slab image
  const unsigned short *Gbp = KM ? Gbf + (size_t)p * RP * FRAG : nullptr;
  if constexpr (KM) {
    const u4 *src = reinterpret_cast<const u4 *>(Gbp);
    u4 *dst = reinterpret_cast<u4 *>(Gs);
    for (int e = tid; e < NPC; e += CHT) dst[e] = src[e];
  } else {
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

  // term-major order as in the FP32 core (eight wavefronts for two-part
  // splits at up to three tiles, and every form at four and five tiles):
  // each wavefront holds its term's split Chat1 fragments and the split
  // Chat2 fragments of the TZ gamma' tiles of its workgroup's split for all
  // slabs; the next slab arrives in 16-byte pieces, EPS per thread and step
  // (the three-part form at five tiles keeps slab-major order: its held
  // fragments would not fit beside the Phi accumulators)
  if constexpr (KM) {
    constexpr int EPS = (NPC + CHT - 1) / CHT;
    typedef float AF[NTG][MT];
    auto load_af = [&](int alpha_, int kq_, AF &af) {
#pragma unroll
      for (int tg = 0; tg < NTG; ++tg) {
        const float *ah = tb.Ahat + ((size_t)alpha_ * D.Kp + NW * kq_ + 4 * tg + lg) * RP + lr;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) af[tg][mt] = ah[16 * mt];
      }
    };
    // the next slab image, 16-byte pieces (threads past the last piece take
    // the last one again and store the same value)
    auto kslab_load = [&](int a_, u4 (&v)[EPS]) {
      const u4 *src = reinterpret_cast<const u4 *>(Gbp + (size_t)a_ * FRAG);
#pragma unroll
      for (int j = 0; j < EPS; ++j) v[j] = src[min(j * CHT + tid, NPC - 1)];
    };
    auto kslab_store = [&](int buf, const u4 (&v)[EPS]) {
      u4 *dst = reinterpret_cast<u4 *>(Gs + buf * FRAG);
#pragma unroll
      for (int j = 0; j < EPS; ++j) dst[min(j * CHT + tid, NPC - 1)] = v[j];
    };
    // the gamma' tiles this workgroup's split meets: mtb .. mtb + nz - 1 (<= TZ);
    // holding all MT tiles, the tile index is compile-time and the tiles
    // outside the split are skipped
    constexpr bool ALLT = TZ == MT;
    const int mtb = ALLT ? 0 : g_lo >> 4;
    const int nz = ALLT ? MT : min(TZ, ((max(g_hi, g_lo + 1) - 1) >> 4) - mtb + 1);
    bf8 hcb[NC][NS];
    bf8 hc2[TZ][NC][NS];
    AF afa, afb;
    load_af(0, 0, afa);
    auto kstep = [&](const int kq, const int alpha, const int step, AF &cur, AF &nxt) __attribute__((always_inline)) {
      const int k = NW * kq + wave;
      const bool last_a = alpha + 1 == D.r0;
      const bool more = !last_a || kq + 1 < nkq;  // uniform
      u4 gnext[EPS];
      kslab_load(last_a ? 0 : alpha + 1, gnext);
      if (more) load_af(last_a ? 0 : alpha + 1, last_a ? kq + 1 : kq, nxt);
      float *Zw = Zs + (size_t)(step & 1) * zsz + (size_t)wave * ZSS;
      if (k < D.K) {
        const unsigned short *gl = Gs + (step & 1) * FRAG + lane * 8;
        acc W[MT];
#pragma unroll
        for (int mg = 0; mg < MT; ++mg) W[mg] = zero4<acc>();
        // the (chunk, tile) pairs in order, their fragments read RA pairs
        // ahead of their MFMAs (a ring of RA + 1; issue order pinned): a
        // pair's MFMAs take about 50 cycles, so the reads need several pairs
        constexpr int NPR = NC * MT;
        constexpr int RA = NS == 2 && NW == 4 ? 4 : 2, RN = RA + 1;  // (eight wavefronts: another hides it)
        bf8 ring[RN][NS];
        auto rdp = [&](int q, bf8 (&o)[NS]) {
#pragma unroll
          for (int sp = 0; sp < NS; ++sp) o[sp] = ld_bf8(gl + ((sp * MT + q % MT) * NC + q / MT) * 512);
        };
#pragma unroll
        for (int q = 0; q < RA; ++q)
          if (q < NPR) rdp(q, ring[q]);
        __builtin_amdgcn_sched_group_barrier(0x100, (NPR < RA ? NPR : RA) * NS, 0);
#pragma unroll
        for (int q = 0; q < NPR; ++q) {
          if (q + RA < NPR) rdp(q + RA, ring[(q + RA) % RN]);
          W[q % MT] = mma_split<NS>(ring[q % RN], hcb[q / MT], W[q % MT]);
          if (q + RA < NPR) __builtin_amdgcn_sched_group_barrier(0x100, NS, 0);
          __builtin_amdgcn_sched_group_barrier(0x008, NS * (NS + 1) / 2, 0);
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
        // the next slab image into the other buffer (last read before the
        // previous barrier) beside the Z chain; on the last step too, where
        // nothing reads it
        kslab_store((step + 1) & 1, gnext);
#pragma unroll
        for (int z = 0; z < TZ; ++z) {
          if (z >= nz) break;  // uniform
          if (ALLT && (16 * z >= g_hi || 16 * z + 16 <= g_lo)) continue;  // uniform: tile outside the split
          acc Z = zero4<acc>();
#pragma unroll
          for (int c = 0; c < NC; ++c) Z = mma_split<NS>(hc2[z][c], wsp[c], Z);
#pragma unroll
          for (int v = 0; v < 4; ++v) Zw[(16 * (mtb + z) + 4 * lg + v) * ZRS + lr] = Z[v];
        }
      } else {
        kslab_store((step + 1) & 1, gnext);
        for (int idx = lane; idx < (g_hi - g_lo) * 16; idx += 64) Zw[(g_lo + (idx >> 4)) * ZRS + (idx & 15)] = 0.f;
      }
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
            for (int z = 0; z < TZ; ++z)
              hc2[z][c][sp] = ld_bf8(c2 + (((size_t)sp * MT + (ALLT ? z : min(mtb + z, MT - 1))) * NC + c) * 512);
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

template <int MT, int NGW, int NS, int NW, int TZ>
hipError_t launch_core_bf2_tz(const Tables<float> &tb, const BfTables &bft, const ChunkArgs<float> &a, bool want_vx,
                              hipStream_t s) {
  const int gper = (a.D.r2 + a.NGS - 1) / a.NGS;
  if ((gper + NW - 1) / NW > NGW) return hipErrorInvalidValue;
  constexpr int RP = 16 * MT, NC = (RP + 31) / 32;
  constexpr size_t frag = (size_t)NS * MT * NC * 512;
  const size_t lds = 2 * frag * sizeof(unsigned short) + (2 * NW * ((size_t)RP * 20 + 16)) * sizeof(float);
  const unsigned nb = (unsigned)((size_t)a.P * a.D.MT1 * a.NGS);
  if (lds > 64 * 1024) {
    const void *fn = want_vx ? (const void *)k_core_bf2<MT, NGW, NS, NW, true, TZ>
                             : (const void *)k_core_bf2<MT, NGW, NS, NW, false, TZ>;
    const hipError_t ea = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (ea != hipSuccess) return ea;
  }
  if (want_vx)
    hipLaunchKernelGGL((k_core_bf2<MT, NGW, NS, NW, true, TZ>), dim3(nb), dim3(64 * NW), lds, s, (const float *)a.G,
                       (const unsigned short *)a.Gbf, a.D, a.P, a.NGS, tb, bft, a.S1, a.epart);
  else
    hipLaunchKernelGGL((k_core_bf2<MT, NGW, NS, NW, false, TZ>), dim3(nb), dim3(64 * NW), lds, s, (const float *)a.G,
                       (const unsigned short *)a.Gbf, a.D, a.P, a.NGS, tb, bft, a.S1, a.epart);
  return hipGetLastError();
}

// held gamma' tiles: 3 when the plan's widest split meets at most three (at
// four and five tiles), else every tile
template <int MT, int NGW, int NS, int NW>
hipError_t launch_core_bf2_mt(const Tables<float> &tb, const BfTables &bft, const ChunkArgs<float> &a, bool want_vx,
                              hipStream_t s) {
  constexpr int TZ3 = MT <= 3 ? MT : 3;
  if (split_tiles(a.D, a.NGS) <= TZ3) return launch_core_bf2_tz<MT, NGW, NS, NW, TZ3>(tb, bft, a, want_vx, s);
  return launch_core_bf2_tz<MT, NGW, NS, NW, MT>(tb, bft, a, want_vx, s);
}

template <int NS>
hipError_t launch_core_bf(const Tables<float> &tb, const BfTables &bft, const ChunkArgs<float> &a, bool want_vx,
                          hipStream_t s) {
  if (bf_frag_elems(a.D.MT0, NS)) {
    // the term-major cores read every slab as its split image
    if (!a.Gbf) return hipErrorInvalidValue;
    const long long threads = (long long)a.P * a.D.rp0 * a.D.MT0 * ((a.D.rp0 + 31) / 32) * 64;
    const dim3 grid((unsigned)std::min<long long>((threads + 255) / 256, 65536));
    switch (a.D.MT0) {
      case 1: hipLaunchKernelGGL((k_split_g<1, NS>), grid, dim3(256), 0, s, (const float *)a.G, a.P, a.Gbf); break;
      case 2: hipLaunchKernelGGL((k_split_g<2, NS>), grid, dim3(256), 0, s, (const float *)a.G, a.P, a.Gbf); break;
      case 3: hipLaunchKernelGGL((k_split_g<3, NS>), grid, dim3(256), 0, s, (const float *)a.G, a.P, a.Gbf); break;
      case 4: hipLaunchKernelGGL((k_split_g<4, NS>), grid, dim3(256), 0, s, (const float *)a.G, a.P, a.Gbf); break;
      default: hipLaunchKernelGGL((k_split_g<5, NS>), grid, dim3(256), 0, s, (const float *)a.G, a.P, a.Gbf); break;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
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

template hipError_t launch_core_bf<2>(const Tables<float> &, const BfTables &, const ChunkArgs<float> &, bool,
                                      hipStream_t);
template hipError_t launch_core_bf<3>(const Tables<float> &, const BfTables &, const ChunkArgs<float> &, bool,
                                      hipStream_t);

}  // namespace txe
