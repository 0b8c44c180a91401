// Device helpers shared by the HIP translation units of the exchange path
// (MFMA wrappers, fragment row order, small loads, pair numbering, XCD-aware
// block order) and the register plans of the core kernels.
//
// All products use 16x16x4 MFMA tiles (f64 or f32) with 64-lane wavefronts.
// Fragment layouts of a 16x16x4 MFMA for lane l (lr = l%16, lg = l/16):
//   A[m][k]: m = lr, k = lg        B[k][n]: k = lg, n = lr
//   D[m][n]: n = lr, m = 4*lg + v (f32) or m = 4*v + lg (f64), v = 0..3 the
//            four accumulator entries (measured on gfx950)
// so an accumulator whose rows are the next contraction index feeds the next
// MFMA as its B operand directly, one entry v at a time ("chained").
#pragma once

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

// row r <= column c of triangle index p of an n x n triangle numbered row by
// row (p = r n - r(r-1)/2 + (c - r))
__device__ __forceinline__ void tri_rc(long long p, int n, int &r, int &c) {
  const double b = 2.0 * (double)n + 1.0;
  long long ii = (long long)floor((b - sqrt(b * b - 8.0 * (double)p)) * 0.5);
  if (ii < 0) ii = 0;
  if (ii > n - 1) ii = n - 1;
  while (ii > 0 && sym_start(ii, n) > p) --ii;
  while (ii + 1 < n && sym_start(ii + 1, n) <= p) ++ii;
  r = (int)ii;
  c = (int)(ii + (p - sym_start(ii, n)));
}

// orbitals (i, j) of local pair p of a tile
__device__ __forceinline__ void pair_ij(const PairMap &pm, long long p, int &i, int &j) {
  if (pm.tri) {
    int r, c;
    tri_rc(p, pm.nr, r, c);
    i = pm.ra + r;
    j = pm.ra + c;
  } else {
    i = pm.ra + (int)(p / pm.nc);
    j = pm.ca + (int)(p % pm.nc);
  }
}

// the apply's number of pair (i, j) (i <= j in symmetric mode)
__device__ __forceinline__ long long apply_pair(const PairMap &pm, int i, int j) {
  return pm.symmetric ? sym_start(i, pm.N) + (j - i) : (long long)(i - pm.i0) * pm.N + j;
}

// local pair of target t and source s in a back-projection launch
__device__ __forceinline__ long long local_pair(const PairMap &pm, const BackRange &br, int t, int s) {
  if (br.side == 2) {
    const int r = min(t, s) - pm.ra, c = max(t, s) - pm.ra;
    return sym_start(r, pm.nr) + (c - r);
  }
  if (br.side == 0) return (long long)(t - pm.ra) * pm.nc + (s - pm.ca);
  return (long long)(s - pm.ra) * pm.nc + (t - pm.ca);
}


inline unsigned blocks_for(long long waves) { return (unsigned)((waves + 3) / 4); }

// Register plans of the core kernels: gamma' rows per wavefront (the Phi
// accumulators take MT * NGW * 4 values per lane) and wavefronts per
// workgroup, per rank-tile count MT.
constexpr int NGW64[MAX_MT + 1] = {0, 4, 8, 10, 4, 4};
constexpr int NGW32[MAX_MT + 1] = {0, 4, 8, 10, 12, 10};
// FP32 core up to four tiles: eight wavefronts per workgroup (two per SIMD,
// so one hides the other's latencies), each with fewer Phi rows
constexpr int NW32[MAX_MT + 1] = {0, 8, 8, 8, 8, 4};
constexpr int NGW32x8[MAX_MT + 1] = {0, 2, 4, 6, 4, 0};

}  // namespace txe
