// One chunk of orbital pairs through the exchange path, and the FP64 energy
// reductions.  A chunk runs four kernels (txe_proj.hip, txe_core*.hip,
// txe_back.hip):
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
#include "txe_dev.h"

namespace txe {

// -------------------------------------------------------------------------------------
// pair energies: e_pair[p0 + p] = sum of the core kernel's partials (fixed order)
// -------------------------------------------------------------------------------------
__global__ void k_epair(const double *__restrict__ epart, int P, int parts, PairMap pm, double *__restrict__ epair) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= P) return;
  double s = 0.0;
  for (int q = 0; q < parts; ++q) s += epart[(size_t)p * parts + q];
  int i, j;
  pair_ij(pm, p, i, j);
  epair[apply_pair(pm, i, j)] = s;
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

// Exchange-matrix diagonal of each target, X_ii = <psi_i, Vx psi_i>_W =
// -sum_j e_ij over every source j (FP64, j ascending), from the pair
// energies of the whole apply.  One thread per target.
__global__ __launch_bounds__(256) void k_orb(const double *__restrict__ epair, int symmetric, int N, int i0, int Ni,
                                             double *__restrict__ e_orb) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= Ni) return;
  const int i = symmetric ? t : i0 + t;
  double s = 0.0;
  for (int j = 0; j < N; ++j) {
    long long pg;
    if (symmetric) {
      const int a = min(i, j), b = max(i, j);
      pg = sym_start(a, N) + (b - a);
    } else {
      pg = (long long)t * N + j;
    }
    s -= epair[pg];
  }
  e_orb[t] = s;
}

namespace {

// the core kernel instance of the largest rank-tile count of the system
template <typename T>
hipError_t launch_core(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s) {
  switch (std::max(a.D.MT0, std::max(a.D.MT1, a.D.MT2))) {
    case 1: return launch_core_for_mt<T, 1>(tb, a, want_vx, s);
    case 2: return launch_core_for_mt<T, 2>(tb, a, want_vx, s);
    case 3: return launch_core_for_mt<T, 3>(tb, a, want_vx, s);
    case 4: return launch_core_for_mt<T, 4>(tb, a, want_vx, s);
    case 5: return launch_core_for_mt<T, 5>(tb, a, want_vx, s);
  }
  return hipErrorInvalidValue;
}

template <typename T, typename Tin>
hipError_t run_chunk_t(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s, Prof *prof,
                       const BfTables *bft = nullptr, int nsplit = 0) {
  hipError_t e = launch_projection<T, Tin>(tb, a, s, prof);
  if (e != hipSuccess) return e;
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
    hipLaunchKernelGGL(k_epair, dim3((a.P + 255) / 256), dim3(256), 0, s, a.epart, a.P, parts, a.pm, a.epair);
    prof->end(s);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (want_vx) {
    for (int b = 0; b < a.nbr; ++b) {
      prof->begin(K_BACK, s);
      e = launch_back<T, Tin>(tb, a, a.br[b], s);
      prof->end(s);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

}  // namespace

int core_rows(bool f64, int nsplit, int mt) {
  if (f64) return 4 * NGW64[mt];
  if (nsplit == 3 || (nsplit == 2 && mt >= 4) || NW32[mt] == 4) return 4 * NGW32[mt];  // four wavefronts
  return 8 * NGW32x8[mt];  // eight: FP32 up to four tiles, two-part bf16 up to three
}

hipError_t launch_core_f64(const Tables<double> &tb, const ChunkArgs<double> &a, bool want_vx, hipStream_t s) {
  return launch_core<double>(tb, a, want_vx, s);
}

hipError_t launch_epair(const double *epart, int P, int parts, const PairMap &pm, double *epair, hipStream_t s) {
  hipLaunchKernelGGL(k_epair, dim3((P + 255) / 256), dim3(256), 0, s, epart, P, parts, pm, epair);
  return hipGetLastError();
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

hipError_t run_energy(const double *epair, long long npairs, int symmetric, int N, int i0, int Ni, double *ex,
                      double *e_out, double *e_orb, hipStream_t s, Prof *prof) {
  prof->begin(K_ENERGY, s);
  hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, s, epair, npairs, symmetric, N, ex, e_out);
  if (e_orb)
    hipLaunchKernelGGL(k_orb, dim3((unsigned)((Ni + 255) / 256)), dim3(256), 0, s, epair, symmetric, N, i0, Ni,
                       e_orb);
  prof->end(s);
  return hipGetLastError();
}

}  // namespace txe
