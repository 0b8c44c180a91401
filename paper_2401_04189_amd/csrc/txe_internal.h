// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

namespace txe {

// ---- FP64 host setup (txe_setup.cpp) ------------------------------------------------
void conv_matrix_1d(int n, const double *x, double alpha, double *C);
void core_matrix(int n, int r, const double *q, const double *U, const double *C, double *Chat);
// ---- order-p Lagrange elements (txe_fe.cpp) ------------------------------------------
void gll_points(int p, double *s, double *w);
void fe_mesh_1d(const double *edges, int ncells, int p, double *x, double *q);
void fe_conv_matrix(const double *edges, int ncells, int p, double alpha, double *C);
constexpr int FE_MAX_ORDER = 10;

inline int rup(int v, int m) { return (v + m - 1) / m * m; }

constexpr int KCHUNK = 8;     // Gaussian terms staged per LDS round in the core kernel
constexpr int MAX_MT = 5;     // rank tiles of 16: r <= 80
constexpr int PB_MAX_N = 96;  // per-pair bases: largest grid extent (two n x n FP64 matrices in LDS)

// Sizes of one system, with the paddings the kernels use.
struct Dims {
  int n0, n1, n2;             // grid points per mode (multiples of 4)
  int na0, nb1, nc2;          // n rounded up to 16
  int r0, r1, r2;             // Tucker ranks
  int rp0, rp1, rp2;          // ranks rounded up to 16
  int MT0, MT1, MT2;          // rp / 16
  int r1k, r2k;               // ranks rounded up to 4
  int K, Kp;                  // Gaussian terms, and K rounded up to KCHUNK
};

// The pairs of one chunk: a tile of orbital pairs, either the rectangle
// rows x cols (block mode: targets x sources; symmetric mode: the pairs
// i < j between two disjoint orbital blocks) or the triangle i <= j of one
// orbital block (symmetric mode).  Local pair p numbers the tile row by row:
// rectangle (i - ra) * nc + (j - ca), triangle r * nr - r(r-1)/2 + (c - r)
// with r = i - ra, c = j - ra.  The apply numbers all of its pairs (the pair
// energies) as symmetric: i*N - i(i-1)/2 + (j-i), block: (i - i0)*N + j.
struct PairMap {
  int tri;                    // 1: triangle of the rows (cols = rows), 0: rectangle
  int ra, nr;                 // first orbital and count of the rows
  int ca, nc;                 // first orbital and count of the columns
  int symmetric, N, i0;       // the apply's numbering
};

// One back-projection launch over a chunk: targets [t0, t0 + nt) against
// sources [s0, s0 + ns).  side 0: the targets are the tile's rows (pair
// (t, s)); 1: its columns (pair (s, t)); 2: triangle (pair (min, max)).
// acc_in: start from the raw sums an earlier chunk left in vx; finish: write
// -scale * sum (times w when weighted) instead of the raw sum.  Each target's
// sources are visited in ascending order across the chunks of an apply, so a
// chunked apply adds the same terms in the same order as a single chunk.
// Output row of target t: t - out0.
struct BackRange {
  int t0, nt, s0, ns;
  int side, acc_in, finish, out0;
};

// Device copies of the setup tables in one compute precision.  Every table
// is zero beyond the true sizes, so padded rows and columns contribute zero.
// "chain" tables hold the A operand of an MFMA whose B operand is the
// accumulator of the previous MFMA, permuted to the accumulator's row order:
// entry [..][v][lane] is M[16*m + lane%16][16*kt + drow(lane/16, v)].  In
// FP32 the core's term tables (C1f, C2chain) keep a lane's four K = 4 steps
// side by side, [..][lane][4], for 16-byte loads.
template <typename T>
struct Tables {
  T *V2B;       // [nc2][rp2]            V2[c][gamma]                    (q2 U2)
  T *V1chain;   // [MT1][nb1/16][4][64]  V1[b][beta] as A[beta][b]
  T *V0K;       // [n0][rp0]             V0[a][alpha]
  // FP32: [Kp][MT1][MT1][64][4] Chat1_k[16bt + l%16][16kq + 4j + l/16] at [k][bt][kq][l][j]
  // FP64: [Kp][rp1][rp1]        Chat1_k[beta'][beta] at [k][beta][beta']
  T *C1f;
  // FP32: [Kp][MT2][MT2][64][4] Chat2_k[16mt' + l%16][16mg + 4v + l/16] at [k][mt'][mg][l][v]
  // FP64: [Kp][MT2][MT2][4][64] the same element at [k][mt'][mg][v][l]
  T *C2chain;
  T *Ahat;      // [r0][Kp][rp0]         w_k Chat0_k[alpha'][alpha] at [alpha][k][alpha']
  T *U0chain;   // [na0/16][MT0][4][64]  U0[a][alpha']
  T *U2T;       // [rp2][nc2]            U2[c][gamma] at [gamma][c]
  T *U1chain;   // [nb1/16][MT1][4][64]  U1[b][beta]
  // per-pair tables (bases of each pair): element strides between the pairs'
  // C1f, C2chain, Ahat and U0chain, indexed by the chunk's local pair; 0 =
  // one table shared by every pair
  long long ps_c1, ps_c2, ps_ah, ps_u0;
};

// Workspace and per-system data of a chunk with per-pair bases (FP64).
struct PairBasesArgs {
  double *X, *X1, *X2, *X3;   // scaled pair densities and the truncated tensors (per-pair strides:
                              // n0 n1 n2, max(r0 n1 n2, n0 n2 rp), r0 r1 n2, r0 r1 r2)
  double *S;                  // Gram matrices, ldS x ldS per pair
  int ldS;
  double *B;                  // the current tensor in its first-stage eigenbasis along the mode (n0 n1 n2)
  double *V, *Wr;             // first-stage eigenvectors (n_d x n_d) and the second-stage leading ones
                              // (n_d x r_d), ldS x ldS per pair
  double *Ut[3];              // leading left singular vectors per mode, n_d x r_d per pair
  const double *Cs[3];        // D C_k^d D^-1 of the system ([K][n][n] per mode, D = diag(sqrt(q_d)))
  const double *w;            // the K term weights (device)
  long long ps_c1, ps_c2, ps_ah, ps_u0;
};

// Values of one slab of G in the split-bf16 core's LDS image (parts x rank
// tiles x K = 32 chunks x 64 lanes x 8), for the rank-tile counts and splits
// whose core runs in term-major order (two-part splits, or four tiles); 0
// otherwise (those cores split the slab as it arrives).
inline int bf_frag_elems(int mt, int nsplit) {
  if (nsplit == 0 || !(nsplit == 2 || mt == 4)) return 0;
  return nsplit * mt * ((16 * mt + 31) / 32) * 512;
}

// Workspace and per-system data of a chunk in the collocation form (FP64).
// Terms are taken in groups of COLLOC_GROUP: modes 2 and 1 per term into a
// stack, then one mode-0 product over the whole group (weights folded into
// the stacked matrix), so phi is read and written once per group.
constexpr int COLLOC_GROUP = 8;
struct CollocArgs {
  const double *A[3];         // A_k^d = C_k^d U_d per mode, [K][n_d][r_d] (device)
  const double *A0s;          // per group g: [n0][COLLOC_GROUP * rp0], column t rp0 + alpha =
                              // w_k A0_k[a][alpha] (k = g COLLOC_GROUP + t; zero past r0 and past K)
  double *Y0;                 // per pair: G x2 A2_k (rp0, rp1, n2)
  double *Ys;                 // per pair: the group's (G x2 A2_k) x1 A1_k stacked, (COLLOC_GROUP rp0, n1, n2)
  double *phi;                // per pair: phi_ij (n0 n1 n2)
};

// Split-bf16 copies of the core kernel's term matrices (bf16 bit patterns).
// Each FP64 value x is split into up to three bf16 parts, x ~ p0 + p1 + p2
// (p0 = bf16(x), p1 = bf16(x - p0), p2 = bf16(x - p0 - p1)); a two-part
// product keeps p0q0 + p0q1 + p1q0, a three-part one adds p0q2 + p1q1 + p2q0.
// K = 32 MFMA fragments hold 8 values per lane: lane l, element i is
// k = 8*(l/16) + i, m or n = l % 16.
struct BfTables {
  const unsigned short *C1;   // [Kp][MT][3][nC][64][8]: B operand, Chat1_k[beta' = 16 bt + n][beta = 32 c + k]
  const unsigned short *C2;   // [Kp][3][MT][nC][64][8]: A operand, Chat2_k[gamma' = 16 mtp + m][gamma(c, k)],
                              //   gamma(c, k) = 16 (2c + i/4) + 4 (l/16) + i%4 (the row order of two
                              //   f32 accumulator tiles)
  int nC;                     // ceil(rp / 32)
};

// Everything one chunk of pairs needs.
template <typename T>
struct ChunkArgs {
  Dims D;
  PairMap pm;
  int P;                      // pairs in the chunk
  int N;                      // orbitals of the apply
  BackRange br[2];            // back-projection launches of the chunk (nbr of them)
  int nbr;
  int NGS;                    // gamma' splits in the core kernel
  int proj_gt;                // gamma tiles per wavefront in proj12 (1, 2 or 3)
  int back_ncg;               // c tiles per wavefront in back (1 or 2; 0 = by size)
  int back_form;              // back kernel form (1 streaming, 2 batched; 0 = default, batched)
  int grid_cap;               // workgroups of the persistent kernels
  const void *psi;
  // FP32 copy of FP64 orbitals for the projection of the reduced-precision
  // forms (null: the projection reads psi); psi32_fill: this chunk writes it
  const float *psi32;
  int psi32_fill;
  size_t psi_elems;           // N * n0 * n1 * n2
  void *vx;
  const double *out_scale;
  int weighted;
  const double *qdev[3];
  T *T2, *G, *S1;
  // split-bf16 cores in term-major order: G split into its bf16 parts once
  // per pair, each slab as the core's LDS image (bf_frag_elems values)
  unsigned short *Gbf;
  double *epart;              // [P][MT1][NGS]
  double *epair;              // all pairs of the apply, in the apply's numbering
};

// Optional per-kernel timing with HIP events recorded on the launch stream.
enum KernelId { K_PROJ12 = 0, K_PROJ3 = 1, K_CORE = 2, K_EPAIR = 3, K_BACK = 4, K_ENERGY = 5, K_COUNT = 6 };

struct Prof {
  bool on = false;
  struct Rec {
    int id;
    hipEvent_t a, b;
  };
  std::vector<Rec> pending;
  std::vector<hipEvent_t> pool;
  Rec cur{};
  double total_ms[K_COUNT] = {};
  long long count[K_COUNT] = {};

  hipEvent_t take() {
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
  void begin(int id, hipStream_t s) {
    if (!on) return;
    cur.id = id;
    cur.a = take();
    cur.b = take();
    (void)hipEventRecord(cur.a, s);
  }
  void end(hipStream_t s) {
    if (!on) return;
    (void)hipEventRecord(cur.b, s);
    pending.push_back(cur);
  }
  // waits for every recorded launch and adds its duration
  void collect() {
    for (Rec &r : pending) {
      (void)hipEventSynchronize(r.b);
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        total_ms[r.id] += ms;
        count[r.id] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    pending.clear();
  }
  void reset() {
    collect();
    for (int i = 0; i < K_COUNT; ++i) {
      total_ms[i] = 0;
      count[i] = 0;
    }
  }
  ~Prof() {
    collect();
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

// Stage launchers of one chunk (each in its own translation unit):
// projection (psi rounding when needed, proj12, proj3), core kernel sum
// (FP64 / FP32 MFMA, or split bf16 with NS parts), back-projection.
template <typename T, typename Tin>
hipError_t launch_projection(const Tables<T> &tb, const ChunkArgs<T> &a, hipStream_t s, Prof *prof);
template <typename T, int MT>
hipError_t launch_core_for_mt(const Tables<T> &tb, const ChunkArgs<T> &a, bool want_vx, hipStream_t s);
template <int NS>
hipError_t launch_core_bf(const Tables<float> &tb, const BfTables &bft, const ChunkArgs<float> &a, bool want_vx,
                          hipStream_t s);
template <typename T, typename Tin>
hipError_t launch_back(const Tables<T> &tb, const ChunkArgs<T> &a, const BackRange &br, hipStream_t s);

// FP64 core kernel of the system's rank tiles, and the pair-energy sums of a
// chunk (txe_chunk.hip)
hipError_t launch_core_f64(const Tables<double> &tb, const ChunkArgs<double> &a, bool want_vx, hipStream_t s);
hipError_t launch_epair(const double *epart, int P, int parts, const PairMap &pm, double *epair, hipStream_t s);

// One chunk with per-pair bases: sequentially truncated HOSVD of every pair
// density, the pair's tables, the core kernel on them, the back-projection
// in the pair's bases (txe_pairbases.hip).  tb holds the per-pair table
// regions (C1f, C2chain, Ahat, U0chain) with their strides.
hipError_t run_chunk_pp(const Tables<double> &tb, const PairBasesArgs &pb, const ChunkArgs<double> &a, bool want_vx,
                        hipStream_t s, Prof *prof);
// One chunk in the collocation form: projection onto the shared bases, the
// term-by-term reconstruction phi = sum_k w_k G x_d (C_k^d U_d), the pair
// energies on the grid and the accumulation of Vx psi (txe_colloc.hip).
hipError_t run_chunk_colloc(const Tables<double> &tb, const CollocArgs &cl, const ChunkArgs<double> &a, bool want_vx,
                            hipStream_t s, Prof *prof);

// Runs one chunk (projection, core sum, back-projection, pair energies).
// Returns hipSuccess or the first launch error.
hipError_t run_chunk_f64(const Tables<double> &tb, const ChunkArgs<double> &a, bool want_vx, hipStream_t s,
                         Prof *prof);
hipError_t run_chunk_f32(const Tables<float> &tb, const ChunkArgs<float> &a, bool psi_f64, bool want_vx,
                         hipStream_t s, Prof *prof);
// FP32 projection and back-projection with the core kernel sum in split bf16
// products (nsplit = 2: three products, 3: six products).
hipError_t run_chunk_bf16(const Tables<float> &tb, const BfTables &bt, int nsplit, const ChunkArgs<float> &a,
                          bool psi_f64, bool want_vx, hipStream_t s, Prof *prof);
// E_x = sum_p c_p e_pair[p] (fixed order), an optional copy of e_pair and
// the optional exchange-matrix diagonal -sum_j e_ij of each target.
hipError_t run_energy(const double *epair, long long npairs, int symmetric, int N, int i0, int Ni, double *ex,
                      double *e_out, double *e_orb, hipStream_t s, Prof *prof);

// Adaptively compressed exchange (txe_ace.hip).  ace_gram: G[i][j] =
// sum_g w(g) X_i(g) Y_j(g) (part: gram_nchunks(NX, NY, ng) * NX * NY
// doubles of scratch); ace_chol_inv: L = chol(-M), T = L^-1, info;
// ace_comb: out[m][g] = scale * sum_i A[m][i] X_i(g).
int gram_nchunks(int NX, int NY, long long ng);
hipError_t ace_gram(bool x64, bool y64, const void *X, int NX, const void *Y, int NY, const Dims &D,
                    const double *const qdev[3], double *part, double *G, hipStream_t s);
hipError_t ace_chol_inv(const double *M, int N, double *L, double *T, int *info, hipStream_t s);
hipError_t ace_comb(bool x64, bool o64, const double *A, int MR, int K, const void *X, long long ng, double scale,
                    int lower, void *out, hipStream_t s);

// Device address of the allocation-free apply's scratch array on `device`
// (txe_scratch.hip; the current device must be `device`).
hipError_t scratch_address(int device, void **ptr);

// Shared bases (txe_hosvd.hip): the mode-d Gram matrix S (n_d x n_d, FP64) of
// the stacked sqrt(w)-scaled pair densities by the Gram identity (targets
// [t0, t0 + nt), sources all N orbitals), staged through T (tcap doubles,
// at least N n_d) and the per-group partial tiles Spart (ngroups * ceil(n_d /
// 16)^2 * 256 doubles); qm_dev: the weights of the other two indices (C
// order), qd_dev: q_d.  Then its eigen-decomposition S = V diag V^T (S
// overwritten, its diagonal the eigenvalues), n_d even and <= 512.
hipError_t hosvd_mode_gram(const void *psi, bool psi64, const Dims &D, int d, int N, int t0, int nt,
                           const double *qm_dev, const double *qd_dev, double *T, long long tcap, double *Spart,
                           int ngroups, double *S, hipStream_t s);
hipError_t hosvd_eigen(double *S, double *V, int n, double *trace_tmp, hipStream_t s);

// Ceiling microbenchmarks (txe_ceiling.hip): kind 0 f64, 1 f32, 2 bf16 MFMA
// in TFLOP/s; 3 HBM stream in GB/s.  Allocates, synchronises the stream.
hipError_t measure_ceiling(int kind, hipStream_t s, double *value);

// Core-kernel variant choice (register budget per precision).
int core_rows(bool f64, int nsplit, int mt);  // gamma' rows one core workgroup covers (nsplit: bf16 parts, 0 = none)

}  // namespace txe
