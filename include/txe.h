/*
 * txe.h -- Tucker-tensor Fock exchange on MI355X (gfx950): C ABI.
 *
 * Computes, for real orbitals psi_i sampled on a tensor-product grid, the
 * action of the Fock exchange operator and the exchange energy
 *
 *     (Vx psi_i)(r) = - sum_j psi_j(r) phi_ij(r),
 *     phi_ij       ~= int psi_i(r') psi_j(r') / |r - r'| dr',
 *     E_x          = -1/2 sum_{i,j} <psi_i psi_j, phi_ij>_W
 *
 * (Subramanian, Das & Gavini, arXiv 2401.04189: eq. `ExchangeOperator` and the
 * exact-exchange term of the functional S in section "Preliminaries"; the
 * convolution of eq. `conv` and the Hadamard sum of eq. `hadam` in section
 * "Overview of the algorithm").  The convolution is evaluated the paper's way
 * (section "Convolution operation"): each pair density psi_i psi_j is
 * projected onto rank-r per-mode Tucker bases (eq. `TuckerDecompField`, here
 * with bases U_d shared by every pair), 1/r is a sum of K separable Gaussians
 * (eq. `gauss`), so the 3-D convolution is a weighted sum of tensor products
 * of 1-D convolution matrices (eq. `final`), built once from the 1-D
 * finite-element mesh (eqs. `quadVal`, `discInteg`).  The library evaluates
 * the kernel sum in the Tucker core space and back-projects:
 *
 *     G_ij   = (psi_i psi_j) x0 V0^T x1 V1^T x2 V2^T,     V_d = diag(q_d) U_d
 *     Phi_ij = sum_k w_k G_ij x0 Chat_k^0 x1 Chat_k^1 x2 Chat_k^2,
 *              Chat_k^d = V_d^T C_k^d U_d
 *     phi_ij = Phi_ij x0 U0 x1 U1 x2 U2,    e_ij = <G_ij, Phi_ij>_F
 *
 * with C_k^d[a,b] = int exp(-alpha_k (x_a - x')^2) N_b(x') dx' for the
 * linear hat functions N_b of the 1-D mesh (every node has a full hat).
 *
 * Conventions
 *   - Grid arrays are C-contiguous (n0, n1, n2): mode 0 is the slowest axis.
 *     Orbital arrays are (N, n0, n1, n2), orbital-major ("band" layout: every
 *     orbital is contiguous), as the paper's structured-mesh storage.
 *   - All pointers marked "device" must be device memory (hipMalloc or a torch
 *     CUDA tensor) on the context's device; "host" pointers are ordinary host
 *     memory.  The caller owns every buffer it passes.
 *   - Every function validates all of its arguments on the host before it
 *     enqueues anything.  On any error nothing is enqueued, no output is
 *     touched, and a status other than TXE_OK is returned; txe_last_error()
 *     then describes the failure (thread-local text, valid until the next
 *     call on the same thread).
 *   - Device work is asynchronous on the context's stream; the host never
 *     waits inside txe_apply.  Same inputs, same plan => bitwise-identical
 *     outputs (no atomics; every reduction has a fixed order).
 */
#ifndef TXE_H
#define TXE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TXE_ABI_VERSION 4

typedef enum {
  TXE_OK = 0,
  TXE_ERR_ARG = 1,          /* bad pointer, value or flag                                   */
  TXE_ERR_SHAPE = 2,        /* inconsistent sizes                                           */
  TXE_ERR_NOMEM = 3,        /* device allocation failed or the workspace limit is exceeded  */
  TXE_ERR_DEVICE = 4,       /* a HIP call failed (sticky on the context)                    */
  TXE_ERR_UNSUPPORTED = 5,  /* valid request that the library does not implement            */
  TXE_ERR_STATE = 6         /* call not allowed in the current state (e.g. would allocate   */
                            /* while the stream is being captured)                          */
} txe_status;

/* Arithmetic of the mode products and kernel sums.  The 1-D convolution
 * matrices and Chat_k^d are always built in FP64 and then rounded or split;
 * the E_x reduction is always FP64.  In the split-bf16 forms every operand x
 * of the two chained contractions of the core-space kernel sum is taken as
 * bf16 parts p0 + p1 (+ p2) and a product keeps the terms p_i q_j with
 * i + j < parts (bf16 MFMA, FP32 accumulation); the projections, the
 * back-projection and the term accumulation run in FP32 MFMA. */
typedef enum {
  TXE_COMPUTE_F64 = 0,      /* FP64 MFMA                                                    */
  TXE_COMPUTE_F32 = 1,      /* FP32 MFMA, FP32 accumulation                                 */
  TXE_COMPUTE_BF16X3 = 2,   /* bf16 hi+lo split operands, 3 products, FP32 accumulation     */
  TXE_COMPUTE_BF16X6 = 3    /* bf16 three-part split operands, 6 products                   */
} txe_compute;

typedef enum { TXE_DTYPE_F64 = 0, TXE_DTYPE_F32 = 1 } txe_dtype;

typedef struct txe_context txe_context;
typedef struct txe_system txe_system;
typedef struct txe_graph txe_graph;

/* One exchange problem's fixed data (grid, bases, kernel).  All host arrays. */
typedef struct {
  int32_t n[3];             /* grid points per mode, each a multiple of 4, 4 <= n <= 512    */
  const double *x[3];       /* host: n[d] 1-D nodes, uniformly spaced, strictly increasing  */
  const double *q[3];       /* host: n[d] 1-D quadrature weights (> 0)                      */
  int32_t r[3];             /* Tucker rank per mode, 1 <= r[d] <= min(n[d], 80)             */
  const double *U[3];       /* host: n[d] x r[d], row-major; must satisfy                   */
                            /*       U^T diag(q) U = I to 1e-10 (checked)                   */
  int32_t K;                /* number of Gaussian terms, 1 <= K <= 256                      */
  const double *w;          /* host: K weights w_k (finite)                                 */
  const double *alpha;      /* host: K exponents alpha_k >= 0 (finite)                      */
  const double *C[3];       /* optional host: K x n[d] x n[d] row-major 1-D convolution     */
                            /* matrices C_k^d[a][b] of mode d (e.g. of another element      */
                            /* order or a non-uniform mesh, eq. `discInteg`); NULL = the    */
                            /* built-in linear-FE closed form, which needs uniform nodes.   */
                            /* With C[d] given, x[d] need only be strictly increasing.      */
} txe_system_desc;

/* Arguments of one apply. */
typedef struct {
  int32_t compute;          /* txe_compute                                                  */
  int32_t dtype;            /* txe_dtype of psi and vxpsi (F64 compute requires F64)        */
  int32_t N;                /* number of orbitals in psi                                    */
  const void *psi;          /* device: N x n0 x n1 x n2                                     */
  int32_t symmetric;        /* 1: all N(N+1)/2 unique pairs; targets = all N orbitals       */
                            /*    (requires i0 = 0 and Ni = N)                              */
                            /* 0: block mode, targets [i0, i0+Ni) against all N sources     */
  int32_t i0, Ni;           /* target block                                                 */
  void *vxpsi;              /* device: Ni x n0 x n1 x n2, overwritten; NULL = energy only   */
  const double *out_scale;  /* device scalar s or NULL (s = 1): vxpsi = s * Vx psi          */
  int32_t out_weighted;     /* 1: vxpsi additionally multiplied by w(r) = q0 q1 q2          */
  double *ex;               /* device: one FP64, overwritten with E_x; NULL = skip          */
  double *e_pairs;          /* device: per-pair energies e_ij (FP64) or NULL.  Symmetric:   */
                            /* N(N+1)/2 entries, pair (i<=j) at i*N - i(i-1)/2 + (j-i);     */
                            /* block: Ni*N entries, pair (i0+t, j) at t*N + j               */
  double *e_orb;            /* device: Ni FP64 entries or NULL: the exchange-matrix         */
                            /* diagonal <psi_i, Vx psi_i>_W = -sum_j e_ij of each target    */
                            /* (entry t: orbital i0+t, or t in symmetric mode), summed in   */
                            /* FP64 over j ascending.  ex, e_pairs and e_orb must be 8-byte */
                            /* aligned and overlap neither each other, psi nor vxpsi.       */
  int32_t pair_bases;       /* 0: the system's bases U_d for every pair.  1: each pair's    */
                            /* own bases, the sequentially truncated HOSVD of its density   */
                            /* (modes 0, 1, 2 in turn, ranks r[d] of the system, in the W   */
                            /* inner product; eq. `TuckerDecompField` with factors of each  */
                            /* pair), its own Chat_k^d = V_ij,d^T C_k^d U_ij,d and its own  */
                            /* back-projection.  Requires FP64 compute and n[d] <= 96       */
                            /* (TXE_ERR_UNSUPPORTED otherwise).                             */
  int32_t form;             /* TXE_FORM_CORE (0): phi_ij = P C P rho_ij, the kernel sum in   */
                            /* the Tucker core, then back-projected (eqs. `gauss`, `final`   */
                            /* evaluated in core space).  TXE_FORM_COLLOCATION (1): the 1-D  */
                            /* convolutions evaluated at every node and the 3-D field        */
                            /* reconstructed, phi_ij = sum_k w_k G_ij x_d (C_k^d U_d), with  */
                            /* e_ij = <rho_ij, phi_ij>_W on the grid (section "Convolution   */
                            /* operation", eqs. `quadVal`, `discInteg`, `final`).  The       */
                            /* collocation form needs FP64 compute and shared bases          */
                            /* (TXE_ERR_UNSUPPORTED otherwise).                              */
} txe_apply_args;

enum { TXE_FORM_CORE = 0, TXE_FORM_COLLOCATION = 1 };

/* ABI version (TXE_ABI_VERSION). */
int32_t txe_abi_version(void);

/* Static text for a status code. */
const char *txe_status_string(int32_t status);

/* Detail of the last failure on this thread ("" when none). */
const char *txe_last_error(void);

/* 1-D convolution matrix of one Gaussian term on a uniform linear-FE mesh,
 * C[a*n + b] = int exp(-alpha (x_a - x')^2) N_b(x') dx' (paper eqs. `quadVal`,
 * `discInteg`, with the node sum evaluated in closed form through erf /
 * erfc / expm1).  Host only: needs no GPU.  x: host, n nodes; C_out: host,
 * n*n doubles. */
txe_status txe_conv_matrix_1d(int32_t n, const double *x, double alpha, double *C_out);

/* Context: one device and one HIP stream (hipStream_t, may be NULL for the
 * default stream).  The context owns a reusable device workspace. */
txe_status txe_context_create(int32_t device, void *hip_stream, txe_context **out);
txe_status txe_context_destroy(txe_context *ctx);
/* Change the stream later work is enqueued on.  When the new stream differs
 * from the old one (and neither is being captured), the new stream first
 * waits for the work already enqueued on the old one, so consecutive calls on
 * one context stay ordered on its single workspace. */
txe_status txe_context_set_stream(txe_context *ctx, void *hip_stream);
/* Diagnostics: how many txe_context_set_stream calls so far ordered the new
 * stream after the old one with an event (host int64 *count). */
txe_status txe_context_stream_changes(txe_context *ctx, int64_t *count);
/* Grow the workspace to at least `bytes` now (so that later applies allocate
 * nothing).  A limit for tests: env TXE_TEST_MAX_WORKSPACE (bytes). */
txe_status txe_workspace_reserve(txe_context *ctx, size_t bytes);

/* Per-kernel timing.  When enabled (on = 1), every kernel launch of
 * txe_apply is bracketed by HIP events recorded on the context stream; the
 * counters restart at each txe_profile_enable call.  Not allowed while the
 * stream is being captured (TXE_ERR_STATE).  Kernel ids:
 *   0 proj12 (pair density, mode-2 and mode-1 projection)
 *   1 proj3  (mode-0 projection)
 *   2 core   (core-space Gaussian kernel sum, pair energies, first back-projection)
 *   3 epair  (pair-energy partial sums)
 *   4 back   (back-projection, product with psi_j, sum over sources)
 *   5 energy (E_x reduction) */
txe_status txe_profile_enable(txe_context *ctx, int32_t on);
/* Waits for the recorded launches, then returns the summed duration (ms)
 * and the number of launches of one kernel since profiling was enabled. */
txe_status txe_profile_read(txe_context *ctx, int32_t kernel, double *total_ms, int64_t *launches);
/* Static name of a kernel id ("" when out of range). */
const char *txe_kernel_name(int32_t kernel);

/* System: validates the description (U orthonormality included), builds the
 * FP64 tables on the host -- the 1-D convolution matrices C_k^d of the
 * Gaussian terms (eqs. `quadVal`, `discInteg` with linear elements, or the
 * caller's C), V_d = diag(q_d) U_d and Chat_k^d = V_d^T C_k^d U_d (the 1-D
 * operators of eq. `final` restricted to the bases of eq. `TuckerDecompField`)
 * -- rounds them to every compute precision and uploads them.  Copies all
 * host arrays; keeps no caller pointer.  Synchronises the context stream once
 * (upload).  Errors: TXE_ERR_SHAPE / _ARG on the description, TXE_ERR_DEVICE
 * when an upload fails (nothing is kept). */
txe_status txe_system_create(txe_context *ctx, const txe_system_desc *desc, txe_system **out);
txe_status txe_system_destroy(txe_system *sys);

/* FP64 copies of the setup tables of one mode (tests): C_out (host, K*n*n,
 * may be NULL) and Chat_out (host, K*r*r, row-major Chat_k[p][s], may be
 * NULL). */
txe_status txe_system_conv(const txe_system *sys, int32_t mode, double *C_out, double *Chat_out);

/* Order-p Lagrange finite elements on a 1-D mesh of cells (section
 * "Creation of Structured FE basis": the nodes of a cell are its
 * Gauss-Lobatto-Legendre points; the 3-D basis is the tensor product of the
 * 1-D Lagrange polynomials).  Host only, no device work; usable without a GPU.
 *   edges: host, ncells + 1 strictly increasing finite values (the cell ends);
 *   p: element order, 1 <= p <= 10.
 * The two end nodes of the domain are held at zero and are not unknowns, so a
 * mesh has n = ncells * p - 1 unknowns (the library's grids need n a multiple
 * of 4).  txe_fe_mesh_1d writes their positions x (host, n) and nodal
 * quadrature weights q (host, n: GLL weight times half the cell length,
 * summed over the cells a node belongs to); either may be NULL.
 * txe_fe_conv_matrices writes, for K Gaussian exponents alpha (host, K, finite,
 * >= 0), C (host, K*n*n, row-major per term) with
 * C_k[a][b] = int exp(-alpha_k (x_a - t)^2) N_b(t) dt (eqs. `quadVal`,
 * `discInteg`), the matrices txe_system_desc.C takes.  Errors: TXE_ERR_ARG
 * (null or non-finite input, edges not increasing), TXE_ERR_SHAPE (ncells,
 * p or K out of range); nothing is written then. */
txe_status txe_fe_mesh_1d(const double *edges, int32_t ncells, int32_t p, double *x, double *q);
txe_status txe_fe_conv_matrices(const double *edges, int32_t ncells, int32_t p, const double *alpha, int32_t K,
                                double *C);

/* Bases shared by all pairs (eq. `TuckerDecompField` with one set of
 * factors for every pair): per mode d the leading r[d] left singular vectors
 * of the mode-d unfolding of all pair densities psi_i psi_j (i over the
 * targets [i0, i0 + Ni), j over all N orbitals) in the W inner product -- a
 * higher-order SVD of the stacked pair densities, computed on the device
 * without forming any pair density: the Gram matrix of each unfolding from
 * the orbitals' own products (sum over pairs factorised over i and j, FP64
 * MFMA), then its eigenvectors by cyclic Jacobi rotations.
 *   n: the grid extents (multiples of 4 in [4, 512]); q: host, the 1-D
 *   weights per mode (finite, > 0); psi: device, N x n0 x n1 x n2 orbitals,
 *   dtype TXE_DTYPE_F64 or _F32; r: the ranks, 1 <= r[d] <= n[d].
 *   U_out[d]: host, n[d] x r[d] row-major, the q-orthonormal bases
 *   (U^T diag(q) U = I), columns by decreasing singular value, each signed so
 *   that its largest-magnitude entry is positive.  sv_out (may be NULL, as
 *   may each sv_out[d]): host, n[d] singular values per mode, descending.
 * Setup call: allocates its device workspace for the call's duration (up to
 * ~0.5 GiB of staging), runs on the context stream and synchronises it.
 * Errors: TXE_ERR_ARG / _SHAPE (nothing run), TXE_ERR_NOMEM, TXE_ERR_DEVICE. */
txe_status txe_hosvd_bases(txe_context *ctx, const int32_t n[3], const double *const q[3], const void *psi,
                           int32_t dtype, int32_t N, int32_t i0, int32_t Ni, const int32_t r[3],
                           double *const U_out[3], double *const sv_out[3]);

/* Workspace bytes one apply with these arguments needs. */
txe_status txe_workspace_query(txe_context *ctx, const txe_system *sys, const txe_apply_args *args,
                               size_t *bytes);

/* One exchange apply: Vx psi for the targets (eq. `ExchangeOperator` with the
 * Hadamard sum of eq. `hadam`), E_x (exact-exchange term of S, section
 * "Preliminaries"), the pair energies and the exchange-matrix diagonal, each
 * optional, through the Tucker-core evaluation of section "Convolution
 * operation" (eqs. `TuckerDecompField`, `gauss`, `final`).  Validates every
 * argument first (TXE_ERR_ARG / _SHAPE, nothing enqueued), grows the context
 * workspace when needed (TXE_ERR_NOMEM past the limit, TXE_ERR_STATE if that
 * would happen while the stream is captured), then enqueues the kernels on
 * the context stream without waiting. */
txe_status txe_apply(txe_context *ctx, const txe_system *sys, const txe_apply_args *args);

/* Bytes of the per-GPU device array txe_apply_noalloc works in. */
#define TXE_NOALLOC_SCRATCH_BYTES ((size_t)512 << 20)

/* Allocation-free apply, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The same arguments, outputs and validation as txe_apply, but
 * the workspace is a file-scope device array of TXE_NOALLOC_SCRATCH_BYTES per
 * GPU, held from context creation (where its address is looked up, once per
 * device) until the process ends, instead of the context's workspace; the
 * apply is planned in pair chunks that fit it.  The reduced-precision forms
 * read FP64 orbitals directly when their FP32 copy would not fit beside the
 * chunk workspace (the pair densities are then rounded from FP64), so their
 * results can differ from txe_apply's in the last bits; FP64 results are
 * bitwise those of txe_apply.  Calls no hipMalloc / hipFree and records no
 * timing events.  Errors: as txe_apply, plus TXE_ERR_NOMEM when one pair's
 * workspace exceeds the array and TXE_ERR_DEVICE when the array's address
 * could not be obtained on this device.  Every call on one GPU shares that
 * GPU's array and leaves its contents behind (nothing in it needs to start
 * at zero): calls that overlap on one GPU (other streams or contexts) race on
 * it, so the caller must order them. */
txe_status txe_apply_noalloc(txe_context *ctx, const txe_system *sys, const txe_apply_args *args);

/* Batched apply: S independent problems (each its own system, orbitals and
 * outputs, e.g. the uneven molecules of a screening run) enqueued as one
 * unit.  The systems are spread over `lanes` concurrent HIP streams
 * (1..16, default priority) that fork from and join back into the context
 * stream, longest estimated work first on the least-loaded lane; each lane
 * has its own slice of the context workspace.  Every problem runs exactly
 * the kernels and launch shapes txe_apply would run for it, so its outputs
 * are bitwise identical to a separate txe_apply.  args: host array of S;
 * systems: host array of S.  Outputs of different problems must not overlap
 * (TXE_ERR_ARG).  1 <= S <= 4096. */
txe_status txe_apply_batched(txe_context *ctx, int32_t S, const txe_system *const *systems,
                             const txe_apply_args *args, int32_t lanes);

/* Graph of a batched apply: captured once (on a private stream of the
 * context, with its own workspace allocated before the capture) and then
 * replayed on the context's current stream by txe_graph_launch with a
 * single host call.  The graph keeps the device pointers of `args`: the
 * orbitals and outputs, and the systems, must stay alive until
 * txe_graph_destroy; a replay reads the orbitals' current contents.  The
 * graph holds no memset nodes.  Replays of one graph on one stream are
 * ordered; replays of one graph overlapping on different streams race on
 * its workspace. */
txe_status txe_graph_capture_batched(txe_context *ctx, int32_t S, const txe_system *const *systems,
                                     const txe_apply_args *args, int32_t lanes, txe_graph **out);
txe_status txe_graph_launch(txe_graph *graph);
/* Waits for the context stream, then frees the graph and its workspace. */
txe_status txe_graph_destroy(txe_graph *graph);

/* Tuner.  Launch shapes of one problem: knobs[0] gamma' splits of the core
 * kernel as a multiple (1, 2, 4) of the fewest that fit its accumulator
 * registers; knobs[1] gamma tiles per wavefront of the projection kernel
 * (1..3; 4 = all of them, in a form compiled for the rank tile count);
 * knobs[2] c tiles per wavefront of the back-projection kernel (1, 2;
 * 0 = chosen by size); knobs[3] workgroups of the persistent projection and
 * back-projection kernels; knobs[4] form of the back-projection kernel (1
 * streaming, 2 batched loads, 3 each source's slab staged in LDS per
 * workgroup; 0 = default: 3 where its LDS leaves room for two workgroups per
 * CU in FP32 compute, or fits one (160 KiB) in FP64, else 2; 3 falls back
 * to 2 where it does not fit).  Results do not depend on
 * knobs[1..4]; knobs[0] changes the summation order of the pair energies
 * only.
 *
 * txe_tune times txe_apply with these args (each candidate: one warm-up and
 * `reps` timed applies, HIP events on the context stream; the host waits) in
 * coordinate descent from the defaults {1, 4, 0, 2048, 0}, at most two sweeps,
 * and keeps the fastest in the context under a key made of the device
 * architecture, grid, ranks, K, N, Ni, compute, mode and whether Vx psi is
 * wanted.  Later applies, batches and graphs with the same key use it.  The
 * outputs of args are overwritten.  best_ms (host, may be NULL): the mean
 * time of the chosen shape.  Not allowed during capture (TXE_ERR_STATE). */
txe_status txe_tune(txe_context *ctx, const txe_system *sys, const txe_apply_args *args, int32_t reps,
                    double *best_ms);
/* The launch shape an apply with these args would use (host knobs[5]);
 * *tuned (host, may be NULL) = 1 if it came from the tuner or a cache. */
txe_status txe_plan_get(txe_context *ctx, const txe_system *sys, const txe_apply_args *args, int32_t knobs[5],
                        int32_t *tuned);
/* The context's tuned shapes as a JSON object {key: {"ngs_mul", "proj_gt",
 * "back_ncg", "grid_cap", "back_form"}}, one entry per line (overwrites
 * `path`).  On load a missing "back_form" means 0. */
txe_status txe_tune_save(txe_context *ctx, const char *path);
/* Merges a file written by txe_tune_save into the context; *loaded (host,
 * may be NULL) = entries read.  A malformed entry or an out-of-range shape
 * fails the whole load (TXE_ERR_ARG) and changes nothing. */
txe_status txe_tune_load(txe_context *ctx, const char *path, int32_t *loaded);

/* Adaptively compressed exchange (section "ACE implementation"), the
 * consumer of the exchange action.  From N orbitals psi and their actions
 * W = Vx psi (device, N x n0 x n1 x n2, dtype; e.g. the vxpsi of a symmetric
 * txe_apply over the same orbitals):
 *     M_ij = <psi_i, W_j>_W,  M = -L L^T (Cholesky),  xi_k = sum_i W_i (L^-1)_ki
 * (eq. `eta`).  xi: device, N x n0 x n1 x n2 FP64, overwritten.  M_out,
 * L_out: optional device N x N FP64 (row-major; L lower triangular with
 * zeros above).  info: optional device int32, set to 0, or to j + 1 when the
 * pivot of column j is not positive (M not negative definite); the outputs
 * are then undefined.  All arithmetic FP64 (MFMA for the grid contractions,
 * one workgroup for the Cholesky factor and its inverse).  Asynchronous on
 * the context stream; uses the context workspace.  1 <= N <= 2048. */
txe_status txe_ace_build(txe_context *ctx, const txe_system *sys, int32_t N, int32_t dtype, const void *psi,
                         const void *W, double *xi, double *M_out, double *L_out, int32_t *info);
/* V_ACE applied to Nphi trial functions: out_j = -sum_k xi_k <xi_k, phi_j>_W
 * (the operator equals Vx on the orbitals it was built from).  xi: device
 * FP64 from txe_ace_build; phi, out: device Nphi x n0 x n1 x n2 in dtype
 * (out overwritten, must not overlap an input).  1 <= Nphi <= 65536. */
txe_status txe_ace_apply(txe_context *ctx, const txe_system *sys, int32_t N, const double *xi, int32_t Nphi,
                         int32_t dtype, const void *phi, void *out);

/* Measured ceilings of this device (the denominators a roofline can use
 * next to the published peaks): kind 0 = FP64 MFMA 16x16x4, 1 = FP32 MFMA
 * 16x16x4, 2 = bf16 MFMA 16x16x32 (TFLOP/s, 8 independent accumulator
 * chains per wavefront, 4 workgroups of 256 per CU); 3 = HBM stream
 * dst = 2*src over 512 MiB (GB/s, bytes read + written).  *value (host)
 * receives the rate.  Allocates (kind 3: 1 GiB, freed before return) and
 * waits for the context stream. */
txe_status txe_measure_ceiling(txe_context *ctx, int32_t kind, double *value);

#ifdef __cplusplus
}
#endif

#endif /* TXE_H */
