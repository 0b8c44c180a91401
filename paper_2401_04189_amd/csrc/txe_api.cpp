// C ABI of the Tucker-tensor exchange library: argument validation, FP64
// setup tables, per-precision device tables, workspace and chunk planning.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/txe.h"
#include "txe_internal.h"

using namespace txe;

// ------------------------------------------------------------------------------------
// error text
// ------------------------------------------------------------------------------------
static thread_local std::string g_last_error;

static txe_status fail(txe_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

static txe_status ok() {
  g_last_error.clear();
  return TXE_OK;
}

// Launch-shape choices of one apply (the tuner's search space).
struct Knobs {
  int ngs_mul = 1;     // gamma' splits of the core kernel, as a multiple of the fewest that fit the registers
  int proj_gt = 4;     // gamma tiles per wavefront in proj12 (1, 2, 3; 4 = all, compile-time form)
  int back_ncg = 0;    // c tiles per wavefront in back (1, 2; 0 = by size)
  int grid_cap = 2048; // workgroups of the persistent proj12 / back kernels
  int back_form = 0;   // back kernel form (1 streaming, 2 batched, 3 LDS-staged; 0 = default by size)
};

struct txe_context {
  int device = 0;
  hipStream_t stream = nullptr;
  void *ws = nullptr;
  size_t ws_bytes = 0;
  bool sticky = false;
  std::string sticky_msg;
  Prof prof;
  std::string arch;                      // gcnArchName of the device
  std::map<std::string, Knobs> plans;    // tuned launch shapes by problem key
  std::vector<hipStream_t> lanes;        // concurrent streams of batched applies
  std::vector<hipEvent_t> lane_done;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;             // private stream for graph capture
  hipEvent_t handoff = nullptr;          // orders a new stream after the old one (set_stream)
  long long handoffs = 0;                // stream changes that were ordered by that event
};

template <typename T>
struct DevTables {
  Tables<T> t{};
  std::vector<void *> owned;
};

struct DevBf {
  BfTables t{};
  std::vector<void *> owned;
};

struct txe_system {
  txe_context *ctx = nullptr;
  int device = 0;
  Dims D{};
  int n[3], r[3], K;
  std::vector<double> x[3], q[3], U[3], w, alpha;
  std::vector<double> C[3];      // K x n x n
  std::vector<double> Chat[3];   // K x r x r
  DevTables<double> t64;
  DevTables<float> t32;
  DevBf tbf;
  double *qdev[3] = {nullptr, nullptr, nullptr};
  // per-pair bases: D C_k^d D^-1 (D = diag(sqrt(q_d)), [K][n][n] per mode) and w_k
  double *csdev[3] = {nullptr, nullptr, nullptr};
  double *wdev = nullptr;
  // collocation form: A_k^d = C_k^d U_d ([K][n][r] per mode)
  double *acol[3] = {nullptr, nullptr, nullptr};
  double *acol0s = nullptr;  // the grouped, weighted A_k^0 of the collocation form (see CollocArgs)
};

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(TXE_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// ------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------
extern "C" int32_t txe_abi_version(void) { return TXE_ABI_VERSION; }

extern "C" const char *txe_status_string(int32_t st) {
  switch (st) {
    case TXE_OK: return "ok";
    case TXE_ERR_ARG: return "invalid argument";
    case TXE_ERR_SHAPE: return "inconsistent shape";
    case TXE_ERR_NOMEM: return "out of device memory or workspace limit";
    case TXE_ERR_DEVICE: return "device error";
    case TXE_ERR_UNSUPPORTED: return "unsupported";
    case TXE_ERR_STATE: return "invalid state";
  }
  return "unknown status";
}

extern "C" const char *txe_last_error(void) { return g_last_error.c_str(); }

static bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

static txe_status check_grid_1d(int n, const double *x, const char *what, bool uniform = true) {
  if (!x) return fail(TXE_ERR_ARG, "%s: null node array", what);
  if (!finite_all(x, n)) return fail(TXE_ERR_ARG, "%s: non-finite node", what);
  const double h = x[1] - x[0];
  if (!(h > 0)) return fail(TXE_ERR_ARG, "%s: nodes must be strictly increasing", what);
  for (int i = 1; i < n; ++i) {
    const double hi = x[i] - x[i - 1];
    if (!(hi > 0)) return fail(TXE_ERR_ARG, "%s: nodes must be strictly increasing", what);
    if (uniform && std::fabs(hi - h) > 1e-9 * std::fabs(h))
      return fail(TXE_ERR_UNSUPPORTED, "%s: nodes must be uniformly spaced (or give C)", what);
  }
  return TXE_OK;
}

extern "C" txe_status txe_conv_matrix_1d(int32_t n, const double *x, double alpha, double *C_out) {
  if (n < 2 || n > 4096) return fail(TXE_ERR_SHAPE, "n = %d out of range [2, 4096]", n);
  if (!C_out) return fail(TXE_ERR_ARG, "C_out is null");
  txe_status st = check_grid_1d(n, x, "x");
  if (st != TXE_OK) return st;
  if (!std::isfinite(alpha) || alpha < 0) return fail(TXE_ERR_ARG, "alpha must be finite and >= 0");
  conv_matrix_1d(n, x, alpha, C_out);
  return ok();
}

// ------------------------------------------------------------------------------------
// context
// ------------------------------------------------------------------------------------
extern "C" txe_status txe_context_create(int32_t device, void *hip_stream, txe_context **out) {
  if (!out) return fail(TXE_ERR_ARG, "out is null");
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(TXE_ERR_ARG, "device %d not in [0, %d)", device, ndev);
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  // set-up of the allocation-free apply's scratch array on this device (its
  // address is looked up once per device and kept; a failure is reported by
  // txe_apply_noalloc)
  HIP_TRY(hipSetDevice(device));
  void *scr = nullptr;
  (void)scratch_address(device, &scr);
  auto *c = new txe_context();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->arch = prop.gcnArchName;
  const size_t colon = c->arch.find(':');
  if (colon != std::string::npos) c->arch.resize(colon);
  *out = c;
  return ok();
}

extern "C" txe_status txe_context_destroy(txe_context *ctx) {
  if (!ctx) return fail(TXE_ERR_ARG, "ctx is null");
  hipSetDevice(ctx->device);
  if (ctx->ws) hipFree(ctx->ws);
  for (hipStream_t l : ctx->lanes) hipStreamDestroy(l);
  for (hipEvent_t e : ctx->lane_done) hipEventDestroy(e);
  if (ctx->fork) hipEventDestroy(ctx->fork);
  if (ctx->cap) hipStreamDestroy(ctx->cap);
  if (ctx->handoff) hipEventDestroy(ctx->handoff);
  delete ctx;
  return ok();
}

extern "C" txe_status txe_profile_enable(txe_context *ctx, int32_t on) {
  if (!ctx) return fail(TXE_ERR_ARG, "ctx is null");
  if (on != 0 && on != 1) return fail(TXE_ERR_ARG, "on must be 0 or 1");
  if (on) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(ctx->stream, &cs));
    if (cs != hipStreamCaptureStatusNone) return fail(TXE_ERR_STATE, "cannot profile while the stream is captured");
  }
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->prof.reset();
  ctx->prof.on = on != 0;
  return ok();
}

extern "C" txe_status txe_profile_read(txe_context *ctx, int32_t kernel, double *total_ms, int64_t *launches) {
  if (!ctx || !total_ms || !launches) return fail(TXE_ERR_ARG, "null argument");
  if (kernel < 0 || kernel >= K_COUNT) return fail(TXE_ERR_ARG, "kernel id %d not in [0, %d)", kernel, (int)K_COUNT);
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->prof.collect();
  *total_ms = ctx->prof.total_ms[kernel];
  *launches = ctx->prof.count[kernel];
  return ok();
}

extern "C" const char *txe_kernel_name(int32_t kernel) {
  static const char *names[K_COUNT] = {"proj12", "proj3", "core", "epair", "back", "energy"};
  return (kernel >= 0 && kernel < K_COUNT) ? names[kernel] : "";
}

extern "C" txe_status txe_context_set_stream(txe_context *ctx, void *hip_stream) {
  if (!ctx) return fail(TXE_ERR_ARG, "ctx is null");
  const hipStream_t next = (hipStream_t)hip_stream;
  if (next == ctx->stream) return ok();
  // Work already enqueued on the old stream uses the context's workspace:
  // the new stream waits for it (an event recorded on the old stream), so
  // applies issued from two streams never overlap on that workspace.  A
  // stream under capture neither records nor waits here (its own capture
  // orders it; the caller joins captures explicitly).
  hipStreamCaptureStatus c0 = hipStreamCaptureStatusNone, c1 = hipStreamCaptureStatusNone;
  HIP_TRY(hipSetDevice(ctx->device));
  HIP_TRY(hipStreamIsCapturing(ctx->stream, &c0));
  HIP_TRY(hipStreamIsCapturing(next, &c1));
  if (c0 == hipStreamCaptureStatusNone && c1 == hipStreamCaptureStatusNone) {
    if (!ctx->handoff) HIP_TRY(hipEventCreateWithFlags(&ctx->handoff, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(ctx->handoff, ctx->stream));
    HIP_TRY(hipStreamWaitEvent(next, ctx->handoff, 0));
    ++ctx->handoffs;
  }
  ctx->stream = next;
  return ok();
}

extern "C" txe_status txe_context_stream_changes(txe_context *ctx, int64_t *count) {
  if (!ctx || !count) return fail(TXE_ERR_ARG, "null argument");
  *count = ctx->handoffs;
  return ok();
}

static size_t workspace_limit() {
  const char *e = getenv("TXE_TEST_MAX_WORKSPACE");
  if (e && *e) return (size_t)strtoull(e, nullptr, 10);
  return (size_t)96 << 30;  // 96 GiB of the 288 GiB HBM
}

static txe_status ensure_workspace(txe_context *ctx, size_t bytes) {
  if (bytes <= ctx->ws_bytes) return TXE_OK;
  if (bytes > workspace_limit())
    return fail(TXE_ERR_NOMEM, "workspace of %zu bytes exceeds the limit of %zu bytes", bytes, workspace_limit());
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(ctx->stream, &cs));
  if (cs != hipStreamCaptureStatusNone)
    return fail(TXE_ERR_STATE, "workspace must grow to %zu bytes while the stream is captured; call "
                               "txe_workspace_reserve first", bytes);
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->ws) {
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    HIP_TRY(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(TXE_ERR_NOMEM, "hipMalloc of %zu bytes failed", bytes);
  }
  ctx->ws = p;
  ctx->ws_bytes = bytes;
  return TXE_OK;
}

extern "C" txe_status txe_workspace_reserve(txe_context *ctx, size_t bytes) {
  if (!ctx) return fail(TXE_ERR_ARG, "ctx is null");
  txe_status st = ensure_workspace(ctx, bytes);
  return st == TXE_OK ? ok() : st;
}

// ------------------------------------------------------------------------------------
// system
// ------------------------------------------------------------------------------------
template <typename T>
static txe_status upload(DevTables<T> &dt, const std::vector<double> &src, T **dst, hipStream_t s) {
  std::vector<T> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (T)src[i];
  void *p = nullptr;
  HIP_TRY(hipMalloc(&p, std::max<size_t>(tmp.size(), 1) * sizeof(T)));
  dt.owned.push_back(p);
  HIP_TRY(hipMemcpyAsync(p, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  *dst = (T *)p;
  return TXE_OK;
}

// Build every table in FP64 with the layouts Tables<T> documents.
struct HostTables {
  std::vector<double> V2B, V1chain, V0K, C1f, C2chain, Ahat, U0chain, U2T, U1chain;
};

// Accumulator row of entry v in lane group lg of a 16x16x4 MFMA: 4*lg + v
// for f32, 4*v + lg for f64.  The chain tables follow the precision's order.
static void build_tables(const txe_system &S, HostTables &H, bool f64) {
  const Dims &D = S.D;
  auto drow = [f64](int lg, int v) { return f64 ? 4 * v + lg : 4 * lg + v; };
  auto U = [&](int d, int i, int s) -> double { return S.U[d][(size_t)i * S.r[d] + s]; };
  auto V = [&](int d, int i, int s) -> double { return S.q[d][i] * U(d, i, s); };
  auto Ch = [&](int d, int k, int p, int s) -> double { return S.Chat[d][((size_t)k * S.r[d] + p) * S.r[d] + s]; };
  // V2B[c][gamma]
  H.V2B.assign((size_t)D.nc2 * D.rp2, 0.0);
  for (int c = 0; c < D.n2; ++c)
    for (int g = 0; g < D.r2; ++g) H.V2B[(size_t)c * D.rp2 + g] = V(2, c, g);
  // V1chain[mt][mb][v][lane] = V1[b = 16mb+4lg+v][beta = 16mt+lr]
  const int nbt = D.nb1 / 16;
  H.V1chain.assign((size_t)D.MT1 * nbt * 256, 0.0);
  for (int mt = 0; mt < D.MT1; ++mt)
    for (int mb = 0; mb < nbt; ++mb)
      for (int v = 0; v < 4; ++v)
        for (int l = 0; l < 64; ++l) {
          const int beta = 16 * mt + (l & 15), b = 16 * mb + drow(l >> 4, v);
          if (beta < D.r1 && b < D.n1) H.V1chain[(((size_t)mt * nbt + mb) * 4 + v) * 64 + l] = V(1, b, beta);
        }
  // V0K[a][alpha]
  H.V0K.assign((size_t)D.n0 * D.rp0, 0.0);
  for (int a = 0; a < D.n0; ++a)
    for (int al = 0; al < D.r0; ++al) H.V0K[(size_t)a * D.rp0 + al] = V(0, a, al);
  // FP32: C1f[k][bt][kq][lane][j] = Chat1_k[beta' = 16bt+lr][beta = 16kq+4j+lg],
  // the B fragments of K = 4 steps kt = 4kq+j of the core's W chain side by
  // side; FP64: C1f[k][beta][beta'] = Chat1_k[beta'][beta]
  if (f64) {
    H.C1f.assign((size_t)D.Kp * D.rp1 * D.rp1, 0.0);
    for (int k = 0; k < D.K; ++k)
      for (int be = 0; be < D.r1; ++be)
        for (int bp = 0; bp < D.r1; ++bp) H.C1f[((size_t)k * D.rp1 + be) * D.rp1 + bp] = Ch(1, k, bp, be);
  } else {
    H.C1f.assign((size_t)D.Kp * D.MT1 * D.MT1 * 256, 0.0);
    for (int k = 0; k < D.K; ++k)
      for (int bt = 0; bt < D.MT1; ++bt)
        for (int kq = 0; kq < D.MT1; ++kq)
          for (int l = 0; l < 64; ++l)
            for (int j = 0; j < 4; ++j) {
              const int bp = 16 * bt + (l & 15), be = 16 * kq + 4 * j + (l >> 4);
              if (bp < D.r1 && be < D.r1)
                H.C1f[((((size_t)k * D.MT1 + bt) * D.MT1 + kq) * 64 + l) * 4 + j] = Ch(1, k, bp, be);
            }
  }
  // C2chain: Chat2_k[gamma' = 16mt'+lr][gamma = 16mg+4v+lg] at [k][mt'][mg][lane][v]
  // (FP32) or [k][mt'][mg][v][lane] (FP64).  In both precisions chunk v of
  // tile mg holds gamma rows 16mg+4v..+3, so chunks past the rank are all
  // zero and the core skips them (the FP32 core orders the slab's gamma rows
  // inside a tile to match)
  H.C2chain.assign((size_t)D.Kp * D.MT2 * D.MT2 * 256, 0.0);
  for (int k = 0; k < D.K; ++k)
    for (int mtp = 0; mtp < D.MT2; ++mtp)
      for (int mg = 0; mg < D.MT2; ++mg)
        for (int v = 0; v < 4; ++v)
          for (int l = 0; l < 64; ++l) {
            const int gp = 16 * mtp + (l & 15), g = 16 * mg + 4 * v + (l >> 4);
            const size_t base = (((size_t)k * D.MT2 + mtp) * D.MT2 + mg) * 256;
            if (gp < D.r2 && g < D.r2) H.C2chain[base + (f64 ? v * 64 + l : l * 4 + v)] = Ch(2, k, gp, g);
          }
  // Ahat[alpha][k][alpha'] = w_k Chat0_k[alpha'][alpha]
  H.Ahat.assign((size_t)D.r0 * D.Kp * D.rp0, 0.0);
  for (int al = 0; al < D.r0; ++al)
    for (int k = 0; k < D.K; ++k)
      for (int ap = 0; ap < D.r0; ++ap) H.Ahat[((size_t)al * D.Kp + k) * D.rp0 + ap] = S.w[k] * Ch(0, k, ap, al);
  // U0chain[ma][mt][v][lane] = U0[a = 16ma+lr][alpha' = 16mt+4lg+v]
  const int nat = D.na0 / 16;
  H.U0chain.assign((size_t)nat * D.MT0 * 256, 0.0);
  for (int ma = 0; ma < nat; ++ma)
    for (int mt = 0; mt < D.MT0; ++mt)
      for (int v = 0; v < 4; ++v)
        for (int l = 0; l < 64; ++l) {
          const int a = 16 * ma + (l & 15), ap = 16 * mt + drow(l >> 4, v);
          if (a < D.n0 && ap < D.r0) H.U0chain[(((size_t)ma * D.MT0 + mt) * 4 + v) * 64 + l] = U(0, a, ap);
        }
  // U2T[gamma][c] = U2[c][gamma]
  H.U2T.assign((size_t)D.rp2 * D.nc2, 0.0);
  for (int g = 0; g < D.r2; ++g)
    for (int c = 0; c < D.n2; ++c) H.U2T[(size_t)g * D.nc2 + c] = U(2, c, g);
  // U1chain[mb][mbeta][v][lane] = U1[b = 16mb+lr][beta = 16mbeta+4lg+v]
  H.U1chain.assign((size_t)nbt * D.MT1 * 256, 0.0);
  for (int mb = 0; mb < nbt; ++mb)
    for (int me = 0; me < D.MT1; ++me)
      for (int v = 0; v < 4; ++v)
        for (int l = 0; l < 64; ++l) {
          const int b = 16 * mb + (l & 15), be = 16 * me + drow(l >> 4, v);
          if (b < D.n1 && be < D.r1) H.U1chain[(((size_t)mb * D.MT1 + me) * 4 + v) * 64 + l] = U(1, b, be);
        }
}

// bf16 bit pattern of a double, rounded to nearest even (through float)
static unsigned short bf16_bits(double x) {
  float f = (float)x;
  unsigned u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
static double bf16_value(unsigned short b) {
  unsigned u = (unsigned)b << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}
// three bf16 parts of x: p0 = bf16(x), p1 = bf16(x - p0), p2 = bf16(x - p0 - p1)
static void split3(double x, unsigned short (&o)[3]) {
  double r = x;
  for (int sp = 0; sp < 3; ++sp) {
    o[sp] = bf16_bits(r);
    r -= bf16_value(o[sp]);
  }
}

// Split-bf16 term matrices of the core kernel (layouts in BfTables).
static void build_bf_tables(const txe_system &S, std::vector<unsigned short> &C1, std::vector<unsigned short> &C2,
                            int &nC) {
  const Dims &D = S.D;
  const int MT = D.MT1, RP = D.rp1;
  nC = (RP + 31) / 32;
  auto Ch = [&](int d, int k, int p, int q) -> double { return S.Chat[d][((size_t)k * S.r[d] + p) * S.r[d] + q]; };
  C1.assign((size_t)D.Kp * MT * 3 * nC * 512, 0);
  C2.assign((size_t)D.Kp * 3 * MT * nC * 512, 0);
  unsigned short part[3];
  for (int k = 0; k < D.K; ++k)
    for (int c = 0; c < nC; ++c)
      for (int l = 0; l < 64; ++l)
        for (int i = 0; i < 8; ++i) {
          const int kk = 8 * (l >> 4) + i;
          // B operand of the beta contraction: Chat1_k[beta' = 16 bt + n][beta = 32 c + kk]
          for (int bt = 0; bt < MT; ++bt) {
            const int bp = 16 * bt + (l & 15), be = 32 * c + kk;
            if (bp < D.r1 && be < D.r1) {
              split3(Ch(1, k, bp, be), part);
              for (int sp = 0; sp < 3; ++sp)
                C1[(((((size_t)k * MT + bt) * 3 + sp) * nC + c) * 64 + l) * 8 + i] = part[sp];
            }
          }
          // A operand of the gamma contraction: Chat2_k[gamma' = 16 mtp + m][gamma(c, kk)]
          const int g = 16 * (2 * c + (i >> 2)) + 4 * (l >> 4) + (i & 3);
          for (int mtp = 0; mtp < MT; ++mtp) {
            const int gp = 16 * mtp + (l & 15);
            if (gp < D.r2 && g < D.r2) {
              split3(Ch(2, k, gp, g), part);
              for (int sp = 0; sp < 3; ++sp)
                C2[(((((size_t)k * 3 + sp) * MT + mtp) * nC + c) * 64 + l) * 8 + i] = part[sp];
            }
          }
        }
}

template <typename T>
static txe_status upload_tables(DevTables<T> &dt, const HostTables &H, hipStream_t s) {
  txe_status st;
  if ((st = upload(dt, H.V2B, &dt.t.V2B, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.V1chain, &dt.t.V1chain, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.V0K, &dt.t.V0K, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.C1f, &dt.t.C1f, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.C2chain, &dt.t.C2chain, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.Ahat, &dt.t.Ahat, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.U0chain, &dt.t.U0chain, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.U2T, &dt.t.U2T, s)) != TXE_OK) return st;
  if ((st = upload(dt, H.U1chain, &dt.t.U1chain, s)) != TXE_OK) return st;
  return TXE_OK;
}

template <typename T>
static void free_tables(DevTables<T> &dt) {
  for (void *p : dt.owned) hipFree(p);
  dt.owned.clear();
}

extern "C" txe_status txe_system_destroy(txe_system *sys) {
  if (!sys) return fail(TXE_ERR_ARG, "sys is null");
  hipSetDevice(sys->device);
  free_tables(sys->t64);
  free_tables(sys->t32);
  for (void *p : sys->tbf.owned) hipFree(p);
  for (int d = 0; d < 3; ++d) {
    if (sys->qdev[d]) hipFree(sys->qdev[d]);
    if (sys->csdev[d]) hipFree(sys->csdev[d]);
    if (sys->acol[d]) hipFree(sys->acol[d]);
  }
  if (sys->acol0s) hipFree(sys->acol0s);
  if (sys->wdev) hipFree(sys->wdev);
  delete sys;
  return ok();
}

extern "C" txe_status txe_system_create(txe_context *ctx, const txe_system_desc *desc, txe_system **out) {
  if (!ctx || !desc || !out) return fail(TXE_ERR_ARG, "null argument");
  for (int d = 0; d < 3; ++d) {
    const int n = desc->n[d], r = desc->r[d];
    if (n < 4 || n > 512 || n % 4 != 0) return fail(TXE_ERR_SHAPE, "n[%d] = %d must be a multiple of 4 in [4, 512]", d, n);
    if (r < 1 || r > n || r > 16 * MAX_MT) return fail(TXE_ERR_SHAPE, "r[%d] = %d must be in [1, min(n, %d)]", d, r, 16 * MAX_MT);
    char what[16];
    snprintf(what, sizeof what, "x[%d]", d);
    // the built-in linear-FE builder needs uniform nodes; user matrices do not
    txe_status st = check_grid_1d(n, desc->x[d], what, desc->C[d] == nullptr);
    if (st != TXE_OK) return st;
    if (!desc->q[d] || !desc->U[d]) return fail(TXE_ERR_ARG, "q[%d] or U[%d] is null", d, d);
    if (!finite_all(desc->q[d], n)) return fail(TXE_ERR_ARG, "q[%d] has a non-finite entry", d);
    for (int i = 0; i < n; ++i)
      if (!(desc->q[d][i] > 0)) return fail(TXE_ERR_ARG, "q[%d][%d] must be > 0", d, i);
    if (!finite_all(desc->U[d], (size_t)n * r)) return fail(TXE_ERR_ARG, "U[%d] has a non-finite entry", d);
    // U^T diag(q) U = I
    double worst = 0.0;
    for (int s1 = 0; s1 < r; ++s1)
      for (int s2 = 0; s2 < r; ++s2) {
        long double acc = 0;
        for (int i = 0; i < n; ++i)
          acc += (long double)desc->q[d][i] * desc->U[d][(size_t)i * r + s1] * desc->U[d][(size_t)i * r + s2];
        worst = std::max(worst, std::fabs((double)acc - (s1 == s2 ? 1.0 : 0.0)));
      }
    if (worst > 1e-10)
      return fail(TXE_ERR_ARG, "U[%d] is not q-orthonormal (max |U^T diag(q) U - I| = %.3g)", d, worst);
  }
  if (desc->K < 1 || desc->K > 256) return fail(TXE_ERR_SHAPE, "K = %d must be in [1, 256]", desc->K);
  if (!desc->w || !desc->alpha) return fail(TXE_ERR_ARG, "w or alpha is null");
  if (!finite_all(desc->w, desc->K) || !finite_all(desc->alpha, desc->K))
    return fail(TXE_ERR_ARG, "w and alpha must be finite");
  for (int k = 0; k < desc->K; ++k)
    if (desc->alpha[k] < 0) return fail(TXE_ERR_ARG, "alpha[%d] < 0", k);
  for (int d = 0; d < 3; ++d)
    if (desc->C[d] && !finite_all(desc->C[d], (size_t)desc->K * desc->n[d] * desc->n[d]))
      return fail(TXE_ERR_ARG, "C[%d] has a non-finite entry", d);

  auto *S = new txe_system();
  S->ctx = ctx;
  S->device = ctx->device;
  S->K = desc->K;
  for (int d = 0; d < 3; ++d) {
    S->n[d] = desc->n[d];
    S->r[d] = desc->r[d];
    S->x[d].assign(desc->x[d], desc->x[d] + S->n[d]);
    S->q[d].assign(desc->q[d], desc->q[d] + S->n[d]);
    S->U[d].assign(desc->U[d], desc->U[d] + (size_t)S->n[d] * S->r[d]);
  }
  S->w.assign(desc->w, desc->w + S->K);
  S->alpha.assign(desc->alpha, desc->alpha + S->K);
  // FP64 setup: C_k^d and Chat_k^d
  for (int d = 0; d < 3; ++d) {
    const int n = S->n[d], r = S->r[d];
    S->C[d].assign((size_t)S->K * n * n, 0.0);
    S->Chat[d].assign((size_t)S->K * r * r, 0.0);
    bool reused = false;
    if (desc->C[d]) {  // caller's matrices (e.g. another element order or mesh)
      S->C[d].assign(desc->C[d], desc->C[d] + (size_t)S->K * n * n);
      reused = true;
    }
    for (int e = 0; e < d && !reused; ++e)
      if (!desc->C[e] && S->x[e] == S->x[d]) {
        S->C[d] = S->C[e];
        reused = true;
      }
    for (int k = 0; k < S->K; ++k) {
      if (!reused) conv_matrix_1d(n, S->x[d].data(), S->alpha[k], &S->C[d][(size_t)k * n * n]);
      core_matrix(n, r, S->q[d].data(), S->U[d].data(), &S->C[d][(size_t)k * n * n], &S->Chat[d][(size_t)k * r * r]);
    }
  }
  Dims &D = S->D;
  D.n0 = S->n[0]; D.n1 = S->n[1]; D.n2 = S->n[2];
  D.na0 = rup(D.n0, 16); D.nb1 = rup(D.n1, 16); D.nc2 = rup(D.n2, 16);
  D.r0 = S->r[0]; D.r1 = S->r[1]; D.r2 = S->r[2];
  // one padded core size for every mode: the core kernel's loops and strides
  // are then compile-time constants (padded rows and columns are zero)
  const int rpad = rup(std::max(D.r0, std::max(D.r1, D.r2)), 16);
  D.rp0 = rpad; D.rp1 = rpad; D.rp2 = rpad;
  D.MT0 = D.rp0 / 16; D.MT1 = D.rp1 / 16; D.MT2 = D.rp2 / 16;
  D.r1k = rup(D.r1, 4); D.r2k = rup(D.r2, 4);
  D.K = S->K; D.Kp = rup(S->K, KCHUNK);

  HostTables H64, H32;
  build_tables(*S, H64, true);
  build_tables(*S, H32, false);
  txe_status st;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete S;
    return fail(TXE_ERR_DEVICE, "hipSetDevice failed");
  }
  if ((st = upload_tables(S->t64, H64, ctx->stream)) != TXE_OK ||
      (st = upload_tables(S->t32, H32, ctx->stream)) != TXE_OK) {
    txe_system_destroy(S);
    return st;
  }
  {
    std::vector<unsigned short> C1, C2;
    int nC = 0;
    build_bf_tables(*S, C1, C2, nC);
    const std::vector<unsigned short> *src[2] = {&C1, &C2};
    for (int t = 0; t < 2; ++t) {
      void *p = nullptr;
      if (hipMalloc(&p, src[t]->size() * 2) != hipSuccess ||
          hipMemcpy(p, src[t]->data(), src[t]->size() * 2, hipMemcpyHostToDevice) != hipSuccess) {
        if (p) hipFree(p);
        txe_system_destroy(S);
        return fail(TXE_ERR_DEVICE, "upload of the bf16 tables failed");
      }
      S->tbf.owned.push_back(p);
    }
    S->tbf.t.C1 = (const unsigned short *)S->tbf.owned[0];
    S->tbf.t.C2 = (const unsigned short *)S->tbf.owned[1];
    S->tbf.t.nC = nC;
  }
  for (int d = 0; d < 3; ++d) {
    void *p = nullptr;
    if (hipMalloc(&p, S->n[d] * sizeof(double)) != hipSuccess ||
        hipMemcpy(p, S->q[d].data(), S->n[d] * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      if (p) hipFree(p);
      txe_system_destroy(S);
      return fail(TXE_ERR_DEVICE, "upload of q failed");
    }
    S->qdev[d] = (double *)p;
  }
  // tables of the per-pair-bases mode (grids it supports, n <= 96): D C_k^d D^-1 per mode, and w
  const bool pb_grid = std::max(S->n[0], std::max(S->n[1], S->n[2])) <= PB_MAX_N;
  for (int d = 0; d < 3 && pb_grid; ++d) {
    const int n = S->n[d];
    std::vector<double> cs((size_t)S->K * n * n);
    for (int k = 0; k < S->K; ++k)
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b)
          cs[((size_t)k * n + a) * n + b] =
              std::sqrt(S->q[d][a]) * S->C[d][((size_t)k * n + a) * n + b] / std::sqrt(S->q[d][b]);
    void *p = nullptr;
    if (hipMalloc(&p, cs.size() * sizeof(double)) != hipSuccess ||
        hipMemcpy(p, cs.data(), cs.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      if (p) hipFree(p);
      txe_system_destroy(S);
      return fail(TXE_ERR_DEVICE, "upload of the per-pair-basis tables failed");
    }
    S->csdev[d] = (double *)p;
  }
  // tables of the collocation form: A_k^d = C_k^d U_d (long double sums)
  for (int d = 0; d < 3; ++d) {
    const int n = S->n[d], r = S->r[d];
    std::vector<double> A((size_t)S->K * n * r);
    for (int k = 0; k < S->K; ++k)
      for (int a = 0; a < n; ++a) {
        const double *Crow = S->C[d].data() + ((size_t)k * n + a) * n;
        for (int s2 = 0; s2 < r; ++s2) {
          long double acc = 0.0L;
          for (int b = 0; b < n; ++b) acc += (long double)Crow[b] * S->U[d][(size_t)b * r + s2];
          A[((size_t)k * n + a) * r + s2] = (double)acc;
        }
      }
    void *p = nullptr;
    if (hipMalloc(&p, A.size() * sizeof(double)) != hipSuccess ||
        hipMemcpy(p, A.data(), A.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      if (p) hipFree(p);
      txe_system_destroy(S);
      return fail(TXE_ERR_DEVICE, "upload of the collocation tables failed");
    }
    S->acol[d] = (double *)p;
    if (d == 0) {  // grouped and weighted: [group][a][t rp0 + alpha]
      const int G = COLLOC_GROUP, RP = S->D.rp0, ng = (S->K + G - 1) / G;
      std::vector<double> A0s((size_t)ng * n * G * RP, 0.0);
      for (int k = 0; k < S->K; ++k)
        for (int a = 0; a < n; ++a)
          for (int al = 0; al < r; ++al)
            A0s[(((size_t)(k / G) * n + a) * G + k % G) * RP + al] = S->w[k] * A[((size_t)k * n + a) * r + al];
      void *q = nullptr;
      if (hipMalloc(&q, A0s.size() * sizeof(double)) != hipSuccess ||
          hipMemcpy(q, A0s.data(), A0s.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        if (q) hipFree(q);
        txe_system_destroy(S);
        return fail(TXE_ERR_DEVICE, "upload of the collocation tables failed");
      }
      S->acol0s = (double *)q;
    }
  }
  {
    void *p = nullptr;
    if (hipMalloc(&p, S->K * sizeof(double)) != hipSuccess ||
        hipMemcpy(p, S->w.data(), S->K * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
      if (p) hipFree(p);
      txe_system_destroy(S);
      return fail(TXE_ERR_DEVICE, "upload of w failed");
    }
    S->wdev = (double *)p;
  }
  *out = S;
  return ok();
}

static txe_status fe_check(const double *edges, int32_t ncells, int32_t p) {
  if (!edges) return fail(TXE_ERR_ARG, "edges is null");
  if (ncells < 1 || ncells > (1 << 20)) return fail(TXE_ERR_SHAPE, "ncells = %d out of [1, 2^20]", ncells);
  if (p < 1 || p > FE_MAX_ORDER) return fail(TXE_ERR_SHAPE, "order p = %d out of [1, %d]", p, FE_MAX_ORDER);
  if ((long long)ncells * p - 1 < 1) return fail(TXE_ERR_SHAPE, "the mesh has no unknown node");
  for (int e = 0; e <= ncells; ++e)
    if (!std::isfinite(edges[e])) return fail(TXE_ERR_ARG, "edges[%d] is not finite", e);
  for (int e = 0; e < ncells; ++e)
    if (!(edges[e + 1] > edges[e])) return fail(TXE_ERR_ARG, "edges must increase (edges[%d])", e + 1);
  return TXE_OK;
}

extern "C" txe_status txe_fe_mesh_1d(const double *edges, int32_t ncells, int32_t p, double *x, double *q) {
  txe_status st = fe_check(edges, ncells, p);
  if (st != TXE_OK) return st;
  fe_mesh_1d(edges, ncells, p, x, q);
  return ok();
}

extern "C" txe_status txe_fe_conv_matrices(const double *edges, int32_t ncells, int32_t p, const double *alpha,
                                           int32_t K, double *C) {
  txe_status st = fe_check(edges, ncells, p);
  if (st != TXE_OK) return st;
  if (!alpha || !C) return fail(TXE_ERR_ARG, "alpha and C must not be null");
  if (K < 1 || K > 4096) return fail(TXE_ERR_SHAPE, "K = %d out of [1, 4096]", K);
  for (int k = 0; k < K; ++k)
    if (!std::isfinite(alpha[k]) || alpha[k] < 0) return fail(TXE_ERR_ARG, "alpha[%d] must be finite and >= 0", k);
  const size_t n = (size_t)ncells * p - 1;
  for (int k = 0; k < K; ++k) fe_conv_matrix(edges, ncells, p, alpha[k], C + (size_t)k * n * n);
  return ok();
}

static txe_status device_failed(txe_context *ctx, hipError_t e);

extern "C" txe_status txe_hosvd_bases(txe_context *ctx, const int32_t n[3], const double *const q[3], const void *psi,
                                      int32_t dtype, int32_t N, int32_t i0, int32_t Ni, const int32_t r[3],
                                      double *const U_out[3], double *const sv_out[3]) {
  if (!ctx || !n || !q || !psi || !r || !U_out) return fail(TXE_ERR_ARG, "null argument");
  if (dtype != TXE_DTYPE_F64 && dtype != TXE_DTYPE_F32) return fail(TXE_ERR_ARG, "dtype must be F64 or F32");
  if (N < 1 || i0 < 0 || Ni < 1 || (long long)i0 + Ni > N)
    return fail(TXE_ERR_SHAPE, "targets [%d, %d) not inside [0, %d)", i0, i0 + Ni, N);
  for (int d = 0; d < 3; ++d) {
    if (n[d] < 4 || n[d] > 512 || n[d] % 4 != 0)
      return fail(TXE_ERR_SHAPE, "n[%d] = %d must be a multiple of 4 in [4, 512]", d, n[d]);
    if (r[d] < 1 || r[d] > n[d]) return fail(TXE_ERR_SHAPE, "r[%d] = %d must be in [1, n[%d]]", d, r[d], d);
    if (!q[d] || !U_out[d]) return fail(TXE_ERR_ARG, "q[%d] or U_out[%d] is null", d, d);
    for (int a = 0; a < n[d]; ++a)
      if (!std::isfinite(q[d][a]) || !(q[d][a] > 0)) return fail(TXE_ERR_ARG, "q[%d] must be finite and > 0", d);
  }
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context is in a failed state: %s", ctx->sticky_msg.c_str());
  HIP_TRY(hipSetDevice(ctx->device));
  Dims D{};
  D.n0 = n[0]; D.n1 = n[1]; D.n2 = n[2];
  const long long ng = (long long)n[0] * n[1] * n[2];
  const int nmax = std::max(n[0], std::max(n[1], n[2]));
  long long mmax = 0, per_m_max = 0;
  for (int d = 0; d < 3; ++d) {
    mmax = std::max(mmax, ng / n[d]);
    per_m_max = std::max(per_m_max, (long long)N * n[d]);
  }
  // staging of the orbitals: up to 64 Mi doubles (512 MiB), at least one m value
  const long long tcap = std::max(per_m_max, std::min<long long>(64LL << 20, per_m_max * mmax));
  const int ntile_max = (nmax + 15) / 16;
  const int tile_pairs_min = 1;
  const int ngroups = std::max(1, std::min(1024, 4096 / std::max(tile_pairs_min, ntile_max * (ntile_max + 1) / 2)));
  std::vector<void *> bufs;
  auto alloc = [&](size_t bytes) -> double * {
    void *p = nullptr;
    if (hipMalloc(&p, std::max<size_t>(bytes, 256)) != hipSuccess) return nullptr;
    bufs.push_back(p);
    return (double *)p;
  };
  auto release = [&]() {
    for (void *p : bufs) hipFree(p);
    bufs.clear();
  };
  double *T = alloc((size_t)tcap * 8), *Spart = alloc((size_t)ngroups * ntile_max * ntile_max * 256 * 8);
  double *S = alloc((size_t)nmax * nmax * 8), *V = alloc((size_t)nmax * nmax * 8);
  double *qm = alloc((size_t)mmax * 8), *qd = alloc((size_t)nmax * 8), *tr = alloc(8);
  if (!T || !Spart || !S || !V || !qm || !qd || !tr) {
    release();
    return fail(TXE_ERR_NOMEM, "device allocation of the decomposition's workspace failed");
  }
  hipStream_t s = ctx->stream;
  std::vector<double> hS((size_t)nmax * nmax), hV((size_t)nmax * nmax), hq;
  for (int d = 0; d < 3; ++d) {
    const int nd = n[d];
    const int e1 = d == 0 ? 1 : 0, e2 = d == 2 ? 1 : 2;
    hq.resize((size_t)n[e1] * n[e2]);
    for (int u = 0; u < n[e1]; ++u)
      for (int v = 0; v < n[e2]; ++v) hq[(size_t)u * n[e2] + v] = q[e1][u] * q[e2][v];
    hipError_t e = hipMemcpyAsync(qm, hq.data(), hq.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(qd, q[d], (size_t)nd * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hosvd_mode_gram(psi, dtype == TXE_DTYPE_F64, D, d, N, i0, Ni, qm, qd, T, tcap, Spart, ngroups, S, s);
    if (e == hipSuccess) e = hosvd_eigen(S, V, nd, tr, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hS.data(), S, (size_t)nd * nd * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hV.data(), V, (size_t)nd * nd * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
      release();
      return device_failed(ctx, e);
    }
    // eigenvalues descending (ties by index); the leading r columns, each
    // signed so that its largest-magnitude entry is positive, scaled by
    // 1/sqrt(q) (q-orthonormal)
    std::vector<int> order(nd);
    for (int k = 0; k < nd; ++k) order[k] = k;
    std::stable_sort(order.begin(), order.end(),
                     [&](int x, int y) { return hS[(size_t)x * nd + x] > hS[(size_t)y * nd + y]; });
    for (int k = 0; k < r[d]; ++k) {
      const int c = order[k];
      int imax = 0;
      for (int a = 1; a < nd; ++a)
        if (std::fabs(hV[(size_t)a * nd + c]) > std::fabs(hV[(size_t)imax * nd + c])) imax = a;
      const double sg = hV[(size_t)imax * nd + c] < 0 ? -1.0 : 1.0;
      for (int a = 0; a < nd; ++a) U_out[d][(size_t)a * r[d] + k] = sg * hV[(size_t)a * nd + c] / std::sqrt(q[d][a]);
    }
    if (sv_out && sv_out[d])
      for (int k = 0; k < nd; ++k) sv_out[d][k] = std::sqrt(std::max(0.0, hS[(size_t)order[k] * nd + order[k]]));
  }
  release();
  return ok();
}

extern "C" txe_status txe_system_conv(const txe_system *sys, int32_t mode, double *C_out, double *Chat_out) {
  if (!sys) return fail(TXE_ERR_ARG, "sys is null");
  if (mode < 0 || mode > 2) return fail(TXE_ERR_ARG, "mode must be 0, 1 or 2");
  if (C_out) memcpy(C_out, sys->C[mode].data(), sys->C[mode].size() * sizeof(double));
  if (Chat_out) memcpy(Chat_out, sys->Chat[mode].data(), sys->Chat[mode].size() * sizeof(double));
  return ok();
}

// ------------------------------------------------------------------------------------
// apply
// ------------------------------------------------------------------------------------
// One chunk of an apply: its tile of pairs and its back-projection launches.
struct Chunk {
  PairMap pm;
  long long P;
  int nbr;
  BackRange br[2];
};

struct Plan {
  bool f64;
  bool symmetric;
  bool want_vx;
  long long npairs;
  int NGS;
  Knobs kn;
  long long Pmax;      // pairs of the largest chunk
  size_t elt;
  size_t psi32_elems;  // FP32 copy of FP64 orbitals for the projection (0: none)
  size_t off_T2, off_G, off_S1, off_epart, off_epair, off_psi32, total;
  std::vector<Chunk> chunks;
  // per-pair bases: per-pair element counts and offsets of its regions
  size_t gbf_per = 0, off_Gbf = 0;  // split-bf16 slab images per pair (values), their region
  bool colloc = false;  // collocation form: Y0, Y1 and phi per pair (FP64)
  size_t off_Y0 = 0, off_Ys = 0, off_phi = 0;
  bool pair_bases = false;
  size_t pb_X, pb_X1, pb_X2, pb_X3, pb_S, pb_B, pb_U[3], pb_ah, pb_c1, pb_c2, pb_u0;
  size_t off_X, off_X1, off_X2, off_X3, off_S, off_B, off_V, off_Wr, off_U[3], off_ah, off_c1, off_c2, off_u0;
  int ldS = 0;
};

static size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// true when both ranges are non-null and share a byte
static bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
  const char *a0 = (const char *)a, *b0 = (const char *)b;
  return a && b && a0 < b0 + nb && b0 < a0 + na;
}

static void plan_sizes(const Dims &D, Plan &pl) {
  const size_t P = (size_t)pl.Pmax;
  const size_t perT2 = pl.pair_bases ? 0 : (size_t)D.n0 * D.rp1 * D.rp2;
  const size_t perG = (size_t)D.rp0 * D.rp1 * D.rp2;
  const size_t perS1 = pl.want_vx && !pl.colloc ? (size_t)D.n0 * D.rp2 * D.rp1 : 0;
  size_t off = 0;
  if (pl.colloc) {  // FP64 intermediates of the term-by-term reconstruction
    const size_t P8 = P * sizeof(double);
    pl.off_Y0 = off; off = align256(off + P8 * D.rp0 * D.rp1 * D.n2);
    pl.off_Ys = off; off = align256(off + P8 * COLLOC_GROUP * D.rp0 * D.n1 * D.n2);
    pl.off_phi = off; off = align256(off + P8 * D.n0 * D.n1 * D.n2);
  }
  if (pl.pair_bases) {  // FP64 regions of the per-pair decomposition and tables
    const size_t RP = D.rp0, nmax = std::max(D.n0, std::max(D.n1, D.n2));
    pl.ldS = (int)nmax;
    pl.pb_X = (size_t)D.n0 * D.n1 * D.n2;
    pl.pb_X1 = std::max((size_t)D.r0 * D.n1 * D.n2, (size_t)D.n0 * D.n2 * RP);
    pl.pb_X2 = (size_t)D.r0 * D.r1 * D.n2;
    pl.pb_X3 = (size_t)D.r0 * D.r1 * D.r2;
    pl.pb_S = nmax * nmax;
    pl.pb_B = pl.pb_X;
    pl.pb_U[0] = (size_t)D.n0 * D.r0; pl.pb_U[1] = (size_t)D.n1 * D.r1; pl.pb_U[2] = (size_t)D.n2 * D.r2;
    pl.pb_ah = (size_t)D.r0 * D.Kp * RP;
    pl.pb_c1 = (size_t)D.Kp * RP * RP;
    pl.pb_c2 = (size_t)D.Kp * D.MT2 * D.MT2 * 256;
    pl.pb_u0 = (size_t)(D.na0 / 16) * D.MT0 * 256;
    const size_t sizes[15] = {pl.pb_X,    pl.pb_X1,   pl.pb_X2,   pl.pb_X3, pl.pb_S,  pl.pb_B,  pl.pb_S, pl.pb_S,
                              pl.pb_U[0], pl.pb_U[1], pl.pb_U[2], pl.pb_ah, pl.pb_c1, pl.pb_c2, pl.pb_u0};
    size_t *offs[15] = {&pl.off_X,    &pl.off_X1,   &pl.off_X2,   &pl.off_X3, &pl.off_S,  &pl.off_B,  &pl.off_V, &pl.off_Wr,
                        &pl.off_U[0], &pl.off_U[1], &pl.off_U[2], &pl.off_ah, &pl.off_c1, &pl.off_c2, &pl.off_u0};
    for (int i = 0; i < 15; ++i) {
      *offs[i] = off;
      off = align256(off + P * sizes[i] * sizeof(double));
    }
  }
  pl.off_T2 = off; off = align256(off + P * perT2 * pl.elt);
  pl.off_G = off; off = align256(off + P * perG * pl.elt);
  pl.off_Gbf = off; off = align256(off + P * pl.gbf_per * sizeof(unsigned short));
  pl.off_S1 = off; off = align256(off + P * perS1 * pl.elt);
  pl.off_epart = off; off = align256(off + P * D.MT1 * pl.NGS * sizeof(double));
  pl.off_epair = off; off = align256(off + (size_t)pl.npairs * sizeof(double));
  pl.off_psi32 = off; off = align256(off + pl.psi32_elems * sizeof(float));
  pl.total = off;
}

// Largest chunk (pairs) whose workspace fits `limit` bytes: plan_sizes is
// affine in Pmax.
static long long max_pairs(const Dims &D, Plan &pl, size_t limit) {
  pl.Pmax = 0;
  plan_sizes(D, pl);
  const size_t fixed = pl.total;
  pl.Pmax = 1;
  plan_sizes(D, pl);
  const size_t per = pl.total - fixed + 256 * 24;  // + alignment slack of the per-pair regions (22 of them)
  if (pl.total > limit) return 0;
  return (long long)((limit - fixed) / per);
}

static PairMap tile(int tri, int ra, int nr, int ca, int nc, int symmetric, int N, int i0) {
  PairMap m;
  m.tri = tri; m.ra = ra; m.nr = nr; m.ca = ca; m.nc = nc;
  m.symmetric = symmetric; m.N = N; m.i0 = i0;
  return m;
}

static BackRange brange(int t0, int nt, int s0, int ns, int side, int acc_in, int finish, int out0) {
  BackRange b;
  b.t0 = t0; b.nt = nt; b.s0 = s0; b.ns = ns;
  b.side = side; b.acc_in = acc_in; b.finish = finish; b.out0 = out0;
  return b;
}

// Chunks of an apply under a workspace limit.
//   Symmetric: all unique pairs in one triangle when they fit; otherwise
//   the orbitals in B blocks of b and the tiles (I, J >= I) row by row: the
//   triangle of block I, the rectangles (I, J > I) feeding targets I (row
//   side) and J (column side).  Every target then meets its sources in
//   ascending order across the tiles.
//   Block: targets in chunks of tc against all sources; when one target
//   against all sources does not fit, one target at a time against source
//   chunks of sc, in ascending order.
static txe_status plan_chunks(const txe_system *sys, const txe_apply_args *a, Plan &pl, size_t limit) {
  const Dims &D = sys->D;
  const long long maxP = max_pairs(D, pl, limit);
  pl.chunks.clear();
  if (maxP < 1) {
    pl.Pmax = 1;
    plan_sizes(D, pl);
    return fail(TXE_ERR_NOMEM, "one pair needs %zu workspace bytes (limit %zu)", pl.total, limit);
  }
  const int N = a->N;
  if (pl.symmetric) {
    if (pl.npairs <= maxP) {
      pl.chunks.push_back({tile(1, 0, N, 0, N, 1, N, 0), pl.npairs, 1, {brange(0, N, 0, N, 2, 0, 1, 0), {}}});
    } else {
      long long b = (long long)std::floor(std::sqrt((double)maxP));
      while (b > 1 && b * b > maxP) --b;
      const int B = (int)((N + b - 1) / b);
      const int bs = (N + B - 1) / B;  // balanced block size (<= b)
      for (int I = 0; I < B; ++I) {
        const int ra = I * bs, nr = std::min(bs, N - ra);
        for (int J = I; J < B; ++J) {
          const int ca = J * bs, nc = std::min(bs, N - ca);
          if (nr <= 0 || nc <= 0) continue;
          Chunk c{};
          if (I == J) {
            c.pm = tile(1, ra, nr, ra, nr, 1, N, 0);
            c.P = (long long)nr * (nr + 1) / 2;
            c.nbr = 1;
            c.br[0] = brange(ra, nr, ra, nr, 2, I > 0, I == B - 1, 0);
          } else {
            c.pm = tile(0, ra, nr, ca, nc, 1, N, 0);
            c.P = (long long)nr * nc;
            c.nbr = 2;
            c.br[0] = brange(ra, nr, ca, nc, 0, 1, J == B - 1, 0);   // targets I, sources J
            c.br[1] = brange(ca, nc, ra, nr, 1, I > 0, 0, 0);        // targets J, sources I
          }
          pl.chunks.push_back(c);
        }
      }
    }
  } else {
    const int i0 = a->i0, Ni = a->Ni;
    if (N <= maxP) {
      const int tmax = (int)std::min<long long>(Ni, maxP / N);
      const int nch = (Ni + tmax - 1) / tmax;
      const int tc = (Ni + nch - 1) / nch;
      for (int t = 0; t < Ni; t += tc) {
        const int nt = std::min(tc, Ni - t);
        pl.chunks.push_back({tile(0, i0 + t, nt, 0, N, 0, N, i0), (long long)nt * N, 1,
                             {brange(i0 + t, nt, 0, N, 0, 0, 1, i0), {}}});
      }
    } else {
      const int nsc = (int)((N + maxP - 1) / maxP);
      const int sc = (N + nsc - 1) / nsc;
      for (int t = 0; t < Ni; ++t)
        for (int c0 = 0; c0 < N; c0 += sc) {
          const int nc = std::min(sc, N - c0);
          pl.chunks.push_back({tile(0, i0 + t, 1, c0, nc, 0, N, i0), (long long)nc, 1,
                               {brange(i0 + t, 1, c0, nc, 0, c0 > 0, c0 + nc == N, i0), {}}});
        }
    }
  }
  pl.Pmax = 0;
  for (const Chunk &c : pl.chunks) pl.Pmax = std::max(pl.Pmax, c.P);
  plan_sizes(D, pl);
  return TXE_OK;
}

static txe_status make_plan(const txe_system *sys, const txe_apply_args *a, const Knobs &kn, Plan &pl,
                            size_t limit) {
  const Dims &D = sys->D;
  pl.kn = kn;
  pl.f64 = a->compute == TXE_COMPUTE_F64;
  pl.symmetric = a->symmetric != 0;
  pl.want_vx = a->vxpsi != nullptr;
  pl.pair_bases = a->pair_bases != 0;
  pl.colloc = a->form == TXE_FORM_COLLOCATION;
  pl.elt = pl.f64 ? sizeof(double) : sizeof(float);
  // the reduced-precision forms project FP64 orbitals from an FP32 copy
  // (half the bytes of the projection's orbital reads) when it fits beside
  // the chunk workspace
  pl.psi32_elems = (!pl.f64 && a->dtype == TXE_DTYPE_F64) ? (size_t)a->N * D.n0 * D.n1 * D.n2 : 0;
  pl.npairs = pl.symmetric ? (long long)a->N * (a->N + 1) / 2 : (long long)a->Ni * a->N;
  const int mt = std::max(D.MT0, std::max(D.MT1, D.MT2));
  const int nsplit = a->compute == TXE_COMPUTE_BF16X3 ? 2 : a->compute == TXE_COMPUTE_BF16X6 ? 3 : 0;
  pl.gbf_per = (size_t)D.rp0 * bf_frag_elems(mt, nsplit);
  const int rows = core_rows(pl.f64, nsplit, mt);
  // fewest gamma' splits whose rows fit the accumulator registers, times the
  // tuned multiplier; then trimmed so that no split is empty
  int ngs = (D.r2 + rows - 1) / rows * std::max(1, kn.ngs_mul);
  const int gper = (D.r2 + ngs - 1) / ngs;
  pl.NGS = (D.r2 + gper - 1) / gper;
  if (pl.psi32_elems && pl.psi32_elems * sizeof(float) > limit / 4) pl.psi32_elems = 0;
  return plan_chunks(sys, a, pl, limit);
}

// Key of the tuning cache: device architecture and every size that selects
// a kernel instance or changes the work per launch.
static std::string plan_key(const txe_context *ctx, const txe_system *sys, const txe_apply_args *a) {
  static const char *cname[] = {"f64", "f32", "bf16x3", "bf16x6"};
  const Dims &D = sys->D;
  char buf[256];
  snprintf(buf, sizeof buf, "%s|n=%d,%d,%d|r=%d,%d,%d|K=%d|N=%d|Ni=%d|%s|%s|%s%s%s", ctx->arch.c_str(), D.n0, D.n1,
           D.n2, D.r0, D.r1, D.r2, D.K, a->N, a->symmetric ? a->N : a->Ni, cname[a->compute & 3],
           a->symmetric ? "sym" : "block", a->vxpsi ? "vx" : "energy", a->pair_bases ? "|pair-bases" : "",
           a->form == TXE_FORM_COLLOCATION ? "|collocation" : "");
  return buf;
}

static Knobs knobs_for(const txe_context *ctx, const txe_system *sys, const txe_apply_args *a) {
  auto it = ctx->plans.find(plan_key(ctx, sys, a));
  return it == ctx->plans.end() ? Knobs{} : it->second;
}

static bool knobs_valid(const Knobs &k) {
  return (k.ngs_mul == 1 || k.ngs_mul == 2 || k.ngs_mul == 4) && k.proj_gt >= 1 && k.proj_gt <= 4 &&
         k.back_ncg >= 0 && k.back_ncg <= 2 && k.grid_cap >= 256 && k.grid_cap <= 16384 && k.back_form >= 0 &&
         k.back_form <= 3;
}

static txe_status validate_args(const txe_context *ctx, const txe_system *sys, const txe_apply_args *a) {
  if (!ctx || !sys || !a) return fail(TXE_ERR_ARG, "null argument");
  if (sys->device != ctx->device) return fail(TXE_ERR_ARG, "system and context are on different devices");
  if (a->compute != TXE_COMPUTE_F64 && a->compute != TXE_COMPUTE_F32 && a->compute != TXE_COMPUTE_BF16X3 &&
      a->compute != TXE_COMPUTE_BF16X6)
    return fail(TXE_ERR_ARG, "unknown compute %d", a->compute);
  if (a->dtype != TXE_DTYPE_F64 && a->dtype != TXE_DTYPE_F32) return fail(TXE_ERR_ARG, "unknown dtype %d", a->dtype);
  if (a->compute == TXE_COMPUTE_F64 && a->dtype != TXE_DTYPE_F64)
    return fail(TXE_ERR_ARG, "FP64 compute requires FP64 orbitals");
  if (a->N < 1) return fail(TXE_ERR_SHAPE, "N = %d must be >= 1", a->N);
  if (!a->psi) return fail(TXE_ERR_ARG, "psi is null");
  if (a->symmetric != 0 && a->symmetric != 1) return fail(TXE_ERR_ARG, "symmetric must be 0 or 1");
  if (a->symmetric) {
    if (a->i0 != 0 || a->Ni != a->N) return fail(TXE_ERR_SHAPE, "symmetric mode requires i0 = 0 and Ni = N");
  } else {
    if (a->i0 < 0 || a->Ni < 1 || (long long)a->i0 + a->Ni > a->N)
      return fail(TXE_ERR_SHAPE, "target block [%d, %d) not inside [0, %d)", a->i0, a->i0 + a->Ni, a->N);
  }
  if (a->out_weighted != 0 && a->out_weighted != 1) return fail(TXE_ERR_ARG, "out_weighted must be 0 or 1");
  if (a->pair_bases != 0 && a->pair_bases != 1) return fail(TXE_ERR_ARG, "pair_bases must be 0 or 1");
  if (a->form != TXE_FORM_CORE && a->form != TXE_FORM_COLLOCATION)
    return fail(TXE_ERR_ARG, "form must be TXE_FORM_CORE or TXE_FORM_COLLOCATION");
  if (a->form == TXE_FORM_COLLOCATION) {
    if (a->compute != TXE_COMPUTE_F64)
      return fail(TXE_ERR_UNSUPPORTED, "the collocation form is implemented in FP64 compute only");
    if (a->pair_bases) return fail(TXE_ERR_UNSUPPORTED, "the collocation form uses the system's shared bases");
  }
  if (a->pair_bases) {
    if (a->compute != TXE_COMPUTE_F64)
      return fail(TXE_ERR_UNSUPPORTED, "per-pair bases are implemented in FP64 compute only");
    if (std::max(sys->n[0], std::max(sys->n[1], sys->n[2])) > PB_MAX_N)
      return fail(TXE_ERR_UNSUPPORTED, "per-pair bases need n[d] <= %d (the Jacobi eigensolver works in LDS)",
                  PB_MAX_N);
  }
  if (!a->vxpsi && !a->ex && !a->e_pairs && !a->e_orb)
    return fail(TXE_ERR_ARG, "nothing to compute (vxpsi, ex, e_pairs and e_orb are null)");
  const size_t elt = a->dtype == TXE_DTYPE_F64 ? 8 : 4;
  const size_t grid = (size_t)sys->n[0] * sys->n[1] * sys->n[2];
  const size_t npairs = a->symmetric ? (size_t)a->N * (a->N + 1) / 2 : (size_t)a->Ni * a->N;
  // every output against every input and every other output
  struct Buf {
    const void *p;
    size_t bytes;
    const char *name;
  };
  const Buf bufs[5] = {{a->psi, (size_t)a->N * grid * elt, "psi"},
                       {a->vxpsi, (size_t)a->Ni * grid * elt, "vxpsi"},
                       {a->ex, 8, "ex"},
                       {a->e_pairs, npairs * 8, "e_pairs"},
                       {a->e_orb, (size_t)a->Ni * 8, "e_orb"}};
  for (int o = 1; o < 5; ++o)
    for (int b = 0; b < o; ++b)
      if (overlaps(bufs[o].p, bufs[o].bytes, bufs[b].p, bufs[b].bytes))
        return fail(TXE_ERR_ARG, "%s overlaps %s", bufs[o].name, bufs[b].name);
  if (((uintptr_t)a->psi % (4 * elt)) != 0) return fail(TXE_ERR_ARG, "psi must be %zu-byte aligned", 4 * elt);
  if (a->vxpsi && ((uintptr_t)a->vxpsi % elt) != 0) return fail(TXE_ERR_ARG, "vxpsi is misaligned");
  if (((uintptr_t)a->ex % 8) || ((uintptr_t)a->e_pairs % 8) || ((uintptr_t)a->e_orb % 8))
    return fail(TXE_ERR_ARG, "ex, e_pairs and e_orb must be 8-byte aligned");
  return TXE_OK;
}

extern "C" txe_status txe_workspace_query(txe_context *ctx, const txe_system *sys, const txe_apply_args *args,
                                          size_t *bytes) {
  if (!bytes) return fail(TXE_ERR_ARG, "bytes is null");
  txe_status st = validate_args(ctx, sys, args);
  if (st != TXE_OK) return st;
  Plan pl;
  if ((st = make_plan(sys, args, knobs_for(ctx, sys, args), pl, workspace_limit())) != TXE_OK) return st;
  *bytes = pl.total;
  return ok();
}

template <typename T>
static ChunkArgs<T> chunk_args(const txe_system *sys, const txe_apply_args *a, const Plan &pl, char *ws) {
  ChunkArgs<T> c{};
  c.D = sys->D;
  c.N = a->N;
  c.NGS = pl.NGS;
  c.proj_gt = pl.kn.proj_gt;
  c.back_ncg = pl.kn.back_ncg;
  c.grid_cap = pl.kn.grid_cap;
  c.back_form = pl.kn.back_form;
  c.psi = a->psi;
  c.vx = a->vxpsi;
  c.out_scale = a->out_scale;
  c.weighted = a->out_weighted;
  for (int d = 0; d < 3; ++d) c.qdev[d] = sys->qdev[d];
  c.T2 = (T *)(ws + pl.off_T2);
  c.G = (T *)(ws + pl.off_G);
  c.Gbf = pl.gbf_per ? (unsigned short *)(ws + pl.off_Gbf) : nullptr;
  c.S1 = (T *)(ws + pl.off_S1);
  c.epart = (double *)(ws + pl.off_epart);
  c.epair = (double *)(ws + pl.off_epair);
  return c;
}

// Enqueues one planned apply on stream s with workspace ws (pl.total bytes):
// its chunks in order, then the energy reductions over all pair energies.
static hipError_t run_plan(const txe_system *sys, const txe_apply_args *args, const Plan &pl, char *ws,
                           hipStream_t s, Prof *prof) {
  // launch errors are read back with hipGetLastError, which also returns the
  // failure of any earlier runtime call of this thread (each of those was
  // reported by its own return code): clear it so it is not taken for a launch's
  (void)hipGetLastError();
  hipError_t e = hipSuccess;
  const bool psi64 = args->dtype == TXE_DTYPE_F64;
  for (size_t ci = 0; ci < pl.chunks.size() && e == hipSuccess; ++ci) {
    const Chunk &ch = pl.chunks[ci];
    if (pl.pair_bases) {
      ChunkArgs<double> c = chunk_args<double>(sys, args, pl, ws);
      c.pm = ch.pm; c.P = (int)ch.P; c.nbr = ch.nbr; c.br[0] = ch.br[0]; c.br[1] = ch.br[1];
      Tables<double> tb = sys->t64.t;  // the per-pair regions replace the shared term tables
      tb.Ahat = (double *)(ws + pl.off_ah);
      tb.C1f = (double *)(ws + pl.off_c1);
      tb.C2chain = (double *)(ws + pl.off_c2);
      tb.U0chain = (double *)(ws + pl.off_u0);
      tb.ps_ah = (long long)pl.pb_ah; tb.ps_c1 = (long long)pl.pb_c1;
      tb.ps_c2 = (long long)pl.pb_c2; tb.ps_u0 = (long long)pl.pb_u0;
      PairBasesArgs pb{};
      pb.X = (double *)(ws + pl.off_X); pb.X1 = (double *)(ws + pl.off_X1);
      pb.X2 = (double *)(ws + pl.off_X2); pb.X3 = (double *)(ws + pl.off_X3);
      pb.S = (double *)(ws + pl.off_S); pb.ldS = pl.ldS;
      pb.B = (double *)(ws + pl.off_B);
      pb.V = (double *)(ws + pl.off_V); pb.Wr = (double *)(ws + pl.off_Wr);
      for (int d = 0; d < 3; ++d) {
        pb.Ut[d] = (double *)(ws + pl.off_U[d]);
        pb.Cs[d] = sys->csdev[d];
      }
      pb.w = sys->wdev;
      pb.ps_ah = tb.ps_ah; pb.ps_c1 = tb.ps_c1; pb.ps_c2 = tb.ps_c2; pb.ps_u0 = tb.ps_u0;
      e = run_chunk_pp(tb, pb, c, pl.want_vx, s, prof);
    } else if (pl.colloc) {
      ChunkArgs<double> c = chunk_args<double>(sys, args, pl, ws);
      c.pm = ch.pm; c.P = (int)ch.P; c.nbr = ch.nbr; c.br[0] = ch.br[0]; c.br[1] = ch.br[1];
      CollocArgs cl{};
      for (int d = 0; d < 3; ++d) cl.A[d] = sys->acol[d];
      cl.A0s = sys->acol0s;
      cl.Y0 = (double *)(ws + pl.off_Y0);
      cl.Ys = (double *)(ws + pl.off_Ys);
      cl.phi = (double *)(ws + pl.off_phi);
      e = run_chunk_colloc(sys->t64.t, cl, c, pl.want_vx, s, prof);
    } else if (pl.f64) {
      ChunkArgs<double> c = chunk_args<double>(sys, args, pl, ws);
      c.pm = ch.pm; c.P = (int)ch.P; c.nbr = ch.nbr; c.br[0] = ch.br[0]; c.br[1] = ch.br[1];
      e = run_chunk_f64(sys->t64.t, c, pl.want_vx, s, prof);
    } else {
      ChunkArgs<float> c = chunk_args<float>(sys, args, pl, ws);
      c.pm = ch.pm; c.P = (int)ch.P; c.nbr = ch.nbr; c.br[0] = ch.br[0]; c.br[1] = ch.br[1];
      if (pl.psi32_elems) {
        c.psi32 = (const float *)(ws + pl.off_psi32);
        c.psi32_fill = ci == 0 ? 1 : 0;
        c.psi_elems = pl.psi32_elems;
      }
      if (args->compute == TXE_COMPUTE_F32)
        e = run_chunk_f32(sys->t32.t, c, psi64, pl.want_vx, s, prof);
      else
        e = run_chunk_bf16(sys->t32.t, sys->tbf.t, args->compute == TXE_COMPUTE_BF16X3 ? 2 : 3, c, psi64,
                           pl.want_vx, s, prof);
    }
  }
  if (e == hipSuccess)
    e = run_energy((const double *)(ws + pl.off_epair), pl.npairs, pl.symmetric ? 1 : 0, args->N,
                   pl.symmetric ? 0 : args->i0, pl.symmetric ? args->N : args->Ni, args->ex, args->e_pairs,
                   args->e_orb, s, prof);
  return e;
}

static txe_status device_failed(txe_context *ctx, hipError_t e) {
  ctx->sticky = true;
  ctx->sticky_msg = hipGetErrorString(e);
  return fail(TXE_ERR_DEVICE, "kernel launch failed: %s", hipGetErrorString(e));
}

static txe_status apply_with(txe_context *ctx, const txe_system *sys, const txe_apply_args *args, const Knobs &kn) {
  txe_status st = validate_args(ctx, sys, args);
  if (st != TXE_OK) return st;
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context has a previous device error: %s", ctx->sticky_msg.c_str());
  Plan pl;
  if ((st = make_plan(sys, args, kn, pl, workspace_limit())) != TXE_OK) return st;
  if ((st = ensure_workspace(ctx, pl.total)) != TXE_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  const hipError_t e = run_plan(sys, args, pl, (char *)ctx->ws, ctx->stream, &ctx->prof);
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}

extern "C" txe_status txe_apply_noalloc(txe_context *ctx, const txe_system *sys, const txe_apply_args *args) {
  if (!ctx || !sys || !args) return fail(TXE_ERR_ARG, "null argument");
  txe_status st = validate_args(ctx, sys, args);
  if (st != TXE_OK) return st;
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context has a previous device error: %s", ctx->sticky_msg.c_str());
  Plan pl;
  if ((st = make_plan(sys, args, knobs_for(ctx, sys, args), pl, TXE_NOALLOC_SCRATCH_BYTES)) != TXE_OK)
    return st == TXE_ERR_NOMEM ? fail(st, "allocation-free apply: %s (scratch array of %zu bytes)",
                                      g_last_error.c_str(), (size_t)TXE_NOALLOC_SCRATCH_BYTES)
                               : st;
  HIP_TRY(hipSetDevice(ctx->device));
  void *ws = nullptr;
  const hipError_t es = scratch_address(ctx->device, &ws);
  if (es != hipSuccess || !ws)
    return fail(TXE_ERR_DEVICE, "the scratch array of device %d is unavailable: %s", ctx->device,
                hipGetErrorString(es));
  Prof off;  // no timing events on this path
  const hipError_t e = run_plan(sys, args, pl, (char *)ws, ctx->stream, &off);
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}

extern "C" txe_status txe_apply(txe_context *ctx, const txe_system *sys, const txe_apply_args *args) {
  if (!ctx || !sys || !args) return fail(TXE_ERR_ARG, "null argument");
  return apply_with(ctx, sys, args, knobs_for(ctx, sys, args));
}

// ------------------------------------------------------------------------------------
// batched apply: S independent systems on L concurrent lanes
// ------------------------------------------------------------------------------------
struct Batch {
  std::vector<Plan> plans;
  std::vector<int> order;            // systems by decreasing estimated cost
  std::vector<int> lane_of;          // lane of each system
  std::vector<size_t> lane_off;      // workspace offset of each lane
  int lanes = 0;
  size_t total = 0;
};

// Work estimate of one apply (multiply-adds of the dominant stages): the
// core's chained contractions K * rp^3 * (rp1 + rp2) plus the projections
// and back-projection n^3 * rp per pair.
static double cost_estimate(const txe_system *sys, const Plan &pl) {
  const Dims &D = sys->D;
  const double rp = D.rp0, n3 = (double)D.n0 * D.n1 * D.n2;
  const double core = (double)D.K * rp * rp * rp * (D.rp1 + D.rp2);
  const double proj = n3 * rp * (pl.want_vx ? 4.0 : 2.0);
  return (double)pl.npairs * (core + proj);
}

static txe_status batch_plan(txe_context *ctx, int S, const txe_system *const *systems, const txe_apply_args *args,
                             int lanes, Batch &b) {
  if (!ctx || !systems || !args) return fail(TXE_ERR_ARG, "null argument");
  if (S < 1 || S > 4096) return fail(TXE_ERR_SHAPE, "S = %d not in [1, 4096]", S);
  if (lanes < 1 || lanes > 16) return fail(TXE_ERR_ARG, "lanes = %d not in [1, 16]", lanes);
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context has a previous device error: %s", ctx->sticky_msg.c_str());
  b.plans.resize(S);
  std::vector<double> cost(S);
  for (int i = 0; i < S; ++i) {
    txe_status st = validate_args(ctx, systems[i], &args[i]);
    if (st != TXE_OK) return fail(st, "system %d: %s", i, g_last_error.c_str());
    if ((st = make_plan(systems[i], &args[i], knobs_for(ctx, systems[i], &args[i]), b.plans[i], workspace_limit())) !=
        TXE_OK)
      return fail(st, "system %d: %s", i, g_last_error.c_str());
    cost[i] = cost_estimate(systems[i], b.plans[i]);
  }
  // outputs of different systems run concurrently and must not overlap
  struct Range { const char *lo, *hi; int sys; };
  std::vector<Range> outs;
  for (int i = 0; i < S; ++i) {
    const txe_apply_args &a = args[i];
    const size_t elt = a.dtype == TXE_DTYPE_F64 ? 8 : 4;
    const size_t grid = (size_t)systems[i]->n[0] * systems[i]->n[1] * systems[i]->n[2];
    if (a.vxpsi) outs.push_back({(const char *)a.vxpsi, (const char *)a.vxpsi + (size_t)a.Ni * grid * elt, i});
    if (a.ex) outs.push_back({(const char *)a.ex, (const char *)a.ex + 8, i});
    if (a.e_pairs) outs.push_back({(const char *)a.e_pairs, (const char *)a.e_pairs + b.plans[i].npairs * 8, i});
    if (a.e_orb) outs.push_back({(const char *)a.e_orb, (const char *)a.e_orb + (size_t)a.Ni * 8, i});
  }
  std::sort(outs.begin(), outs.end(), [](const Range &x, const Range &y) { return x.lo < y.lo; });
  for (size_t k = 1; k < outs.size(); ++k)
    if (outs[k].lo < outs[k - 1].hi && outs[k].sys != outs[k - 1].sys)
      return fail(TXE_ERR_ARG, "outputs of systems %d and %d overlap", outs[k - 1].sys, outs[k].sys);
  // longest-processing-time-first assignment of systems to lanes
  b.lanes = std::min(lanes, S);
  b.order.resize(S);
  for (int i = 0; i < S; ++i) b.order[i] = i;
  std::stable_sort(b.order.begin(), b.order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
  std::vector<double> load(b.lanes, 0.0);
  std::vector<size_t> need(b.lanes, 0);
  b.lane_of.assign(S, 0);
  for (int i : b.order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b.lane_of[i] = l;
    load[l] += cost[i];
    need[l] = std::max(need[l], b.plans[i].total);  // a lane runs its systems one after another
  }
  b.lane_off.resize(b.lanes);
  size_t off = 0;
  for (int l = 0; l < b.lanes; ++l) {
    b.lane_off[l] = off;
    off = align256(off + need[l]);
  }
  b.total = off;
  if (b.total > workspace_limit())
    return fail(TXE_ERR_NOMEM, "batched workspace of %zu bytes exceeds the limit of %zu bytes", b.total,
                workspace_limit());
  return TXE_OK;
}

// Streams and events of the lanes (created outside any capture).
static txe_status ensure_lanes(txe_context *ctx, int lanes) {
  HIP_TRY(hipSetDevice(ctx->device));
  if (!ctx->fork) HIP_TRY(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  while ((int)ctx->lanes.size() < lanes) {
    hipStream_t s = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ctx->lanes.push_back(s);
    hipEvent_t e = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    ctx->lane_done.push_back(e);
  }
  return TXE_OK;
}

// Enqueues the batch: lanes fork from s, run their systems in cost order,
// and s waits for every lane (the fork/join pattern also joins the lanes
// into a capture of s).
static hipError_t batch_enqueue(txe_context *ctx, const txe_system *const *systems, const txe_apply_args *args,
                                const Batch &b, char *ws, hipStream_t s) {
  Prof off;  // per-kernel timing is not taken inside batches
  if (b.lanes == 1) {
    for (int i : b.order) {
      const hipError_t e = run_plan(systems[i], &args[i], b.plans[i], ws, s, &off);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e = hipEventRecord(ctx->fork, s);
  for (int l = 0; l < b.lanes && e == hipSuccess; ++l) e = hipStreamWaitEvent(ctx->lanes[l], ctx->fork, 0);
  for (int i : b.order) {
    if (e != hipSuccess) break;
    const int l = b.lane_of[i];
    e = run_plan(systems[i], &args[i], b.plans[i], ws + b.lane_off[l], ctx->lanes[l], &off);
  }
  for (int l = 0; l < b.lanes; ++l) {
    // the join is recorded even after a failure so that a capture can end
    const hipError_t e1 = hipEventRecord(ctx->lane_done[l], ctx->lanes[l]);
    const hipError_t e2 = hipStreamWaitEvent(s, ctx->lane_done[l], 0);
    if (e == hipSuccess) e = e1 != hipSuccess ? e1 : e2;
  }
  return e;
}

extern "C" txe_status txe_apply_batched(txe_context *ctx, int32_t S, const txe_system *const *systems,
                                        const txe_apply_args *args, int32_t lanes) {
  Batch b;
  txe_status st = batch_plan(ctx, S, systems, args, lanes, b);
  if (st != TXE_OK) return st;
  if ((st = ensure_workspace(ctx, b.total)) != TXE_OK) return st;
  if ((st = ensure_lanes(ctx, b.lanes)) != TXE_OK) return st;
  const hipError_t e = batch_enqueue(ctx, systems, args, b, (char *)ctx->ws, ctx->stream);
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}

// ------------------------------------------------------------------------------------
// graph: a batch captured once and replayed
// ------------------------------------------------------------------------------------
struct txe_graph {
  txe_context *ctx = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void *ws = nullptr;  // the graph's own workspace
  size_t ws_bytes = 0;
};

static void graph_free(txe_graph *g) {
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  if (g->ws) hipFree(g->ws);
  delete g;
}

extern "C" txe_status txe_graph_capture_batched(txe_context *ctx, int32_t S, const txe_system *const *systems,
                                                const txe_apply_args *args, int32_t lanes, txe_graph **out) {
  if (!out) return fail(TXE_ERR_ARG, "out is null");
  *out = nullptr;
  Batch b;
  txe_status st = batch_plan(ctx, S, systems, args, lanes, b);
  if (st != TXE_OK) return st;
  if ((st = ensure_lanes(ctx, b.lanes)) != TXE_OK) return st;
  if (!ctx->cap) HIP_TRY(hipStreamCreateWithFlags(&ctx->cap, hipStreamNonBlocking));
  auto *g = new txe_graph();
  g->ctx = ctx;
  g->ws_bytes = std::max<size_t>(b.total, 256);
  if (hipMalloc(&g->ws, g->ws_bytes) != hipSuccess) {
    (void)hipGetLastError();
    g->ws = nullptr;
    graph_free(g);
    return fail(TXE_ERR_NOMEM, "hipMalloc of %zu bytes for the graph workspace failed", b.total);
  }
  hipError_t e = hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    const hipError_t el = batch_enqueue(ctx, systems, args, b, (char *)g->ws, ctx->cap);
    const hipError_t ec = hipStreamEndCapture(ctx->cap, &g->graph);
    e = el != hipSuccess ? el : ec;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    graph_free(g);
    return fail(TXE_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
  }
  *out = g;
  return ok();
}

extern "C" txe_status txe_graph_launch(txe_graph *g) {
  if (!g) return fail(TXE_ERR_ARG, "graph is null");
  txe_context *ctx = g->ctx;
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context has a previous device error: %s", ctx->sticky_msg.c_str());
  HIP_TRY(hipSetDevice(ctx->device));
  const hipError_t e = hipGraphLaunch(g->exec, ctx->stream);
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}

extern "C" txe_status txe_graph_destroy(txe_graph *g) {
  if (!g) return fail(TXE_ERR_ARG, "graph is null");
  HIP_TRY(hipSetDevice(g->ctx->device));
  HIP_TRY(hipStreamSynchronize(g->ctx->stream));
  graph_free(g);
  return ok();
}

// ------------------------------------------------------------------------------------
// tuner: coordinate descent over the launch shapes, timed on the device
// ------------------------------------------------------------------------------------
static txe_status time_apply(txe_context *ctx, const txe_system *sys, const txe_apply_args *args, const Knobs &kn,
                             int reps, double *ms) {
  txe_status st = apply_with(ctx, sys, args, kn);  // warm-up (and workspace growth)
  if (st != TXE_OK) return st;
  hipEvent_t a = nullptr, z = nullptr;
  HIP_TRY(hipEventCreate(&a));
  if (hipEventCreate(&z) != hipSuccess) {
    hipEventDestroy(a);
    return fail(TXE_ERR_DEVICE, "hipEventCreate failed");
  }
  hipError_t e = hipEventRecord(a, ctx->stream);
  for (int i = 0; i < reps && e == hipSuccess && st == TXE_OK; ++i) st = apply_with(ctx, sys, args, kn);
  if (e == hipSuccess) e = hipEventRecord(z, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(z);
  float t = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, a, z);
  hipEventDestroy(a);
  hipEventDestroy(z);
  if (st != TXE_OK) return st;
  if (e != hipSuccess) return fail(TXE_ERR_DEVICE, "timing failed: %s", hipGetErrorString(e));
  *ms = t / reps;
  return TXE_OK;
}

extern "C" txe_status txe_tune(txe_context *ctx, const txe_system *sys, const txe_apply_args *args, int32_t reps,
                               double *best_ms) {
  if (!ctx || !sys || !args) return fail(TXE_ERR_ARG, "null argument");
  if (reps < 1 || reps > 1000) return fail(TXE_ERR_ARG, "reps = %d not in [1, 1000]", reps);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(ctx->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(TXE_ERR_STATE, "cannot tune while the stream is captured");
  const bool prof_on = ctx->prof.on;
  ctx->prof.on = false;
  Knobs best{};
  double best_t = 0.0;
  txe_status st = time_apply(ctx, sys, args, best, reps, &best_t);
  const std::vector<int> ngs = {1, 2, 4}, gt = {1, 2, 3, 4}, ncg = {1, 2}, cap = {1024, 2048, 4096}, form = {1, 2, 3};
  for (int sweep = 0; sweep < 2 && st == TXE_OK; ++sweep) {
    const Knobs start = best;
    for (int knob = 0; knob < 5 && st == TXE_OK; ++knob) {
      const std::vector<int> &vals = knob == 0 ? ngs : knob == 1 ? gt : knob == 2 ? ncg : knob == 3 ? cap : form;
      for (int v : vals) {
        Knobs k = best;
        int &field = knob == 0 ? k.ngs_mul
                     : knob == 1 ? k.proj_gt
                     : knob == 2 ? k.back_ncg
                     : knob == 3 ? k.grid_cap
                                 : k.back_form;
        if (field == v) continue;
        field = v;
        double t = 0.0;
        if ((st = time_apply(ctx, sys, args, k, reps, &t)) != TXE_OK) break;
        if (t < best_t) {
          best_t = t;
          best = k;
        }
      }
    }
    if (start.ngs_mul == best.ngs_mul && start.proj_gt == best.proj_gt && start.back_ncg == best.back_ncg &&
        start.grid_cap == best.grid_cap && start.back_form == best.back_form)
      break;
  }
  ctx->prof.on = prof_on;
  if (st != TXE_OK) return st;
  ctx->plans[plan_key(ctx, sys, args)] = best;
  if (best_ms) *best_ms = best_t;
  return ok();
}

extern "C" txe_status txe_plan_get(txe_context *ctx, const txe_system *sys, const txe_apply_args *args,
                                   int32_t knobs[5], int32_t *tuned) {
  if (!ctx || !sys || !args || !knobs) return fail(TXE_ERR_ARG, "null argument");
  txe_status st = validate_args(ctx, sys, args);
  if (st != TXE_OK) return st;
  const std::string key = plan_key(ctx, sys, args);
  auto it = ctx->plans.find(key);
  const Knobs k = it == ctx->plans.end() ? Knobs{} : it->second;
  knobs[0] = k.ngs_mul; knobs[1] = k.proj_gt; knobs[2] = k.back_ncg; knobs[3] = k.grid_cap; knobs[4] = k.back_form;
  if (tuned) *tuned = it != ctx->plans.end();
  return ok();
}

// Cache file: a JSON object mapping each problem key to its launch shape,
// one entry per line:
//   {
//    "gfx950|n=64,64,64|...": {"ngs_mul": 1, "proj_gt": 4, "back_ncg": 0, "grid_cap": 2048, "back_form": 0},
//    ...
//   }
// ("back_form" may be absent: 0.)
extern "C" txe_status txe_tune_save(txe_context *ctx, const char *path) {
  if (!ctx || !path) return fail(TXE_ERR_ARG, "null argument");
  FILE *f = fopen(path, "w");
  if (!f) return fail(TXE_ERR_ARG, "cannot open %s for writing", path);
  fprintf(f, "{\n");
  size_t i = 0;
  for (const auto &kv : ctx->plans) {
    const Knobs &k = kv.second;
    fprintf(f, " \"%s\": {\"ngs_mul\": %d, \"proj_gt\": %d, \"back_ncg\": %d, \"grid_cap\": %d, \"back_form\": %d}%s\n",
            kv.first.c_str(), k.ngs_mul, k.proj_gt, k.back_ncg, k.grid_cap, k.back_form,
            ++i < ctx->plans.size() ? "," : "");
  }
  fprintf(f, "}\n");
  const bool bad = ferror(f) != 0;
  if (fclose(f) != 0 || bad) return fail(TXE_ERR_ARG, "write to %s failed", path);
  return ok();
}

static bool read_int_field(const std::string &line, const char *name, int *v) {
  const std::string pat = std::string("\"") + name + "\":";
  const size_t at = line.find(pat);
  if (at == std::string::npos) return false;
  char *end = nullptr;
  const long x = strtol(line.c_str() + at + pat.size(), &end, 10);
  if (end == line.c_str() + at + pat.size()) return false;
  *v = (int)x;
  return true;
}

extern "C" txe_status txe_tune_load(txe_context *ctx, const char *path, int32_t *loaded) {
  if (!ctx || !path) return fail(TXE_ERR_ARG, "null argument");
  FILE *f = fopen(path, "r");
  if (!f) return fail(TXE_ERR_ARG, "cannot open %s", path);
  std::map<std::string, Knobs> got;
  char buf[1024];
  int lineno = 0;
  txe_status st = TXE_OK;
  while (fgets(buf, sizeof buf, f)) {
    ++lineno;
    const std::string line(buf);
    const size_t q0 = line.find('"');
    if (q0 == std::string::npos) continue;  // braces
    const size_t q1 = line.find('"', q0 + 1);
    Knobs k;
    if (q1 == std::string::npos || !read_int_field(line, "ngs_mul", &k.ngs_mul) ||
        !read_int_field(line, "proj_gt", &k.proj_gt) || !read_int_field(line, "back_ncg", &k.back_ncg) ||
        !read_int_field(line, "grid_cap", &k.grid_cap) ||
        (line.find("\"back_form\":") != std::string::npos && !read_int_field(line, "back_form", &k.back_form)) ||
        !knobs_valid(k)) {
      st = fail(TXE_ERR_ARG, "%s:%d: not a valid cache entry", path, lineno);
      break;
    }
    got[line.substr(q0 + 1, q1 - q0 - 1)] = k;
  }
  fclose(f);
  if (st != TXE_OK) return st;
  for (const auto &kv : got) ctx->plans[kv.first] = kv.second;
  if (loaded) *loaded = (int32_t)got.size();
  return ok();
}

// ------------------------------------------------------------------------------------
// measured ceilings
// ------------------------------------------------------------------------------------
extern "C" txe_status txe_measure_ceiling(txe_context *ctx, int32_t kind, double *value) {
  if (!ctx || !value) return fail(TXE_ERR_ARG, "null argument");
  if (kind < 0 || kind > 3) return fail(TXE_ERR_ARG, "kind %d not in [0, 3]", kind);
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  HIP_TRY(hipStreamIsCapturing(ctx->stream, &cs));
  if (cs != hipStreamCaptureStatusNone) return fail(TXE_ERR_STATE, "cannot measure while the stream is captured");
  HIP_TRY(hipSetDevice(ctx->device));
  const hipError_t e = measure_ceiling(kind, ctx->stream, value);
  if (e == hipErrorOutOfMemory) {
    (void)hipGetLastError();
    return fail(TXE_ERR_NOMEM, "no memory for the stream buffers");
  }
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}

// ------------------------------------------------------------------------------------
// adaptively compressed exchange
// ------------------------------------------------------------------------------------
extern "C" txe_status txe_ace_build(txe_context *ctx, const txe_system *sys, int32_t N, int32_t dtype,
                                    const void *psi, const void *W, double *xi, double *M_out, double *L_out,
                                    int32_t *info) {
  if (!ctx || !sys || !psi || !W || !xi) return fail(TXE_ERR_ARG, "null argument");
  if (sys->device != ctx->device) return fail(TXE_ERR_ARG, "system and context are on different devices");
  if (N < 1 || N > 2048) return fail(TXE_ERR_SHAPE, "N = %d not in [1, 2048]", N);
  if (dtype != TXE_DTYPE_F64 && dtype != TXE_DTYPE_F32) return fail(TXE_ERR_ARG, "unknown dtype %d", dtype);
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context has a previous device error: %s", ctx->sticky_msg.c_str());
  const size_t elt = dtype == TXE_DTYPE_F64 ? 8 : 4;
  const long long ng = (long long)sys->n[0] * sys->n[1] * sys->n[2];
  const size_t nin = (size_t)N * ng * elt, nxi = (size_t)N * ng * 8, nmat = (size_t)N * N * 8;
  if (((uintptr_t)psi % elt) || ((uintptr_t)W % elt) || ((uintptr_t)xi % 8) || ((uintptr_t)M_out % 8) ||
      ((uintptr_t)L_out % 8) || ((uintptr_t)info % 4))
    return fail(TXE_ERR_ARG, "misaligned pointer");
  if (overlaps(xi, nxi, psi, nin) || overlaps(xi, nxi, W, nin) || overlaps(M_out, nmat, psi, nin) ||
      overlaps(M_out, nmat, W, nin) || overlaps(L_out, nmat, psi, nin) || overlaps(L_out, nmat, W, nin) ||
      overlaps(M_out, nmat, xi, nxi) || overlaps(L_out, nmat, xi, nxi) || overlaps(M_out, nmat, L_out, nmat))
    return fail(TXE_ERR_ARG, "outputs overlap inputs or each other");
  const int nch = gram_nchunks(N, N, ng);
  size_t off = 0;
  const size_t o_part = off; off = align256(off + (size_t)nch * N * N * 8);
  const size_t o_M = off; off = align256(off + nmat);
  const size_t o_L = off; off = align256(off + nmat);
  const size_t o_T = off; off = align256(off + nmat);
  const size_t o_info = off; off = align256(off + 4);
  txe_status st = ensure_workspace(ctx, off);
  if (st != TXE_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  char *ws = (char *)ctx->ws;
  double *M = M_out ? M_out : (double *)(ws + o_M);
  double *L = L_out ? L_out : (double *)(ws + o_L);
  int *inf = info ? (int *)info : (int *)(ws + o_info);
  const bool f64 = dtype == TXE_DTYPE_F64;
  hipError_t e = ace_gram(f64, f64, psi, N, W, N, sys->D, sys->qdev, (double *)(ws + o_part), M, ctx->stream);
  if (e == hipSuccess) e = ace_chol_inv(M, N, L, (double *)(ws + o_T), inf, ctx->stream);
  if (e == hipSuccess) e = ace_comb(f64, true, (const double *)(ws + o_T), N, N, W, ng, 1.0, 1, xi, ctx->stream);
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}

extern "C" txe_status txe_ace_apply(txe_context *ctx, const txe_system *sys, int32_t N, const double *xi,
                                    int32_t Nphi, int32_t dtype, const void *phi, void *out) {
  if (!ctx || !sys || !xi || !phi || !out) return fail(TXE_ERR_ARG, "null argument");
  if (sys->device != ctx->device) return fail(TXE_ERR_ARG, "system and context are on different devices");
  if (N < 1 || N > 2048) return fail(TXE_ERR_SHAPE, "N = %d not in [1, 2048]", N);
  if (Nphi < 1 || Nphi > 65536) return fail(TXE_ERR_SHAPE, "Nphi = %d not in [1, 65536]", Nphi);
  if (dtype != TXE_DTYPE_F64 && dtype != TXE_DTYPE_F32) return fail(TXE_ERR_ARG, "unknown dtype %d", dtype);
  if (ctx->sticky) return fail(TXE_ERR_DEVICE, "context has a previous device error: %s", ctx->sticky_msg.c_str());
  const size_t elt = dtype == TXE_DTYPE_F64 ? 8 : 4;
  const long long ng = (long long)sys->n[0] * sys->n[1] * sys->n[2];
  if (((uintptr_t)xi % 8) || ((uintptr_t)phi % elt) || ((uintptr_t)out % elt))
    return fail(TXE_ERR_ARG, "misaligned pointer");
  const size_t nphi = (size_t)Nphi * ng * elt;
  if (overlaps(out, nphi, phi, nphi) || overlaps(out, nphi, xi, (size_t)N * ng * 8))
    return fail(TXE_ERR_ARG, "out overlaps an input");
  const int nch = gram_nchunks(Nphi, N, ng);
  size_t off = 0;
  const size_t o_part = off; off = align256(off + (size_t)nch * Nphi * N * 8);
  const size_t o_C = off; off = align256(off + (size_t)Nphi * N * 8);
  txe_status st = ensure_workspace(ctx, off);
  if (st != TXE_OK) return st;
  HIP_TRY(hipSetDevice(ctx->device));
  char *ws = (char *)ctx->ws;
  const bool f64 = dtype == TXE_DTYPE_F64;
  double *Ct = (double *)(ws + o_C);  // Ct[j][k] = <phi_j, xi_k>_W
  hipError_t e = ace_gram(f64, true, phi, Nphi, xi, N, sys->D, sys->qdev, (double *)(ws + o_part), Ct, ctx->stream);
  if (e == hipSuccess) e = ace_comb(true, f64, Ct, Nphi, N, xi, ng, -1.0, 0, out, ctx->stream);
  if (e != hipSuccess) return device_failed(ctx, e);
  return ok();
}
