// Ceiling microbenchmarks: the MFMA rates and the HBM stream rate this device
// actually sustains, the measured denominators next to the published peaks
// in a roofline.  Each MFMA kernel keeps eight independent accumulator
// chains per wavefront (enough to cover the pipeline latency of every shape
// used here) and runs a fixed trip count on operands that differ from lane
// to lane and element to element (hashed values in [0.5, 1.5), as in real
// tiles); the stream kernel reads and writes float4 with a grid-stride loop.
#include <hip/hip_runtime.h>

#include <cstddef>

#include "txe_internal.h"

namespace txe {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int CHAINS = 8;
constexpr int ITERS = 2048;

// an integer hash of x mapped to [0.5, 1.5)
__device__ __forceinline__ float hashed(unsigned x) {
  x ^= x >> 16;
  x *= 0x7feb352du;
  x ^= x >> 15;
  x *= 0x846ca68bu;
  x ^= x >> 16;
  return 0.5f + (float)(x >> 8) * (1.0f / 16777216.0f);
}

__global__ __launch_bounds__(256) void k_peak_f64(double seed, double *out) {
  d4 c[CHAINS];
  const double a = seed * hashed(2 * threadIdx.x), b = seed * hashed(2 * threadIdx.x + 1);
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) c[i] = d4{0.0, 0.0, 0.0, 0.0};
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) c[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[i], 0, 0, 0);
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_f32(float seed, float *out) {
  f4v c[CHAINS];
  const float a = seed * hashed(2 * threadIdx.x), b = seed * hashed(2 * threadIdx.x + 1);
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) c[i] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[i], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_bf16(float seed, float *out) {
  f4v c[CHAINS];
  bf8v a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(seed * hashed(16 * threadIdx.x + i));
    b[i] = (__bf16)(seed * hashed(16 * threadIdx.x + 8 + i));
  }
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) c[i] = f4v{0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < ITERS; ++it)
#pragma unroll
    for (int i = 0; i < CHAINS; ++i) c[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c[i], 0, 0, 0);
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < CHAINS; ++i) s += c[i][0] + c[i][1] + c[i][2] + c[i][3];
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fill(f4v *p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = f4v{v, v, v, v};
}

__global__ __launch_bounds__(256) void k_stream(const f4v *__restrict__ src, f4v *__restrict__ dst, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i] * 2.0f;
}

}  // namespace

// Times `reps` launches of one ceiling kernel on stream s and returns the
// rate: TFLOP/s for the MFMA kinds (0 f64 16x16x4, 1 f32 16x16x4, 2 bf16
// 16x16x32), GB/s (read + write) for kind 3.
hipError_t measure_ceiling(int kind, hipStream_t s, double *value) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int blocks = 4 * ncu, threads = 256, reps = 5;
  void *buf = nullptr, *buf2 = nullptr;
  const size_t sbytes = (size_t)512 << 20;
  const size_t n4 = sbytes / sizeof(f4v);
  if (kind == 3) {
    if ((e = hipMalloc(&buf, sbytes)) != hipSuccess) return e;
    if ((e = hipMalloc(&buf2, sbytes)) != hipSuccess) {
      (void)hipFree(buf);
      return e;
    }
    hipLaunchKernelGGL(k_fill, dim3(blocks * 4), dim3(threads), 0, s, (f4v *)buf, n4, 1.0f);
  } else {
    if ((e = hipMalloc(&buf, (size_t)blocks * threads * sizeof(double))) != hipSuccess) return e;
  }
  auto launch = [&]() {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_peak_f64, dim3(blocks), dim3(threads), 0, s, 1.0, (double *)buf); break;
      case 1: hipLaunchKernelGGL(k_peak_f32, dim3(blocks), dim3(threads), 0, s, 1.0f, (float *)buf); break;
      case 2: hipLaunchKernelGGL(k_peak_bf16, dim3(blocks), dim3(threads), 0, s, 1.0f, (float *)buf); break;
      default: hipLaunchKernelGGL(k_stream, dim3(blocks * 4), dim3(threads), 0, s, (const f4v *)buf, (f4v *)buf2, n4);
    }
  };
  hipEvent_t a = nullptr, z = nullptr;
  if ((e = hipEventCreate(&a)) == hipSuccess && (e = hipEventCreate(&z)) == hipSuccess) {
    launch();  // warm-up
    e = hipEventRecord(a, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) launch();
    if (e == hipSuccess) e = hipGetLastError();
    if (e == hipSuccess) e = hipEventRecord(z, s);
    if (e == hipSuccess) e = hipEventSynchronize(z);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, z);
    if (e == hipSuccess) {
      const double sec = ms * 1e-3 / reps;
      const double waves = (double)blocks * threads / 64;
      // flops of one MFMA: 2 * M * N * K
      const double per = kind == 0 ? 2.0 * 16 * 16 * 4 : kind == 1 ? 2.0 * 16 * 16 * 4 : 2.0 * 16 * 16 * 32;
      if (kind == 3)
        *value = 2.0 * (double)sbytes / sec / 1e9;
      else
        *value = waves * ITERS * CHAINS * per / sec / 1e12;
    }
  }
  if (a) (void)hipEventDestroy(a);
  if (z) (void)hipEventDestroy(z);
  (void)hipStreamSynchronize(s);
  (void)hipFree(buf);
  if (buf2) (void)hipFree(buf2);
  return e;
}

}  // namespace txe
