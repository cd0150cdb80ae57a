// Achievable peaks of the device, the denominators of measured roofline
// fractions: MFMA throughput of the instruction shapes the kernels use (float32
// 16x16x4, bf16 16x16x32, float64 16x16x4; register operands, eight independent
// accumulation chains per wave, every compute unit busy), and the HBM bandwidth
// of a plain grid-stride copy (bytes read + bytes written per second).
#include <algorithm>

#include "kernels.h"

namespace qmc {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int PEAK_CHAINS = 8;

template <int KIND>
__global__ __launch_bounds__(256) void mfma_peak_kernel(float* __restrict__ out, int iters) {
  const float a = threadIdx.x * 1e-3f, b = 1.0f - a;
  float s = 0.f;
  if constexpr (KIND == 0) {
    f4 c[PEAK_CHAINS];
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) c[j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int j = 0; j < PEAK_CHAINS; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c[j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) s += c[j][0];
  } else if constexpr (KIND == 1) {
    bf16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      av[e] = (__bf16)a;
      bv[e] = (__bf16)b;
    }
    f4 c[PEAK_CHAINS];
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) c[j] = f4{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int j = 0; j < PEAK_CHAINS; ++j) c[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, c[j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) s += c[j][0];
  } else {
    d4 c[PEAK_CHAINS];
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) c[j] = d4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it)
#pragma unroll
      for (int j = 0; j < PEAK_CHAINS; ++j)
        c[j] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)a, (double)b, c[j], 0, 0, 0);
#pragma unroll
    for (int j = 0; j < PEAK_CHAINS; ++j) s += (float)c[j][0];
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void copy_peak_kernel(const f4* __restrict__ in, f4* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[i];
}

static int peak_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) ==
                                               hipSuccess && n > 0)
    return n;
  return 256;
}

// Times f on stream st (best of three after one warm-up), in milliseconds; < 0 on a HIP error.
template <typename F>
static float time_best(hipStream_t st, F f) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -1.f;
  float best = -1.f;
  for (int rep = 0; rep < 4; ++rep) {
    if (hipEventRecord(e0, st) != hipSuccess) break;
    f();
    if (hipGetLastError() != hipSuccess || hipEventRecord(e1, st) != hipSuccess ||
        hipEventSynchronize(e1) != hipSuccess)
      break;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) break;
    if (rep > 0 && (best < 0.f || ms < best)) best = ms;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return best;
}

hipError_t measure_peaks(void* scratch, size_t bytes, double* out, hipStream_t st) {
  const int cus = peak_cus();
  const int blocks = 8 * cus, iters = 2000;
  float* sink = (float*)scratch;
  const double per_block = 4.0 * PEAK_CHAINS * iters;  // instructions per block (four waves)
  const double flop[3] = {2.0 * 16 * 16 * 4, 2.0 * 16 * 16 * 32, 2.0 * 16 * 16 * 4};
  for (int k = 0; k < 3; ++k) {
    const float ms = time_best(st, [&] {
      if (k == 0) hipLaunchKernelGGL(mfma_peak_kernel<0>, dim3(blocks), dim3(256), 0, st, sink, iters);
      if (k == 1) hipLaunchKernelGGL(mfma_peak_kernel<1>, dim3(blocks), dim3(256), 0, st, sink, iters);
      if (k == 2) hipLaunchKernelGGL(mfma_peak_kernel<2>, dim3(blocks), dim3(256), 0, st, sink, iters);
    });
    if (ms <= 0.f) return hipErrorUnknown;
    out[k] = flop[k] * per_block * blocks / (ms * 1e-3) / 1e12;
  }
  const int64_t n = (int64_t)(bytes / 2 / sizeof(f4));
  const f4* in = (const f4*)scratch;
  f4* o = (f4*)scratch + n;
  const float ms = time_best(st, [&] {
    hipLaunchKernelGGL(copy_peak_kernel, dim3((unsigned)(4 * cus)), dim3(256), 0, st, in, o, n);
  });
  if (ms <= 0.f) return hipErrorUnknown;
  out[3] = 2.0 * n * sizeof(f4) / (ms * 1e-3) / 1e9;
  return hipSuccess;
}

}  // namespace qmc
