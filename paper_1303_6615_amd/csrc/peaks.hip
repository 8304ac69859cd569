// Microbenchmarks of the rates the hot path is priced against: FP32 and FP64
// vector FMA throughput and LDS read bandwidth, measured on the device the
// library runs on (diagnostics; aparareal_measure_peaks).
#include <hip/hip_runtime.h>

#include "launch.hpp"

namespace ap {
namespace {

constexpr int kChains = 16;      // independent FMA chains per lane
constexpr int kPeakThreads = 256;

// kChains independent chains x = x * a + b per lane and iteration; the result
// is written so that nothing is dead.  2 kChains flops per lane per iteration.
template <typename T>
__global__ void __launch_bounds__(kPeakThreads) k_fma_peak(T* out, int iters, T a, T b) {
  T x[kChains];
#pragma unroll
  for (int j = 0; j < kChains; ++j) x[j] = T(threadIdx.x) * T(1e-3) + T(j);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < kChains; ++j) x[j] = x[j] * a + b;
  }
  T s = T(0);
#pragma unroll
  for (int j = 0; j < kChains; ++j) s += x[j];
  out[blockIdx.x * kPeakThreads + threadIdx.x] = s;
}

// Conflict-free 64-bit LDS reads: lane l of a wavefront reads element
// (base + l) of a 32 KiB array, 8 reads per iteration at different bases.
__global__ void __launch_bounds__(kPeakThreads) k_lds_peak(float* out, int iters) {
  __shared__ float2 buf[4096];
  for (int i = threadIdx.x; i < 4096; i += kPeakThreads) buf[i] = make_float2(float(i), float(-i));
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  float acc = 0.0f;
  int base = wave * 512;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) acc += buf[(base + j * 64 + lane) & 4095].x;
    base = (base + 1024) & 4095;
  }
  out[blockIdx.x * kPeakThreads + threadIdx.x] = acc;
}

template <typename K>
hipError_t time_ms(K&& launch, hipStream_t s, float* ms) {
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  if (e == hipSuccess) e = launch();                         // warm-up
  if (e == hipSuccess) e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return e;
}

}  // namespace

hipError_t measure_peaks(void* scratch, size_t scratch_bytes, hipStream_t s, double* fp32_tflops,
                         double* fp64_tflops, double* lds_tbps) {
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  const int blocks = cus * 16;                                // 16 workgroups of 4 wavefronts per CU
  if (scratch_bytes < size_t(blocks) * kPeakThreads * sizeof(double)) return hipErrorInvalidValue;
  const int iters = 4096;
  float ms = 0.0f;
  const double lanes = double(blocks) * kPeakThreads;
  e = time_ms([&] {
    hipLaunchKernelGGL(k_fma_peak<float>, dim3(blocks), dim3(kPeakThreads), 0, s, static_cast<float*>(scratch), iters,
                       0.999f, 1e-4f);
    return hipGetLastError();
  }, s, &ms);
  if (e != hipSuccess) return e;
  *fp32_tflops = lanes * iters * 2.0 * kChains / (ms * 1e-3) / 1e12;
  e = time_ms([&] {
    hipLaunchKernelGGL(k_fma_peak<double>, dim3(blocks), dim3(kPeakThreads), 0, s, static_cast<double*>(scratch),
                       iters, 0.999, 1e-4);
    return hipGetLastError();
  }, s, &ms);
  if (e != hipSuccess) return e;
  *fp64_tflops = lanes * iters * 2.0 * kChains / (ms * 1e-3) / 1e12;
  e = time_ms([&] {
    hipLaunchKernelGGL(k_lds_peak, dim3(blocks), dim3(kPeakThreads), 0, s, static_cast<float*>(scratch), iters);
    return hipGetLastError();
  }, s, &ms);
  if (e != hipSuccess) return e;
  *lds_tbps = lanes * iters * 8.0 * sizeof(float2) / (ms * 1e-3) / 1e12;
  return hipSuccess;
}

}  // namespace ap
