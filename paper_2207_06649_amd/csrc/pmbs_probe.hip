// pmbs_probe.hip -- achievable-peak probes of the GPU the library runs on:
// an FP32 multiply-add loop (vector ALU) and a device-to-device copy (HBM).
// The step kernel's roofline fractions are quoted against these next to the
// vendor figures.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "pmbs.h"
#include "pmbs_internal.h"

namespace pmbs {
namespace {

constexpr int CHAINS = 16;  // independent multiply-add chains per lane (hides the ALU latency)

// Every lane runs CHAINS dependent chains of `iters` multiply-adds (2 flop
// each); the sums go to `sink` so the loop is not removed.
__global__ __launch_bounds__(256) void fma_probe_kernel(float* sink, int iters, float a, float b) {
  float acc[CHAINS];
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) acc[k] = (float)(threadIdx.x + k);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < CHAINS; ++k) acc[k] = fmaf(acc[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < CHAINS; ++k) s += acc[k];
  sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

// Grid-stride 16-byte copy.
__global__ __launch_bounds__(256) void copy_probe_kernel(const float4* __restrict__ src, float4* __restrict__ dst,
                                                         size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace
}  // namespace pmbs

using namespace pmbs;

extern "C" {

pmbs_status pmbs_probe_fma(float* d_sink, int32_t blocks, int32_t iters, void* hip_stream, double* flop) {
  if (!d_sink || blocks <= 0 || iters <= 0) return fail(PMBS_ERR_INVALID_ARG, "bad probe arguments");
  hipLaunchKernelGGL(fma_probe_kernel, dim3(blocks), dim3(256), 0, static_cast<hipStream_t>(hip_stream), d_sink,
                     iters, 0.999999f, 1e-7f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "fma probe launch");
  if (flop) *flop = 2.0 * CHAINS * (double)iters * (double)blocks * 256.0;
  return PMBS_OK;
}

pmbs_status pmbs_probe_copy(const void* d_src, void* d_dst, size_t bytes, void* hip_stream) {
  if (!d_src || !d_dst || bytes % 16 != 0 || (reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) % 16)
    return fail(PMBS_ERR_INVALID_ARG, "copy probe needs 16-byte aligned buffers and sizes");
  int dev = 0, cus = 256;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
  hipLaunchKernelGGL(copy_probe_kernel, dim3(cus * 8), dim3(256), 0, static_cast<hipStream_t>(hip_stream),
                     static_cast<const float4*>(d_src), static_cast<float4*>(d_dst), bytes / 16);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "copy probe launch");
  return PMBS_OK;
}

}  // extern "C"
