// Measurement probe (not part of the C ABI of bard.h): the FP32 vector FMA
// throughput this build can reach, for the benchmark's roofline peaks.
// Every lane runs eight independent FMA chains, so issue is never waiting on
// a dependency; built like the library (packed FP32 instructions off), it
// measures the unpacked VALU peak the kernels can use.
#include <hip/hip_runtime.h>

namespace {

__global__ void __launch_bounds__(256) fma_chains(float* out, int iters) {
  const float b = 1.0000001f, c = 1e-7f;
  float a0 = threadIdx.x * 1e-6f, a1 = a0 + 1e-3f, a2 = a0 + 2e-3f, a3 = a0 + 3e-3f;
  float a4 = a0 + 4e-3f, a5 = a0 + 5e-3f, a6 = a0 + 6e-3f, a7 = a0 + 7e-3f;
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      a0 = __builtin_fmaf(a0, b, c);
      a1 = __builtin_fmaf(a1, b, c);
      a2 = __builtin_fmaf(a2, b, c);
      a3 = __builtin_fmaf(a3, b, c);
      a4 = __builtin_fmaf(a4, b, c);
      a5 = __builtin_fmaf(a5, b, c);
      a6 = __builtin_fmaf(a6, b, c);
      a7 = __builtin_fmaf(a7, b, c);
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = a0 + a1 + a2 + a3 + a4 + a5 + a6 + a7;
}

}  // namespace

// Launches `blocks` x 256 threads, each doing iters x 64 FMAs; `out` holds
// blocks * 256 floats.  Returns the FLOP count (2 per FMA), or -1 on a launch
// error.
extern "C" double bard_peak_fma_fp32(float* out, int blocks, int iters, void* stream) {
  hipLaunchKernelGGL(fma_chains, dim3(blocks), dim3(256), 0, (hipStream_t)stream, out, iters);
  if (hipGetLastError() != hipSuccess) return -1.0;
  return 2.0 * 64.0 * (double)iters * 256.0 * (double)blocks;
}
