// peak_agpr.hip -- the fp64 matrix-core rate with the accumulators in AGPRs
// (this file is compiled with the compiler's default MFMA register form; the
// library's fp64 kernels and peak.hip use architectural VGPRs, which sustain
// a much higher v_mfma_f64_16x16x4f64 rate on gfx950).  Same loop as kind 5
// of peak.hip: eight independent accumulator chains per wave, four waves per
// SIMD, register operands only.
#include "common.h"

namespace dl {

__global__ void __launch_bounds__(256) k_mfma_peak_f64_agpr(int iters, unsigned seed, int store, int* sink) {
  const unsigned x = seed ^ threadIdx.x;
  const double a = (double)(x & 7) * 0.125;
  v4d acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = v4d{(double)c, 0.0, 0.0, 0.0};
  for (int i = 0; i < iters; ++i)
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc[c], 0, 0, 0);
  double t = 0.0;
  for (auto& c : acc) t += c[0] + c[1] + c[2] + c[3];
  if (store) sink[threadIdx.x] = (int)t;
}

hipError_t launch_peak_f64_agpr(int grid, int iters, int* sink, hipStream_t s) {
  hipLaunchKernelGGL(k_mfma_peak_f64_agpr, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink);
  return hipGetLastError();
}

}  // namespace dl
