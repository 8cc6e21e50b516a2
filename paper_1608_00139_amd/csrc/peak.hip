// peak.hip -- measured matrix-core throughput of this device, the reference
// the step kernels' rates are compared with besides the datasheet figure.
// Built with MFMA accumulators in architectural VGPRs (the library's fp64
// kernels use the same form; kind 8, in peak_agpr.hip, is the fp64 loop with
// AGPR accumulators).
// Every wave runs chains of independent MFMAs on register operands (no memory
// traffic inside the loop); the operands come from a kernel argument and the
// results are stored only under a run-time flag that is never set, so the
// compiler keeps every product.
#include "common.h"

namespace dl {

constexpr int kPeakChains = 8;  // independent accumulators per wave (4 for int8)

template <int KIND>
__global__ void __launch_bounds__(256) k_mfma_peak(int iters, unsigned seed, int store, int* sink) {
  const unsigned x = seed ^ threadIdx.x;
  if constexpr (KIND == 0) {  // int8 32x32x32 (the faster of the two int8 shapes on gfx950)
    v4i a = {(int)x, (int)(x * 3u), (int)(x * 5u), (int)(x * 7u)};
    v16i acc[kPeakChains / 2];
#pragma unroll
    for (int c = 0; c < kPeakChains / 2; ++c) {
      acc[c] = v16i{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      acc[c][0] = c;
    }
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kPeakChains / 2; ++c) acc[c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, a, acc[c], 0, 0, 0);
    int t = 0;
#pragma unroll
    for (int c = 0; c < kPeakChains / 2; ++c) t += acc[c][0] + acc[c][15];
    if (store) sink[threadIdx.x] = t;
  } else if constexpr (KIND == 1) {  // fp32 16x16x4
    const float a = (float)(x & 7) * 0.125f;
    v4f acc[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = v4f{(float)c, 0.f, 0.f, 0.f};  // distinct chains
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, acc[c], 0, 0, 0);
    float t = 0.f;
    for (auto& c : acc) t += c[0] + c[1] + c[2] + c[3];
    if (store) sink[threadIdx.x] = (int)t;
  } else if constexpr (KIND == 2) {  // bf16 16x16x32
    v8bf a;
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = (__bf16)(float)((x >> k) & 1);
    v4f acc[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = v4f{(float)c, 0.f, 0.f, 0.f};  // distinct chains
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, a, acc[c], 0, 0, 0);
    float t = 0.f;
    for (auto& c : acc) t += c[0] + c[1] + c[2] + c[3];
    if (store) sink[threadIdx.x] = (int)t;
  } else if constexpr (KIND == 3 || KIND == 4) {  // fp8 e4m3 / fp4 e2m1, 16x16x128 with unit scales
    v8i a = {(int)x, (int)(x * 3u), (int)(x * 5u), (int)(x * 7u), (int)(x * 9u), (int)(x * 11u), (int)(x * 13u),
             (int)(x * 15u)};
    if constexpr (KIND == 4) a[4] = a[5] = a[6] = a[7] = 0;
    v4f acc[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = v4f{(float)c, 0.f, 0.f, 0.f};  // distinct chains
    constexpr int fmt = KIND == 3 ? 0 : 4;
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c)
        acc[c] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, a, acc[c], fmt, fmt, 0, 127, 0, 127);
    float t = 0.f;
    for (auto& c : acc) t += c[0] + c[1] + c[2] + c[3];
    if (store) sink[threadIdx.x] = (int)t;
  } else {  // fp64 16x16x4
    const double a = (double)(x & 7) * 0.125;
    v4d acc[kPeakChains];
#pragma unroll
    for (int c = 0; c < kPeakChains; ++c) acc[c] = v4d{(double)c, 0.0, 0.0, 0.0};  // distinct chains
    for (int i = 0; i < iters; ++i)
#pragma unroll
      for (int c = 0; c < kPeakChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc[c], 0, 0, 0);
    double t = 0.0;
    for (auto& c : acc) t += c[0] + c[1] + c[2] + c[3];
    if (store) sink[threadIdx.x] = (int)t;
  }
}

// LDS read throughput: every wave reads 1 KB per ds_read_b128 (lane l the
// 16 bytes at 16 l of a 1 KB row, so the 64 lanes cover all banks once per
// quarter-wave), eight independent reads per loop iteration from rows that
// rotate through a 32 KB region; the values are folded into a register so
// no read is dropped.
__global__ void __launch_bounds__(256) k_lds_read_peak(int iters, int store, int* sink) {
  __shared__ __attribute__((aligned(16))) u32x4 buf[2048];  // 32 KB
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < 2048; i += 256) buf[i] = u32x4{(unsigned)i, (unsigned)i * 3u, (unsigned)i * 5u, (unsigned)i * 7u};
  __syncthreads();
  u32x4 acc = {0u, 0u, 0u, 0u};
  int row = wave * 8;
  for (int i = 0; i < iters; ++i) {
    u32x4 v[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[((row + r) & 31) * 64 + lane];
#pragma unroll
    for (int r = 0; r < 8; ++r) acc ^= v[r];
    row += 8;
  }
  if (store) sink[tid] = (int)(acc[0] ^ acc[1] ^ acc[2] ^ acc[3]);
}

// Global-to-LDS fill throughput (global_load_lds_dwordx4, the step kernel's
// operand path): every wave moves 1 KB per instruction from a 1 MB buffer
// (L2-resident after the first pass) into its own 8 KB of LDS, eight
// instructions per wait.
__global__ void __launch_bounds__(256) k_lds_fill_peak(const uint8_t* src, int iters, int store, int* sink) {
  __shared__ __attribute__((aligned(16))) uint8_t buf[32768];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const size_t first = (size_t)(blockIdx.x * 4 + wave) * 8192;
  for (int i = 0; i < iters; ++i) {
    const uint8_t* g = src + (first + (size_t)i * 8192) % (1 << 20);  // 8 KB blocks of the 1 MB buffer
#pragma unroll
    for (int r = 0; r < 8; ++r)
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(g + r * 1024 + lane * 16),
                                       (__attribute__((address_space(3))) void*)(buf + wave * 8192 + r * 1024), 16, 0,
                                       0);
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  if (store) sink[tid] = buf[tid];
}

hipError_t launch_peak_f64_agpr(int grid, int iters, int* sink, hipStream_t s);  // peak_agpr.hip

// Operations per wave and loop iteration (2 M N K per instruction).
static double mfma_ops(int kind) {
  switch (kind) {
    case 0: return 2.0 * 32 * 32 * 32 * (kPeakChains / 2);
    case 1: return 2.0 * 16 * 16 * 4 * kPeakChains;
    case 2: return 2.0 * 16 * 16 * 32 * kPeakChains;
    case 3:
    case 4: return 2.0 * 16 * 16 * 128 * kPeakChains;
    default: return 2.0 * 16 * 16 * 4 * kPeakChains;
  }
}

// Bytes per second of kind 6 (LDS reads) or 7 (global-to-LDS fill), four
// 256-thread workgroups per compute unit; src: 1 MB of device memory.
static hipError_t measure_lds(int kind, const uint8_t* src, int* sink, double* bytes_per_s, hipStream_t s, int cus) {
  const int grid = 4 * cus;
  const int iters = kind == 6 ? 8192 : 2048;
  auto launch = [&]() {
    if (kind == 6) hipLaunchKernelGGL(k_lds_read_peak, dim3(grid), dim3(256), 0, s, iters, 0, sink);
    else hipLaunchKernelGGL(k_lds_fill_peak, dim3(grid), dim3(256), 0, s, src, iters, 0, sink);
    return hipGetLastError();
  };
  hipError_t e;
  if ((e = launch()) != hipSuccess) return e;
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  const int reps = 5;
  (void)hipEventRecord(a, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
  (void)hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return e;
  const double bytes = (double)grid * 4 * iters * 8 * 1024 * reps;  // waves x iterations x 8 KB
  *bytes_per_s = bytes / (ms * 1e-3);
  return hipSuccess;
}

hipError_t measure_peak(int kind, int* sink, double* ops_per_s, hipStream_t s, const uint8_t* src) {
  int dev = 0, cus = 0;
  hipError_t e;
  if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
  if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
  if (kind == 6 || kind == 7) return measure_lds(kind, src, sink, ops_per_s, s, cus);
  // four 256-thread workgroups per CU (four waves per SIMD), two for int8
  const int grid = (kind == 0 ? 2 : 4) * cus;
  auto launch = [&](int iters) {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_mfma_peak<0>, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink); break;
      case 1: hipLaunchKernelGGL(k_mfma_peak<1>, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink); break;
      case 2: hipLaunchKernelGGL(k_mfma_peak<2>, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink); break;
      case 3: hipLaunchKernelGGL(k_mfma_peak<3>, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink); break;
      case 4: hipLaunchKernelGGL(k_mfma_peak<4>, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink); break;
      case 8: return launch_peak_f64_agpr(grid, iters, sink, s);
      default: hipLaunchKernelGGL(k_mfma_peak<5>, dim3(grid), dim3(256), 0, s, iters, 12345u, 0, sink); break;
    }
    return hipGetLastError();
  };
  const int iters = (kind == 1 || kind == 5 || kind == 8) ? 1024 : 4096;
  if ((e = launch(iters)) != hipSuccess) return e;  // warm-up (clocks, code load)
  hipEvent_t a, b;
  if ((e = hipEventCreate(&a)) != hipSuccess) return e;
  if ((e = hipEventCreate(&b)) != hipSuccess) {
    (void)hipEventDestroy(a);
    return e;
  }
  const int reps = 5;
  (void)hipEventRecord(a, s);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch(iters);
  (void)hipEventRecord(b, s);
  if (e == hipSuccess) e = hipEventSynchronize(b);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e != hipSuccess) return e;
  const double waves = (double)grid * 4;
  const double ops = mfma_ops(kind) * (double)iters * waves * reps;
  *ops_per_s = ops / (ms * 1e-3);
  return hipSuccess;
}

}  // namespace dl
