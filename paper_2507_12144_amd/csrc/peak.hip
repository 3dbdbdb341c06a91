// Microbenchmarks of the machine peaks the roofline fractions are quoted
// against, measured on the GPU the library runs on (diagnostics):
//  * HBM: a streaming copy of a large buffer (four float4 loads in flight per
//    thread, grid stride), bytes read + written per second;
//  * FP32 matrix cores: v_mfma_f32_16x16x4_f32 back to back with eight
//    independent accumulators per wave (enough to cover the instruction's
//    latency), 2048 flops each;
//  * BF16 matrix cores: v_mfma_f32_16x16x32_bf16 the same way, 16384 flops
//    each.
// Timed with HIP events around one launch after a warm-up launch.
#include "internal.h"

namespace sht {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Four 16-byte loads in flight per thread before their stores.
__global__ __launch_bounds__(256) void copy_kernel(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
  size_t i = blockIdx.x * static_cast<size_t>(blockDim.x) + threadIdx.x;
  for (; i + 3 * stride < n; i += 4 * stride) {
    const float4 v0 = a[i], v1 = a[i + stride], v2 = a[i + 2 * stride], v3 = a[i + 3 * stride];
    b[i] = v0;
    b[i + stride] = v1;
    b[i + 2 * stride] = v2;
    b[i + 3 * stride] = v3;
  }
  for (; i < n; i += stride) b[i] = a[i];
}

__global__ __launch_bounds__(256) void mfma_f32_loop(int iters, float seed, float* __restrict__ out) {
  floatx4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  const float a = seed + threadIdx.x * 1e-7f, b = seed - threadIdx.x * 1e-7f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  if (s == 1234.5f) out[threadIdx.x] = s;  // never true for these inputs; keeps the loop
}

__global__ __launch_bounds__(256) void mfma_bf16_loop(int iters, float seed, float* __restrict__ out) {
  floatx4 acc[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = static_cast<__bf16>(seed + e * 1e-3f);
    b[e] = static_cast<__bf16>(seed - e * 1e-3f);
  }
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 8; ++i) acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
  if (s == 1234.5f) out[threadIdx.x] = s;
}

}  // namespace

hipError_t measure_peak(int kind, size_t size, double* result, hipStream_t st) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  void* a = nullptr;
  void* b = nullptr;
  double work = 0.0;
  auto launch = [&]() -> hipError_t {
    if (kind == 0) {
      const size_t n = size / sizeof(float4);
      hipLaunchKernelGGL(copy_kernel, dim3(2048), dim3(256), 0, st, static_cast<const float4*>(a),
                         static_cast<float4*>(b), n);
    } else {
      // 4 waves per workgroup, 8 workgroups per CU over 256 CUs
      const int iters = static_cast<int>(size);
      if (kind == 1)
        hipLaunchKernelGGL(mfma_f32_loop, dim3(2048), dim3(256), 0, st, iters, 0.5f, static_cast<float*>(b));
      else
        hipLaunchKernelGGL(mfma_bf16_loop, dim3(2048), dim3(256), 0, st, iters, 0.5f, static_cast<float*>(b));
    }
    return hipGetLastError();
  };
  if (e == hipSuccess) {
    if (kind == 0) {
      e = hipMalloc(&a, size);
      if (e == hipSuccess) e = hipMalloc(&b, size);
      if (e == hipSuccess) e = hipMemsetAsync(a, 0, size, st);
      work = 2.0 * static_cast<double>(size);  // bytes read + written
    } else {
      e = hipMalloc(&b, 256 * sizeof(float));
      const double per = kind == 1 ? 2048.0 : 16384.0;
      work = 2048.0 * 4 * 8 * static_cast<double>(size) * per;  // waves x MFMAs x flops
    }
  }
  if (e == hipSuccess) e = launch();                  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, st);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) *result = work / (ms * 1e-3);
  if (a) (void)hipFree(a);
  if (b) (void)hipFree(b);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return e;
}

}  // namespace sht
