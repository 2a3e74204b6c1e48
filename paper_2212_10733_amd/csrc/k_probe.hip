// Measured ceilings for the roofline figures (measurement infrastructure, not part of
// compression): a streaming copy for the practical HBM rate, and compute loops that keep
// every SIMD busy with independent FP64 fused multiply-adds, FP32 matrix-core operations
// (v_mfma_f32_32x32x2f32) or BF16 matrix-core operations (v_mfma_f32_32x32x16_bf16).
#include "hcz_internal.h"

namespace hcz {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kProbeBlocks = 2048, kProbeThreads = 256, kCopyBlocks = 4096;

__global__ __launch_bounds__(256) void k_probe_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                    long long n4) {
  const long long stride = (long long)gridDim.x * 256;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n4; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(256) void k_probe_fma64(long long iters, double* sink) {
  const int t = threadIdx.x;
  const double b = 1.0 + 1e-12 * t, c = 1e-15;
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = 1.0 + k + t;
  for (long long i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fma(a[k], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  sink[(long long)blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void k_probe_mfma32(long long iters, float* sink) {
  const int t = threadIdx.x;
  const float a = 1.0f + 1e-6f * t, b = 1.0f - 1e-6f * t;
  f32x16 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  for (long long i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[j][r];
  sink[(long long)blockIdx.x * 256 + t] = s;
}

__global__ __launch_bounds__(256) void k_probe_mfma_bf16(long long iters, float* sink) {
  const int t = threadIdx.x;
  bf16x8 a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(1.0f + 0.001f * e);
    b[e] = (__bf16)(1.0f - 0.001f * (t & 7));
  }
  f32x16 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[j][r] = 0.0f;
  for (long long i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < 4; ++j)
#pragma unroll
    for (int r = 0; r < 16; ++r) s += acc[j][r];
  sink[(long long)blockIdx.x * 256 + t] = s;
}

}  // namespace hcz

using namespace hcz;

extern "C" {

hcz_status hcz_probe_sink_bytes(size_t* bytes) {
  if (!bytes) return set_error(HCZ_EINVAL, "NULL argument");
  *bytes = (size_t)kProbeBlocks * kProbeThreads * 8;
  return HCZ_OK;
}

hcz_status hcz_probe_copy(const void* src, void* dst, size_t bytes, hcz_stream_t stream) {
  if (!src || !dst) return set_error(HCZ_EINVAL, "NULL argument");
  if (bytes % 16 || ((uintptr_t)src | (uintptr_t)dst) % 16) return set_error(HCZ_EINVAL, "copy needs 16-byte multiples and alignment");
  if (!bytes) return HCZ_OK;
  hipLaunchKernelGGL(k_probe_copy, dim3(kCopyBlocks), dim3(256), 0, (hipStream_t)stream, (const f32x4*)src,
                     (f32x4*)dst, (long long)(bytes / 16));
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HCZ_OK : set_error(HCZ_EHIP, hipGetErrorString(e));
}

hcz_status hcz_probe_compute(int32_t kind, int64_t iters, void* sink, double* flops, hcz_stream_t stream) {
  if (!sink || !flops) return set_error(HCZ_EINVAL, "NULL argument");
  if (iters < 0) return set_error(HCZ_EINVAL, "iters must be >= 0");
  const double waves = (double)kProbeBlocks * (kProbeThreads / 64);
  hipStream_t st = (hipStream_t)stream;
  if (kind == HCZ_PROBE_FP64_FMA) {
    hipLaunchKernelGGL(k_probe_fma64, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, (long long)iters, (double*)sink);
    *flops = 2.0 * 8.0 * (double)iters * waves * 64.0;
  } else if (kind == HCZ_PROBE_FP32_MFMA) {
    hipLaunchKernelGGL(k_probe_mfma32, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, (long long)iters, (float*)sink);
    *flops = 4.0 * (2.0 * 32 * 32 * 2) * (double)iters * waves;
  } else if (kind == HCZ_PROBE_BF16_MFMA) {
    hipLaunchKernelGGL(k_probe_mfma_bf16, dim3(kProbeBlocks), dim3(kProbeThreads), 0, st, (long long)iters, (float*)sink);
    *flops = 4.0 * (2.0 * 32 * 32 * 16) * (double)iters * waves;
  } else {
    return set_error(HCZ_EINVAL, "unknown probe kind");
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? HCZ_OK : set_error(HCZ_EHIP, hipGetErrorString(e));
}

}  // extern "C"
