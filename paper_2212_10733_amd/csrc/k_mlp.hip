// Warm-start multiplier network (the learned addition to Section III Stage 5):
// lam0 = scale * (W3 relu(W2 relu(W1 zhat + b1) + b2) + b3), zhat = codebook[codes],
// 16 -> 64 -> 64 -> 4.  Inference runs one histogram per thread with the 5,508 weights
// in LDS (every thread reads the same weight: broadcast, no bank conflicts).
#include "hcz_internal.h"

namespace hcz {

constexpr int kMlpIn = 16, kMlpH = 64, kMlpOut = 4;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;

__global__ __launch_bounds__(256) void k_mlp_infer(const float* params, const double* scale,
                                                   const uint8_t* codes, const float* centroids, int kcb,
                                                   long long H, double* lam0) {
  __shared__ float w[kMlpParams];
  for (int k = threadIdx.x; k < kMlpParams; k += 256) w[k] = params[k];
  __syncthreads();
  const long long h = (long long)blockIdx.x * 256 + threadIdx.x;
  if (h >= H) return;
  const float* W1 = w;
  const float* b1 = W1 + kMlpH * kMlpIn;
  const float* W2 = b1 + kMlpH;
  const float* b2 = W2 + kMlpH * kMlpH;
  const float* W3 = b2 + kMlpH;
  const float* b3 = W3 + kMlpOut * kMlpH;
  float z[kMlpIn];
#pragma unroll
  for (int d = 0; d < kMlpIn; ++d) z[d] = centroids[d * kcb + min((int)codes[h * kMlpIn + d], kcb - 1)];
  float h1[kMlpH];
#pragma unroll
  for (int o = 0; o < kMlpH; ++o) {
    float s = b1[o];
#pragma unroll
    for (int d = 0; d < kMlpIn; ++d) s = fmaf(W1[o * kMlpIn + d], z[d], s);
    h1[o] = fmaxf(s, 0.0f);
  }
  float out[kMlpOut];
#pragma unroll
  for (int q = 0; q < kMlpOut; ++q) out[q] = b3[q];
  for (int o = 0; o < kMlpH; ++o) {
    float s = b2[o];
#pragma unroll
    for (int d = 0; d < kMlpH; ++d) s = fmaf(W2[o * kMlpH + d], h1[d], s);
    const float h2 = fmaxf(s, 0.0f);
#pragma unroll
    for (int q = 0; q < kMlpOut; ++q) out[q] = fmaf(W3[q * kMlpH + o], h2, out[q]);
  }
#pragma unroll
  for (int q = 0; q < kMlpOut; ++q) lam0[h * 4 + q] = scale[q] * (double)out[q];
}

// zhat[n][d] = C[d][code[n][d]]
__global__ void k_dequant(const uint8_t* codes, long long n, int latent, const float* centroids, int kcb,
                          float* z) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= n * latent) return;
  const int d = (int)(q % latent);
  z[q] = centroids[(long long)d * kcb + min((int)codes[q], kcb - 1)];
}

int mlp_param_count() { return kMlpParams; }

hipError_t launch_mlp_infer(const float* params, const double* scale, const uint8_t* codes,
                            const float* centroids, int bits, long long H, double* lam0, hipStream_t st) {
  if (H <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, st, params, scale, codes,
                     centroids, 1 << bits, H, lam0);
  return hipGetLastError();
}

hipError_t launch_dequant(const uint8_t* codes, long long n, int latent, const float* centroids, int bits,
                          float* z, hipStream_t st) {
  const long long tot = n * latent;
  if (tot <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_dequant, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, codes, n, latent,
                     centroids, 1 << bits, z);
  return hipGetLastError();
}

}  // namespace hcz
