// Convolutional autoencoder for 39 x 39 histograms, BF16 form (Section III Stage 2, the
// autoencoder of Stages 2-3 in its convolutional variant).  One workgroup of 256 threads
// (four waves) per histogram.
//
// Encoder (k_conv_enc): x = (f - mu) / sigma in FP32 -> LDS; conv1 (3x3, 1 -> 32, stride
// 2) on the vector ALUs as an FP32 fused multiply-add chain over the in-range taps in
// row-major order, ReLU, rounded to bfloat16 into LDS as [y+1][x+1][channel] with a zero
// border; conv2 (3x3, 32 -> 64, stride 2) as an implicit GEMM on v_mfma_f32_32x32x16_bf16:
// rows = the 100 output positions (four 32-row tiles, one per wave), columns = 64 output
// channels, K = 9 taps x 32 input channels, each lane's eight operands one 16-byte LDS
// read; ReLU(acc + b) in FP32 to LDS in flattening order (channel-major); the dense
// 6400 -> 16 layer on the vector ALUs (16 lanes per output, shuffle reduction).
// Decoder (k_conv_dec): hd = relu(db + sum_d zhat_d dw[:, d]) as an FP32 chain, rounded to
// bfloat16 into LDS as [y][x][channel] (10 x 10 plus a zero row and column); the
// transposed conv1 (64 -> 32, stride 2, output padding 1) as an implicit GEMM per output
// parity class: an output cell of parity (cy, cx) receives 1, 2 or 4 taps, K = taps x 64;
// ReLU(acc + b) in FP32 to LDS [y][x][channel]; the transposed conv2 (32 -> 1) on the
// vector ALUs; fhat = sigma y + mu.
#include "hcz_internal.h"

namespace hcz {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kCP1 = 40;   // LDS pitch (bfloat16) of a conv1 output cell (32 channels)
constexpr int kCPD = 72;   // LDS pitch (bfloat16) of a decoder hidden cell (64 channels)
constexpr int kCP3 = 33;   // LDS pitch (floats) of a transposed-conv1 output cell (32 channels)

__device__ __forceinline__ f32x16 mfma_bf16c(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

template <typename TIn>
__global__ __launch_bounds__(256, 2) void k_conv_enc(ModelDev M, const TIn* hist, long long hs, long long rs,
                                                     float* z) {
  __shared__ float xs[39 * 39];
  __shared__ __attribute__((aligned(16))) __bf16 h1p[21 * 21 * kCP1];   // later: h2 (6400 floats)
  float* h2s = (float*)h1p;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h = blockIdx.x;
  const TIn* f = hist + h * hs;
  for (int e = t; e < 1521; e += 256) {
    const int j = e / 39, i = e - 39 * j;
    float fv = (float)f[j * rs + i];
    if (!isfinite(fv)) fv = 0.0f;
    xs[e] = (fv - M.mu[e]) * M.rsd[e];
  }
  // zero border of the conv1 output (row 0 and column 0 of the padded layout)
  for (int q = t; q < 41 * 32; q += 256) {
    const int cell = q >> 5, c = q & 31;
    const int cy = cell < 21 ? 0 : cell - 20, cx = cell < 21 ? cell : 0;
    h1p[(cy * 21 + cx) * kCP1 + c] = (__bf16)0.0f;
  }
  __syncthreads();
  // conv1: thread -> channel c = t % 32, positions p = t / 32 + 8 q
  {
    const int c = t & 31;
    float wv[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) wv[k] = M.c1w[c * 9 + k];
    const float bv = M.c1b[c];
    for (int p = t >> 5; p < 400; p += 8) {
      const int oy = p / 20, ox = p - 20 * oy;
      float s = bv;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const int iy = 2 * oy - 1 + ky;
        if (iy < 0 || iy >= 39) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int ix = 2 * ox - 1 + kx;
          if (ix < 0 || ix >= 39) continue;
          s = fmaf(xs[iy * 39 + ix], wv[ky * 3 + kx], s);
        }
      }
      h1p[((oy + 1) * 21 + (ox + 1)) * kCP1 + c] = (__bf16)fmaxf(s, 0.0f);
    }
  }
  __syncthreads();
  // conv2 on matrix cores: wave w owns output positions 32 w .. 32 w + 31
  const int li = l & 31, kh = l >> 5;
  const int P = min(32 * w + li, 99);
  const int oy2 = P / 10, ox2 = P - 10 * oy2;
  const __bf16* W2 = (const __bf16*)M.c2w;
  f32x16 acc[2];
#pragma unroll
  for (int n = 0; n < 2; ++n)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[n][r] = 0.0f;
#pragma unroll 3
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap - 3 * ky;
    const __bf16* arow = &h1p[((2 * oy2 + ky) * 21 + (2 * ox2 + kx)) * kCP1];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int ci0 = 16 * half + 8 * kh;
      const bf16x8 a = *(const bf16x8*)(arow + ci0);
#pragma unroll
      for (int n = 0; n < 2; ++n) {
        const bf16x8 b = *(const bf16x8*)(W2 + ((long long)(tap * 64 + 32 * n + li)) * 32 + ci0);
        acc[n] = mfma_bf16c(a, b, acc[n]);
      }
    }
  }
  __syncthreads();          // every wave is done reading h1p before h2 overwrites it
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const int co = 32 * n + li;
    const float bias = M.c2b[co];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * w + 8 * (r >> 2) + 4 * kh + (r & 3);
      if (row < 100) h2s[co * 100 + row] = fmaxf(acc[n][r] + bias, 0.0f);
    }
  }
  __syncthreads();
  // dense 6400 -> 16: 16 lanes per output
  {
    const int o = t >> 4, sl = t & 15;
    const float* fw = M.fw + (long long)o * 6400;
    float s = 0.0f;
    for (int k = sl; k < 6400; k += 16) s = fmaf(fw[k], h2s[k], s);
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) s += __shfl_xor(s, m, 16);
    if (sl == 0) z[h * kLatent + o] = s + M.fb[o];
  }
}

__global__ __launch_bounds__(256, 2) void k_conv_dec(ModelDev M, const uint8_t* codes, const float* centroids,
                                                     int kcb, float* fhat) {
  __shared__ __attribute__((aligned(16))) __bf16 hdp[11 * 11 * kCPD];
  __shared__ __attribute__((aligned(16))) float h3s[20 * 20 * kCP3];
  __shared__ float zs[kLatent];
  __shared__ float t2s[32 * 9];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h = blockIdx.x;
  if (t < kLatent) zs[t] = centroids[t * kcb + min((int)codes[h * kLatent + t], kcb - 1)];
  for (int q = t; q < 32 * 9; q += 256) t2s[q] = M.t2w[q];
  // zero row 10 and column 10 of the padded hidden layout
  for (int q = t; q < 21 * 64; q += 256) {
    const int cell = q >> 6, c = q & 63;
    const int y = cell < 11 ? 10 : cell - 11, x = cell < 11 ? cell : 10;
    hdp[(y * 11 + x) * kCPD + c] = (__bf16)0.0f;
  }
  __syncthreads();
  // dense 16 -> 6400 as the FP32 chain over d = 0..15, ReLU, bfloat16
  for (int k = t; k < 6400; k += 256) {
    const f32x4* dw = (const f32x4*)(M.dw + (long long)k * kLatent);
    float s = M.db[k];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f32x4 wv = dw[u];
#pragma unroll
      for (int e = 0; e < 4; ++e) s = fmaf(zs[4 * u + e], wv[e], s);
    }
    const int c = k / 100, p = k - 100 * c, y = p / 10, x = p - 10 * y;
    hdp[(y * 11 + x) * kCPD + c] = (__bf16)fmaxf(s, 0.0f);
  }
  __syncthreads();
  // transposed conv1 on matrix cores, one parity class (cy, cx) at a time; wave w owns
  // the class's positions 32 w .. 32 w + 31 (of 100)
  const int li = l & 31, kh = l >> 5;
  const int q = min(32 * w + li, 99);
  const int py = q / 10, px = q - 10 * py;
  const __bf16* T1 = (const __bf16*)M.t1w;
  const float bias1 = M.t1b[li];
#pragma unroll
  for (int cls = 0; cls < 4; ++cls) {
    const int cy = cls >> 1, cx = cls & 1;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    // taps: even output -> k = 1 from input p; odd output -> k = 0 from p + 1, k = 2 from p
#pragma unroll
    for (int ty = 0; ty < 1 + cy; ++ty) {
      const int ky = cy ? (ty == 0 ? 0 : 2) : 1;
      const int iy = cy ? (ty == 0 ? py + 1 : py) : py;
#pragma unroll
      for (int tx = 0; tx < 1 + cx; ++tx) {
        const int kx = cx ? (tx == 0 ? 0 : 2) : 1;
        const int ix = cx ? (tx == 0 ? px + 1 : px) : px;
        const __bf16* arow = &hdp[(iy * 11 + ix) * kCPD];
        const __bf16* brow = T1 + ((long long)((ky * 3 + kx) * 32 + li)) * 64;
#pragma unroll
        for (int c4 = 0; c4 < 4; ++c4) {
          const int ci0 = 16 * c4 + 8 * kh;
          acc = mfma_bf16c(*(const bf16x8*)(arow + ci0), *(const bf16x8*)(brow + ci0), acc);
        }
      }
    }
    // D layout: lane holds output channel li for 16 of the wave's 32 positions
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * w + 8 * (r >> 2) + 4 * kh + (r & 3);
      if (row < 100) {
        const int ry = row / 10, rx = row - 10 * ry;
        const int oy = 2 * ry + cy, ox = 2 * rx + cx;
        h3s[(oy * 20 + ox) * kCP3 + li] = fmaxf(acc[r] + bias1, 0.0f);
      }
    }
  }
  __syncthreads();
  // transposed conv2 (32 -> 1) on the vector ALUs: output (oy, ox) takes input
  // (iy, ix) = ((oy + 1 - ky) / 2, (ox + 1 - kx) / 2) where that is whole and in range
  const float b2 = M.t2b[0];
  for (int o = t; o < 1521; o += 256) {
    const int oy = o / 39, ox = o - 39 * oy;
    float s = 0.0f;
#pragma unroll
    for (int ky = 0; ky < 3; ++ky) {
      const int ny = oy + 1 - ky;
      if (ny < 0 || (ny & 1) || (ny >> 1) >= 20) continue;
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int nx = ox + 1 - kx;
        if (nx < 0 || (nx & 1) || (nx >> 1) >= 20) continue;
        const float* cell = &h3s[((ny >> 1) * 20 + (nx >> 1)) * kCP3];
#pragma unroll 8
        for (int ci = 0; ci < 32; ++ci) s = fmaf(cell[ci], t2s[ci * 9 + ky * 3 + kx], s);
      }
    }
    fhat[h * 1521 + o] = fmaf(M.sd[o], s + b2, M.mu[o]);
  }
}

hipError_t launch_conv_encode(const ModelDev& M, const void* hist, int dtype, long long H, long long hs,
                              long long rs, float* z, hipStream_t st) {
  if (H <= 0) return hipSuccess;
  if (dtype == HCZ_F32)
    hipLaunchKernelGGL(k_conv_enc<float>, dim3((unsigned)H), dim3(256), 0, st, M, (const float*)hist, hs, rs, z);
  else
    hipLaunchKernelGGL(k_conv_enc<double>, dim3((unsigned)H), dim3(256), 0, st, M, (const double*)hist, hs, rs, z);
  return hipGetLastError();
}

hipError_t launch_conv_decode(const ModelDev& M, const uint8_t* codes, const float* centroids, int bits,
                              long long H, float* fhat, hipStream_t st) {
  if (H <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_conv_dec, dim3((unsigned)H), dim3(256), 0, st, M, codes, centroids, 1 << bits, fhat);
  return hipGetLastError();
}

}  // namespace hcz
