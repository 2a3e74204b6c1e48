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
// read; ReLU(acc + b) in FP32 stored to the h2 buffer in flattening order (channel-major).
// The dense 6400 -> 16 layer (k_conv_fc) runs over 32 histograms per workgroup on
// v_mfma_f32_16x16x4f32.
// Decoder (k_conv_dec): hd = relu(db + sum_d zhat_d dw[:, d]) as an FP32 chain, rounded to
// bfloat16 into LDS as [y][x][channel] (10 x 10 plus a zero row and column); the
// transposed conv1 (64 -> 32, stride 2, output padding 1) as an implicit GEMM per output
// parity class: an output cell of parity (cy, cx) receives 1, 2 or 4 taps, K = taps x 64;
// ReLU(acc + b) in FP32 to LDS [y][x][channel]; the transposed conv2 (32 -> 1) on the
// vector ALUs; fhat = sigma y + mu.
#include <algorithm>

#include "hcz_internal.h"

namespace hcz {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

constexpr int kCP1 = 40;   // LDS pitch (bfloat16) of a conv1 output cell (32 channels)
constexpr int kCPD = 72;   // LDS pitch (bfloat16) of a decoder hidden cell (64 channels)
constexpr int kCP3 = 36;   // LDS pitch (floats) of a transposed-conv1 output cell (32 channels, 16-byte rows)
constexpr int kConvGrid = 1024;  // workgroups of the looping decoder kernel
constexpr int kConvEncGrid = 512; // workgroups of the looping encoder kernel (two per CU)

__device__ __forceinline__ f32x16 mfma_bf16c(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// A workgroup loops over histograms (h = blockIdx.x, + gridDim.x, ...) with conv2's
// weights staged once in LDS; 77 KB of LDS lets two share a CU.  The input is staged with
// a zero border, so every tap of conv1 reads a value: a padding tap adds a zero product,
// which leaves the chain's value as skipping it would (only the sign of an exact-zero
// sum can differ, and ReLU makes it a zero either way).  Each histogram's input is loaded while the
// previous one is convolved.
template <typename TIn>
__global__ __launch_bounds__(256, 2) void k_conv_enc(ModelDev M, const TIn* hist, long long n, long long hs,
                                                     long long rs, float* h2out) {
  __shared__ float xs[41 * 41];                                        // x at (iy + 1, ix + 1)
  __shared__ __attribute__((aligned(16))) __bf16 h1p[21 * 21 * kCP1];
  __shared__ __attribute__((aligned(16))) __bf16 w2s[9 * 64 * 32];      // conv2 weights [tap][out][in]
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int li = l & 31, kh = l >> 5;
  {
    const bf16x8* src = (const bf16x8*)M.c2w;
    for (int q = t; q < 9 * 64 * 32 / 8; q += 256) ((bf16x8*)w2s)[q] = src[q];
  }
  for (int q = t; q < 41 * 41; q += 256) {
    const int y = q / 41, x = q - 41 * y;
    if (y == 0 || y == 40 || x == 0 || x == 40) xs[q] = 0.0f;
  }
  // zero border of the conv1 output (row 0 and column 0 of the padded layout), which
  // conv1 never writes
  for (int q = t; q < 41 * 32; q += 256) {
    const int cell = q >> 5, c = q & 31;
    const int cy = cell < 21 ? 0 : cell - 20, cx = cell < 21 ? cell : 0;
    h1p[(cy * 21 + cx) * kCP1 + c] = (__bf16)0.0f;
  }
  // conv1's weights: thread -> channels 8 cg .. 8 cg + 7
  const int cg = t & 3;
  float wv1[8][9], bv1[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
#pragma unroll
    for (int k = 0; k < 9; ++k) wv1[c][k] = M.c1w[(8 * cg + c) * 9 + k];
    bv1[c] = M.c1b[8 * cg + c];
  }
  // the thread's six input cells: z-score factors and padded LDS index
  float mv[6], rv[6];
  int xo[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int e = min(t + 256 * q, 1520);
    const int j = e / 39, i = e - 39 * j;
    mv[q] = M.mu[e];
    rv[q] = M.rsd[e];
    xo[q] = (j + 1) * 41 + i + 1;
  }
  TIn fv[6];
  auto load_f = [&](long long hh) {
    const TIn* f = hist + hh * hs;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int e = min(t + 256 * q, 1520);
      const int j = e / 39, i = e - 39 * j;
      fv[q] = f[j * rs + i];
    }
  };
  if ((long long)blockIdx.x < n) load_f(blockIdx.x);
  for (long long h = blockIdx.x; h < n; h += gridDim.x) {
  __syncthreads();          // the previous histogram is done with xs and h1p
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (t + 256 * q < 1521) {
      const float v = (float)fv[q];
      xs[xo[q]] = ((isfinite(v) ? v : 0.0f) - mv[q]) * rv[q];
    }
  }
  load_f(min(h + (long long)gridDim.x, n - 1));     // unconditional: the waits stay exact
  __syncthreads();
  // conv1: thread -> channels 8 cg .. 8 cg + 7 of positions p = t / 4 + 64 q; the nine
  // taps are read first, then every channel's chain runs over them in row-major order
  for (int p = t >> 2; p < 400; p += 64) {
    const int oy = p / 20, ox = p - 20 * oy;
    const float* xb = &xs[2 * oy * 41 + 2 * ox];
    float xv[9];
#pragma unroll
    for (int ky = 0; ky < 3; ++ky)
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) xv[3 * ky + kx] = xb[ky * 41 + kx];
    float s[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) s[c] = bv1[c];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
      for (int c = 0; c < 8; ++c) s[c] = fmaf(xv[k], wv1[c][k], s[c]);
    bf16x8 o;
#pragma unroll
    for (int c = 0; c < 8; ++c) o[c] = (__bf16)fmaxf(s[c], 0.0f);
    *(bf16x8*)&h1p[((oy + 1) * 21 + (ox + 1)) * kCP1 + 8 * cg] = o;
  }
  __syncthreads();
  // conv2 on matrix cores: wave w owns output positions 32 w .. 32 w + 31
  const int P = min(32 * w + li, 99);
  const int oy2 = P / 10, ox2 = P - 10 * oy2;
  f32x16 acc[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[nt][r] = 0.0f;
#pragma unroll
  for (int tap = 0; tap < 9; ++tap) {
    const int ky = tap / 3, kx = tap - 3 * ky;
    const __bf16* arow = &h1p[((2 * oy2 + ky) * 21 + (2 * ox2 + kx)) * kCP1];
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const bf16x8 a = *(const bf16x8*)(arow + 16 * half + 8 * kh);
#pragma unroll
      for (int nt = 0; nt < 2; ++nt)
        acc[nt] = mfma_bf16c(a, *(const bf16x8*)(w2s + (tap * 64 + 32 * nt + li) * 32 + 16 * half + 8 * kh),
                             acc[nt]);
    }
  }
  // ReLU(acc + b) straight to h2 in flattening order (channel-major): the lane's four
  // consecutive rows 8 g + 4 kh .. + 3 of channel co are one 16-byte store (100 rows per
  // channel, so a group of four is all in range or all out)
  float* dst = h2out + h * 6400;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const int co = 32 * nt + li;
    const float bias = M.c2b[co];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int row = 32 * w + 8 * g + 4 * kh;
      if (row < 100) {
        float4 v;
        v.x = fmaxf(acc[nt][4 * g] + bias, 0.0f);
        v.y = fmaxf(acc[nt][4 * g + 1] + bias, 0.0f);
        v.z = fmaxf(acc[nt][4 * g + 2] + bias, 0.0f);
        v.w = fmaxf(acc[nt][4 * g + 3] + bias, 0.0f);
        *(float4*)(dst + co * 100 + row) = v;
      }
    }
  }
  }
}

// z[h][o] = fb[o] + sum_k h2[h][k] fw[o][k] on v_mfma_f32_16x16x4f32: a workgroup takes 32
// histograms as two 16-row tiles that share every fw operand, its four waves a quarter of
// K = 6400 each.  Per 16-wide k step lane l holds k = 16 c + 4 (l / 16) .. + 3 of row
// l % 16 of each operand (one 16-byte load each; the products are summed in this lane
// order, which the operands share), and the four partial tiles are added in wave order.
__global__ __launch_bounds__(256) void k_conv_fc(const float* h2, long long n, const float* fw, const float* fb,
                                                 float* z) {
  __shared__ float part[4][2][16 * 16];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, lr = l & 15, lq = l >> 4;
  const long long r0 = (long long)blockIdx.x * 32;
  const long long row0 = min(r0 + lr, n - 1), row1 = min(r0 + 16 + lr, n - 1);
  constexpr int kSteps = 6400 / 16 / 4;          // 16-wide k steps per wave
  const f32x4* a0 = (const f32x4*)(h2 + row0 * 6400 + (long long)w * (6400 / 4) + 4 * lq);
  const f32x4* a1 = (const f32x4*)(h2 + row1 * 6400 + (long long)w * (6400 / 4) + 4 * lq);
  const f32x4* b = (const f32x4*)(fw + (long long)lr * 6400 + w * (6400 / 4) + 4 * lq);
  f32x4 acc0 = {0.0f, 0.0f, 0.0f, 0.0f}, acc1 = {0.0f, 0.0f, 0.0f, 0.0f};
  f32x4 an0[4], an1[4], bn[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    an0[u] = a0[4 * u];
    an1[u] = a1[4 * u];
    bn[u] = b[4 * u];
  }
  for (int c = 0; c < kSteps; c += 4) {
    f32x4 av0[4], av1[4], bv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av0[u] = an0[u];
      av1[u] = an1[u];
      bv[u] = bn[u];
    }
    if (c + 4 < kSteps) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        an0[u] = a0[4 * (c + 4 + u)];
        an1[u] = a1[4 * (c + 4 + u)];
        bn[u] = b[4 * (c + 4 + u)];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        acc0 = __builtin_amdgcn_mfma_f32_16x16x4f32(av0[u][e], bv[u][e], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(av1[u][e], bv[u][e], acc1, 0, 0, 0);
      }
  }
  // D layout: lane l holds rows 4 (l / 16) + r, column l % 16
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    part[w][0][(4 * lq + r) * 16 + lr] = acc0[r];
    part[w][1][(4 * lq + r) * 16 + lr] = acc1[r];
  }
  __syncthreads();
#pragma unroll
  for (int tile = 0; tile < 2; ++tile) {
    const int q = t;                             // 256 outputs: row q / 16, column q % 16
    const long long hr = r0 + 16 * tile + q / 16;
    if (hr < n)
      z[hr * kLatent + (q & 15)] =
          fb[q & 15] + (((part[0][tile][q] + part[1][tile][q]) + part[2][tile][q]) + part[3][tile][q]);
  }
}

// Decoder hidden layer: hd = bf16(relu(db[k] + sum_d zhat[h][d] dw[k][d])) as the FP32
// chain over d = 0..15, for unit k = channel * 100 + position, stored position-major:
// hd[h][position * 64 + channel] (the layout the decoder stages into LDS).  A workgroup
// of 320 threads takes 1,280 consecutive stored units, four per thread (their dw rows in
// registers, one 8-byte store per histogram), for 64 histograms; five workgroups cover
// the 6,400 units.
constexpr int kHidThreads = 320;
__global__ __launch_bounds__(kHidThreads) void k_conv_hidden(ModelDev M, const uint8_t* codes,
                                                             const float* centroids, int kcb, long long n,
                                                             __bf16* hd) {
  __shared__ __attribute__((aligned(16))) float zs[64 * kLatent];
  const int t = threadIdx.x;
  const long long h0 = (long long)blockIdx.y * 64;
  for (int q = t; q < 64 * kLatent; q += kHidThreads) {
    const long long hh = h0 + q / kLatent;
    const int d = q % kLatent;
    zs[q] = hh < n ? centroids[d * kcb + min((int)codes[hh * kLatent + d], kcb - 1)] : 0.0f;
  }
  __syncthreads();
  const int ks0 = 4 * (blockIdx.x * kHidThreads + t);   // stored index of the first unit
  float wv[4][kLatent], bv[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int ks = ks0 + j;
    const int k = (ks & 63) * 100 + (ks >> 6);          // unit: channel * 100 + position
    const f32x4* dw = (const f32x4*)(M.dw + (long long)k * kLatent);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f32x4 q4 = dw[u];
#pragma unroll
      for (int e = 0; e < 4; ++e) wv[j][4 * u + e] = q4[e];
    }
    bv[j] = M.db[k];
  }
  const int m = (int)min((long long)64, n - h0);
  for (int r = 0; r < m; ++r) {
    float s[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) s[j] = bv[j];
#pragma unroll
    for (int d = 0; d < kLatent; ++d) {
      const float zd = zs[r * kLatent + d];
#pragma unroll
      for (int j = 0; j < 4; ++j) s[j] = fmaf(zd, wv[j][d], s[j]);
    }
    bf16x4 o;
#pragma unroll
    for (int j = 0; j < 4; ++j) o[j] = (__bf16)fmaxf(s[j], 0.0f);
    *(bf16x4*)&hd[(h0 + r) * 6400 + ks0] = o;
  }
}

// Lane l's float x from its quad partner: CTRL 0xB1 swaps lanes 0 <-> 1 and 2 <-> 3 of
// every quad, 0x4E lanes 0 <-> 2 and 1 <-> 3.
template <int CTRL>
__device__ __forceinline__ float quad_swap(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Transposed conv1, parity class CLS = (cy, cx) = (CLS / 2, CLS % 2): an output cell of
// that parity receives (1 + cy) (1 + cx) taps; even output -> k = 1 from input p, odd
// output -> k = 0 from p + 1 and k = 2 from p.  Tap ty, tx of the class is ky = 1 (cy = 0)
// or ky = 0, 2 (ty = 0, 1), likewise kx.
template <int CLS>
__device__ __forceinline__ void tconv1_weights(const __bf16* T1, int li, int kh, int zo,
                                               bf16x8 (&b)[(1 + CLS / 2) * (1 + CLS % 2)][4]) {
  constexpr int cy = CLS >> 1, cx = CLS & 1;
#pragma unroll
  for (int ty = 0; ty < 1 + cy; ++ty)
#pragma unroll
    for (int tx = 0; tx < 1 + cx; ++tx) {
      const int ky = cy ? (ty == 0 ? 0 : 2) : 1, kx = cx ? (tx == 0 ? 0 : 2) : 1;
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4)
        b[ty * (1 + cx) + tx][c4] =
            *(const bf16x8*)(T1 + ((long long)((ky * 3 + kx) * 32 + li)) * 64 + 16 * c4 + 8 * kh + zo);
    }
}

// The class's matrix-core steps for the wave's 32 positions (position q = (py, px) on
// this lane's row of the A operand), then ReLU(acc + b) to h3s [y][x][channel].
template <int CLS>
__device__ __forceinline__ void tconv1_class(const __bf16* hdp, float* h3s,
                                             const bf16x8 (&b)[(1 + CLS / 2) * (1 + CLS % 2)][4], int py, int px,
                                             int w, int li, int kh, float bias1) {
  constexpr int cy = CLS >> 1, cx = CLS & 1;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
  for (int ty = 0; ty < 1 + cy; ++ty) {
    const int iy = cy ? (ty == 0 ? py + 1 : py) : py;
#pragma unroll
    for (int tx = 0; tx < 1 + cx; ++tx) {
      const int ix = cx ? (tx == 0 ? px + 1 : px) : px;
      const __bf16* arow = &hdp[(iy * 11 + ix) * kCPD];
#pragma unroll
      for (int c4 = 0; c4 < 4; ++c4)
        acc = mfma_bf16c(*(const bf16x8*)(arow + 16 * c4 + 8 * kh), b[ty * (1 + cx) + tx][c4], acc);
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

// A workgroup loops over histograms like the encoder.  Per histogram, the transposed conv1
// weights of each parity class are issued one class ahead of its matrix-core steps, and
// the next histogram's hidden layer is loaded while this one is computed.
__global__ __launch_bounds__(256, 2) void k_conv_dec(ModelDev M, const __bf16* hd, long long n, float* fhat) {
  __shared__ __attribute__((aligned(16))) __bf16 hdp[11 * 11 * kCPD];
  __shared__ __attribute__((aligned(16))) float h3s[20 * 20 * kCP3];
  __shared__ __attribute__((aligned(16))) float t2v[9 * 32];     // transposed conv2 weights [tap][channel]
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const int li = l & 31, kh = l >> 5;
  for (int q = t; q < 9 * 32; q += 256) t2v[(q % 9) * 32 + q / 9] = M.t2w[q];   // t2w[ci][tap]
  const __bf16* T1 = (const __bf16*)M.t1w;
  const float bias1 = M.t1b[li];
  const float bias2 = M.t2b[0];
  // the hidden layer of a histogram: 800 16-byte chunks ([position][channel], 8 channels each)
  bf16x8 hv[4];
  auto load_hd = [&](long long hh) {
    const bf16x8* src = (const bf16x8*)(hd + hh * 6400);
#pragma unroll
    for (int r = 0; r < 4; ++r) hv[r] = src[min(t + 256 * r, 799)];
  };
  if ((long long)blockIdx.x < n) load_hd(blockIdx.x);
  const int q = min(32 * w + li, 99);
  const int py = q / 10, px = q - 10 * py;
  for (long long h = blockIdx.x; h < n; h += gridDim.x) {
  // a zero the compiler cannot see through: the weight loads below stay inside the loop
  // instead of being hoisted (holding them across iterations would not fit the registers)
  int zo = 0;
  asm volatile("" : "+v"(zo));
  // transposed conv1's weights by parity class, each class's issued one class ahead of
  // its matrix-core steps (classes 0 and 1 before the hidden layer is staged)
  bf16x8 wb0[1][4], wb1[2][4], wb2[2][4], wb3[4][4];
  tconv1_weights<0>(T1, li, kh, zo, wb0);
  tconv1_weights<1>(T1, li, kh, zo, wb1);
  __syncthreads();          // the previous histogram is done with hdp and h3s
  // the hidden layer into [y][x][channel], and zeros in row 10 and column 10 (the output
  // of the previous histogram went over part of the buffer)
  if (t < 21 * 8) {
    const int cell = t >> 3;
    const int y = cell < 11 ? 10 : cell - 11, x = cell < 11 ? cell : 10;
    bf16x8 z;
#pragma unroll
    for (int c = 0; c < 8; ++c) z[c] = (__bf16)0.0f;
    *(bf16x8*)&hdp[(y * 11 + x) * kCPD + 8 * (t & 7)] = z;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int m = t + 256 * r;
    if (m >= 800) continue;
    const int p = m >> 3, y = p / 10, x = p - 10 * y;
    *(bf16x8*)&hdp[(y * 11 + x) * kCPD + 8 * (m & 7)] = hv[r];
  }
  load_hd(min(h + (long long)gridDim.x, n - 1));    // unconditional: the waits stay exact
  __syncthreads();
  // transposed conv1 on matrix cores, one parity class (cy, cx) at a time; wave w owns
  // the class's positions 32 w .. 32 w + 31 (of 100)
  tconv1_class<0>(hdp, h3s, wb0, py, px, w, li, kh, bias1);
  tconv1_weights<2>(T1, li, kh, zo, wb2);
  tconv1_class<1>(hdp, h3s, wb1, py, px, w, li, kh, bias1);
  tconv1_weights<3>(T1, li, kh, zo, wb3);
  tconv1_class<2>(hdp, h3s, wb2, py, px, w, li, kh, bias1);
  tconv1_class<3>(hdp, h3s, wb3, py, px, w, li, kh, bias1);
  __syncthreads();
  // transposed conv2 (32 -> 1) on the vector ALUs.  A quad of lanes takes one 2 x 2 output
  // block, lane cq of the quad channels 8 cq .. 8 cq + 7: output (2m + a, 2n + b) takes
  // input cells (m, n), (m, n + 1), (m + 1, n), (m + 1, n + 1) with taps ky = 1 (a = 0) or
  // ky = 0 from row m + 1 and ky = 2 from row m (a = 1), likewise kx.  The quad then sums
  // its four channel groups with two swaps, lane cq keeping output cq = 2a + b, which goes
  // to LDS; sigma y + mu is written out afterwards in natural order.  Row and column 39 do
  // not exist, so cells past 19 are never needed (clamped reads, outputs skipped).
  {
    const int cq = t & 3;
    float wt[9][8];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const float4 u0 = *(const float4*)&t2v[k * 32 + 8 * cq + zo];
      const float4 u1 = *(const float4*)&t2v[k * 32 + 8 * cq + 4 + zo];
      wt[k][0] = u0.x; wt[k][1] = u0.y; wt[k][2] = u0.z; wt[k][3] = u0.w;
      wt[k][4] = u1.x; wt[k][5] = u1.y; wt[k][6] = u1.z; wt[k][7] = u1.w;
    }
    // sigma and mu of the six outputs this thread writes at the end (o = t + 256 k)
    float sdv[6], muv[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int o = min(t + 256 * k, 1520) + zo;
      sdv[k] = M.sd[o];
      muv[k] = M.mu[o];
    }
    float* ys = (float*)hdp;     // y before sigma and mu; the hidden layer is no longer read
#pragma unroll 1
    for (int task = t >> 2; task < 400; task += 64) {
      const int m = task / 20, nn = task - 20 * m;
      const int m1 = min(m + 1, 19), n1 = min(nn + 1, 19);
      const float* c00 = &h3s[(m * 20 + nn) * kCP3 + 8 * cq];
      const float* c01 = &h3s[(m * 20 + n1) * kCP3 + 8 * cq];
      const float* c10 = &h3s[(m1 * 20 + nn) * kCP3 + 8 * cq];
      const float* c11 = &h3s[(m1 * 20 + n1) * kCP3 + 8 * cq];
      float v00[8], v01[8], v10[8], v11[8];
#pragma unroll
      for (int hq = 0; hq < 2; ++hq) {
        const float4 a = *(const float4*)(c00 + 4 * hq), b = *(const float4*)(c01 + 4 * hq);
        const float4 c = *(const float4*)(c10 + 4 * hq), d = *(const float4*)(c11 + 4 * hq);
        v00[4 * hq] = a.x; v00[4 * hq + 1] = a.y; v00[4 * hq + 2] = a.z; v00[4 * hq + 3] = a.w;
        v01[4 * hq] = b.x; v01[4 * hq + 1] = b.y; v01[4 * hq + 2] = b.z; v01[4 * hq + 3] = b.w;
        v10[4 * hq] = c.x; v10[4 * hq + 1] = c.y; v10[4 * hq + 2] = c.z; v10[4 * hq + 3] = c.w;
        v11[4 * hq] = d.x; v11[4 * hq + 1] = d.y; v11[4 * hq + 2] = d.z; v11[4 * hq + 3] = d.w;
      }
      float see = 0.0f, seo = 0.0f, soe = 0.0f, soo = 0.0f;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        see = fmaf(v00[c], wt[4][c], see);
        seo = fmaf(v01[c], wt[3][c], seo);
        seo = fmaf(v00[c], wt[5][c], seo);
        soe = fmaf(v10[c], wt[1][c], soe);
        soe = fmaf(v00[c], wt[7][c], soe);
        soo = fmaf(v11[c], wt[0][c], soo);
        soo = fmaf(v10[c], wt[2][c], soo);
        soo = fmaf(v01[c], wt[6][c], soo);
        soo = fmaf(v00[c], wt[8][c], soo);
      }
      // transposed reduction over the quad: after the first swap lane cq holds, summed over
      // its pair, the outputs of column b = cq & 1; after the second, output cq
      const bool odd = (cq & 1) != 0, high = (cq & 2) != 0;
      const float r0 = (odd ? seo : see) + quad_swap<0xB1>(odd ? see : seo);
      const float r1 = (odd ? soo : soe) + quad_swap<0xB1>(odd ? soe : soo);
      const float v = (high ? r1 : r0) + quad_swap<0x4E>(high ? r0 : r1);
      const int oy = 2 * m + (high ? 1 : 0), ox = 2 * nn + (odd ? 1 : 0);
      if (oy < 39 && ox < 39) ys[oy * 39 + ox] = v;
    }
    __syncthreads();
    float* out = fhat + h * 1521;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int o = t + 256 * k;
      if (o < 1521) out[o] = fmaf(sdv[k], ys[o] + bias2, muv[k]);
    }
  }
  }
}

// Both directions run in chunks of at most kConvChunk histograms through the model's
// scratch buffer (conv2 output, FP32; the decoder's hidden layer, bfloat16).
hipError_t launch_conv_encode(const ModelDev& M, const void* hist, int dtype, long long H, long long hs,
                              long long rs, float* z, hipStream_t st) {
  for (long long c0 = 0; c0 < H; c0 += kConvChunk) {
    const long long n = std::min((long long)kConvChunk, H - c0);
    const dim3 eg((unsigned)std::min(n, (long long)kConvEncGrid));
    if (dtype == HCZ_F32)
      hipLaunchKernelGGL(k_conv_enc<float>, eg, dim3(256), 0, st, M, (const float*)hist + c0 * hs, n, hs, rs,
                         M.scratch);
    else
      hipLaunchKernelGGL(k_conv_enc<double>, eg, dim3(256), 0, st, M, (const double*)hist + c0 * hs, n, hs, rs,
                         M.scratch);
    hipLaunchKernelGGL(k_conv_fc, dim3((unsigned)((n + 31) / 32)), dim3(256), 0, st, (const float*)M.scratch, n,
                       M.fw, M.fb, z + c0 * kLatent);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_conv_decode(const ModelDev& M, const uint8_t* codes, const float* centroids, int bits,
                              long long H, float* fhat, hipStream_t st) {
  __bf16* hd = (__bf16*)M.scratch;
  for (long long c0 = 0; c0 < H; c0 += kConvChunk) {
    const long long n = std::min((long long)kConvChunk, H - c0);
    static_assert(5 * kHidThreads * 4 == 6400, "the hidden layer's workgroups cover its units exactly");
    hipLaunchKernelGGL(k_conv_hidden, dim3(5, (unsigned)((n + 63) / 64)), dim3(kHidThreads), 0, st, M,
                       codes + c0 * kLatent, centroids, 1 << bits, n, hd);
    hipLaunchKernelGGL(k_conv_dec, dim3((unsigned)std::min(n, (long long)kConvGrid)), dim3(256), 0, st, M,
                       (const __bf16*)hd, n, fhat + c0 * 1521);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


// ---- training of the convolutional model (Section III Stage 2, Eq. 5) -----------------------
// Generic batched layers, one thread per output value, FP32 fused multiply-adds; the
// training path favours plainness over speed.  Layout [b][channel][y][x].  BF = true is
// the BF16 training form: both operands of every product are rounded to the nearest
// bfloat16 (ties to even) before the multiply, whose result is then exact in FP32, and
// the sums stay FP32 (FP64 in the weight gradients); biases are not rounded.

template <bool BF>
__device__ __forceinline__ float opnd(float v) {
  if constexpr (BF) return (float)(__bf16)v;
  else return v;
}

// 3x3 convolution, stride 2, padding 1: out[b][o][oy][ox] = bias[o] + sum over c and the
// in-range taps of in'[b][c][2oy-1+ky][2ox-1+kx] w[o][c][ky][kx]; in' = relu(in) if relu_in.
template <bool BF>
__global__ __launch_bounds__(256) void k_cv_fwd(const float* in, int C, int n, int relu_in, const float* w,
                                                const float* bias, float* out, int O, int m, long long B) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= B * O * m * m) return;
  const int ox = (int)(q % m), oy = (int)((q / m) % m), o = (int)((q / ((long long)m * m)) % O);
  const long long b = q / ((long long)m * m * O);
  float s = bias ? bias[o] : 0.0f;
  for (int c = 0; c < C; ++c) {
    const float* ip = in + ((b * C + c) * n) * n;
    const float* wp = w + (o * C + c) * 9;
    for (int ky = 0; ky < 3; ++ky) {
      const int iy = 2 * oy - 1 + ky;
      if (iy < 0 || iy >= n) continue;
      for (int kx = 0; kx < 3; ++kx) {
        const int ix = 2 * ox - 1 + kx;
        if (ix < 0 || ix >= n) continue;
        float v = ip[iy * n + ix];
        if (relu_in) v = fmaxf(v, 0.0f);
        s = fmaf(opnd<BF>(v), opnd<BF>(wp[ky * 3 + kx]), s);
      }
    }
  }
  out[q] = s;
}

// 3x3 transposed convolution, stride 2, padding 1, output m x m: out[b][o][oy][ox] =
// bias[o] + sum over c and the taps with oy = 2 iy - 1 + ky (iy in range) of in'[b][c][iy][ix] w[c][o][ky][kx].
template <bool BF>
__global__ __launch_bounds__(256) void k_cvt_fwd(const float* in, int C, int n, int relu_in, const float* w,
                                                 const float* bias, float* out, int O, int m, long long B) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= B * O * m * m) return;
  const int ox = (int)(q % m), oy = (int)((q / m) % m), o = (int)((q / ((long long)m * m)) % O);
  const long long b = q / ((long long)m * m * O);
  float s = bias ? bias[o] : 0.0f;
  for (int c = 0; c < C; ++c) {
    const float* ip = in + ((b * C + c) * n) * n;
    const float* wp = w + (c * O + o) * 9;
    for (int ky = 0; ky < 3; ++ky) {
      const int ny = oy + 1 - ky;
      if (ny < 0 || (ny & 1) || (ny >> 1) >= n) continue;
      for (int kx = 0; kx < 3; ++kx) {
        const int nx = ox + 1 - kx;
        if (nx < 0 || (nx & 1) || (nx >> 1) >= n) continue;
        float v = ip[(ny >> 1) * n + (nx >> 1)];
        if (relu_in) v = fmaxf(v, 0.0f);
        s = fmaf(opnd<BF>(v), opnd<BF>(wp[ky * 3 + kx]), s);
      }
    }
  }
  out[q] = s;
}

// Weight gradient of a stride-2 3x3 layer: G[cc][cf][ky][kx] = sum over b and coarse cells
// (py, px) of coarse'[b][cc][py][px] fine'[b][cf][2py-1+ky][2px-1+kx] (in-range cells).
// For a convolution coarse = dL/d(output), fine = its input; for a transposed one coarse =
// its input, fine = dL/d(output).  One workgroup per (cc, cf), FP64 partial sums.
template <bool BF>
__global__ __launch_bounds__(256) void k_cv_wgrad(const float* coarse, int Cc, int m, int relu_c, const float* fine,
                                                  int Cf, int n, int relu_f, long long B, float* G) {
  __shared__ double red[9][256];
  const int cc = blockIdx.x / Cf, cf = blockIdx.x % Cf, t = threadIdx.x;
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int mm = m * m;
  // thread t takes the flattened (sample, coarse pixel) indices t, t + 256, ...; the sample
  // and pixel advance incrementally instead of by 64-bit division
  long long b = t / mm;
  int pix = t - (int)b * mm;
  for (; b < B;) {
    const int py = pix / m, px = pix - py * m;
    float cv = coarse[(b * Cc + cc) * mm + pix];
    if (relu_c) cv = fmaxf(cv, 0.0f);
    cv = opnd<BF>(cv);
    if (cv != 0.0f) {
      const float* fp = fine + ((b * Cf + cf) * n) * n;
#pragma unroll
      for (int ky = 0; ky < 3; ++ky) {
        const int iy = 2 * py - 1 + ky;
        if (iy < 0 || iy >= n) continue;
#pragma unroll
        for (int kx = 0; kx < 3; ++kx) {
          const int ix = 2 * px - 1 + kx;
          if (ix < 0 || ix >= n) continue;
          float fv = fp[iy * n + ix];
          if (relu_f) fv = fmaxf(fv, 0.0f);
          acc[ky * 3 + kx] += (double)cv * (double)opnd<BF>(fv);
        }
      }
    }
    pix += 256;
    while (pix >= mm) {
      pix -= mm;
      ++b;
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) red[k][t] = acc[k];
  __syncthreads();
  for (int wdt = 128; wdt > 0; wdt >>= 1) {
    if (t < wdt)
#pragma unroll
      for (int k = 0; k < 9; ++k) red[k][t] += red[k][t + wdt];
    __syncthreads();
  }
  if (t < 9) G[(cc * Cf + cf) * 9 + t] = (float)red[t][0];
}

// out[c] = sum over b and p of d[b][c][p] (P cells per channel), FP64; one workgroup per c.
__global__ __launch_bounds__(256) void k_chsum(const float* d, int C, int P, long long B, float* out) {
  __shared__ double red[256];
  const int c = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  // flattened (sample, cell) indices t, t + 256, ..., advanced without 64-bit division
  long long b = t / P;
  int i = t - (int)b * P;
  for (; b < B;) {
    s += (double)d[(b * C + c) * P + i];
    i += 256;
    while (i >= P) {
      i -= P;
      ++b;
    }
  }
  red[t] = s;
  __syncthreads();
  for (int wdt = 128; wdt > 0; wdt >>= 1) {
    if (t < wdt) red[t] += red[t + wdt];
    __syncthreads();
  }
  if (t == 0) out[c] = (float)red[0];
}

__global__ __launch_bounds__(256) void k_relu_copy(const float* a, float* h, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n) h[i] = fmaxf(a[i], 0.0f);
}

static unsigned nblk(long long n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_cv_fwd(const float* in, int C, int n, int relu_in, const float* w, const float* bias, float* out,
                         int O, int m, long long B, hipStream_t st, int bf) {
  if (B <= 0) return hipSuccess;
  if (bf)
    hipLaunchKernelGGL(k_cv_fwd<true>, dim3(nblk(B * O * m * m)), dim3(256), 0, st, in, C, n, relu_in, w, bias, out, O,
                       m, B);
  else
    hipLaunchKernelGGL(k_cv_fwd<false>, dim3(nblk(B * O * m * m)), dim3(256), 0, st, in, C, n, relu_in, w, bias, out,
                       O, m, B);
  return hipGetLastError();
}

hipError_t launch_cvt_fwd(const float* in, int C, int n, int relu_in, const float* w, const float* bias, float* out,
                          int O, int m, long long B, hipStream_t st, int bf) {
  if (B <= 0) return hipSuccess;
  if (bf)
    hipLaunchKernelGGL(k_cvt_fwd<true>, dim3(nblk(B * O * m * m)), dim3(256), 0, st, in, C, n, relu_in, w, bias, out,
                       O, m, B);
  else
    hipLaunchKernelGGL(k_cvt_fwd<false>, dim3(nblk(B * O * m * m)), dim3(256), 0, st, in, C, n, relu_in, w, bias, out,
                       O, m, B);
  return hipGetLastError();
}

hipError_t launch_cv_wgrad(const float* coarse, int Cc, int m, int relu_c, const float* fine, int Cf, int n,
                           int relu_f, long long B, float* G, hipStream_t st, int bf) {
  if (bf)
    hipLaunchKernelGGL(k_cv_wgrad<true>, dim3((unsigned)(Cc * Cf)), dim3(256), 0, st, coarse, Cc, m, relu_c, fine, Cf,
                       n, relu_f, B, G);
  else
    hipLaunchKernelGGL(k_cv_wgrad<false>, dim3((unsigned)(Cc * Cf)), dim3(256), 0, st, coarse, Cc, m, relu_c, fine,
                       Cf, n, relu_f, B, G);
  return hipGetLastError();
}

hipError_t launch_chsum(const float* d, int C, int P, long long B, float* out, hipStream_t st) {
  hipLaunchKernelGGL(k_chsum, dim3((unsigned)C), dim3(256), 0, st, d, C, P, B, out);
  return hipGetLastError();
}

hipError_t launch_relu_copy(const float* a, float* h, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_copy, dim3(nblk(n)), dim3(256), 0, st, a, h, n);
  return hipGetLastError();
}

}  // namespace hcz
