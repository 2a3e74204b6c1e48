// Autoencoder training kernels (Section III Stage 2, Eq. 5; Section IV-C): a strided FP32 or
// BF16 matrix-core GEMM used for every forward and backward product of the dense model, ReLU
// masks, column sums for bias gradients, the MSE loss with its gradient, Adam, and the
// per-pixel z-score statistics (Section IV-D).  All reductions run in a fixed order, so
// a training step is bitwise repeatable.
#include "hcz_internal.h"

namespace hcz {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 64;      // GEMM tile (M and N)
constexpr int kGK = 32;      // K chunk
constexpr int kGP = 36;      // LDS pitch

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
constexpr int kGPB = 40;     // LDS pitch (bfloat16 elements) of the BF16 tiles

// C[m][n] = alpha * sum_k A(m,k) B(k,n) + beta * C[m][n] (+ bias[n]) (relu), with
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn], C[m*scm + n].
// BF = false: FP32 operands on v_mfma_f32_32x32x2f32.  BF = true: both operands rounded to
// the nearest bfloat16 (ties to even) as they are staged, products on
// v_mfma_f32_32x32x16_bf16 (exact products, FP32 accumulation); alpha, beta, bias and the
// ReLU stay FP32.
template <bool BF>
__global__ __launch_bounds__(256) void k_gemm(const float* A, long long sam, long long sak,
                                              const float* B, long long sbk, long long sbn,
                                              float* C, long long scm, long long M, long long Nc,
                                              long long K, float alpha, float beta,
                                              const float* bias, int relu) {
  __shared__ __attribute__((aligned(16))) float As[BF ? 1 : kGT * kGP];
  __shared__ __attribute__((aligned(16))) float Bs[BF ? 1 : kGT * kGP];
  __shared__ __attribute__((aligned(16))) __bf16 Ab[BF ? kGT * kGPB : 8];
  __shared__ __attribute__((aligned(16))) __bf16 Bb[BF ? kGT * kGPB : 8];
  const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 31, lh = l >> 5;
  const long long m0 = (long long)blockIdx.x * kGT, n0 = (long long)blockIdx.y * kGT;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
  const bool ak = sak == 1, bk = sbk == 1;
  for (long long k0 = 0; k0 < K; k0 += kGK) {
    if constexpr (BF) {
      // pairs of k per thread, packed into one 32-bit LDS store
#pragma unroll
      for (int it = 0; it < 4; ++it) {
        const int idx = t + 256 * it;
        int mm, kp;
        if (ak) { mm = idx >> 4; kp = idx & 15; } else { mm = idx & 63; kp = idx >> 6; }
        const long long gm = m0 + mm, gk = k0 + 2 * kp;
        const float a0 = (gm < M && gk < K) ? A[gm * sam + gk * sak] : 0.0f;
        const float a1 = (gm < M && gk + 1 < K) ? A[gm * sam + (gk + 1) * sak] : 0.0f;
        int nn, kq;
        if (bk) { nn = idx >> 4; kq = idx & 15; } else { nn = idx & 63; kq = idx >> 6; }
        const long long gn = n0 + nn, gkb = k0 + 2 * kq;
        const float b0 = (gn < Nc && gkb < K) ? B[gkb * sbk + gn * sbn] : 0.0f;
        const float b1 = (gn < Nc && gkb + 1 < K) ? B[(gkb + 1) * sbk + gn * sbn] : 0.0f;
        *(bf16x2*)&Ab[mm * kGPB + 2 * kp] = bf16x2{(__bf16)a0, (__bf16)a1};
        *(bf16x2*)&Bb[nn * kGPB + 2 * kq] = bf16x2{(__bf16)b0, (__bf16)b1};
      }
    } else {
#pragma unroll
      for (int it = 0; it < 8; ++it) {
        const int idx = t + 256 * it;
        int mm, kk;
        if (ak) { mm = idx >> 5; kk = idx & 31; } else { mm = idx & 63; kk = idx >> 6; }
        const long long gm = m0 + mm, gk = k0 + kk;
        As[mm * kGP + (kk & 1) * 16 + (kk >> 1)] = (gm < M && gk < K) ? A[gm * sam + gk * sak] : 0.0f;
        int nn, kb;
        if (bk) { nn = idx >> 5; kb = idx & 31; } else { nn = idx & 63; kb = idx >> 6; }
        const long long gn = n0 + nn, gkb = k0 + kb;
        Bs[nn * kGP + (kb & 1) * 16 + (kb >> 1)] = (gn < Nc && gkb < K) ? B[gkb * sbk + gn * sbn] : 0.0f;
      }
    }
    __syncthreads();
    if constexpr (BF) {
      // lane l: row (col) l % 32 of the wave's tile, k = 16 s + 8 (l / 32) + e
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 a = *(const bf16x8*)&Ab[(wm + li) * kGPB + 16 * s + 8 * lh];
        const bf16x8 b = *(const bf16x8*)&Bb[(wn + li) * kGPB + 16 * s + 8 * lh];
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    } else {
      const f32x4* pa = (const f32x4*)&As[(wm + li) * kGP + lh * 16];
      const f32x4* pb = (const f32x4*)&Bs[(wn + li) * kGP + lh * 16];
      f32x4 av[4], bv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) { av[u] = pa[u]; bv[u] = pb[u]; }
#pragma unroll
      for (int s = 0; s < 16; ++s)
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(av[s >> 2][s & 3], bv[s >> 2][s & 3], acc, 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const long long gm = m0 + wm + 8 * (r >> 2) + 4 * lh + (r & 3);
    const long long gn = n0 + wn + li;
    if (gm < M && gn < Nc) {
      float v = alpha * acc[r];
      if (beta != 0.0f) v = v + beta * C[gm * scm + gn];
      if (bias) v = v + bias[gn];
      if (relu) v = fmaxf(v, 0.0f);
      C[gm * scm + gn] = v;
    }
  }
}

// d = d * (h > 0)
__global__ void k_relu_mask(float* d, const float* h, long long n) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < n && !(h[i] > 0.0f)) d[i] = 0.0f;
}

// out[n] = sum_m D[m][n], FP64 accumulation in a fixed order: a workgroup takes 32
// columns; its 8 row groups g sum rows m = g, g + 8, ... in order, then the 8 partial sums
// are added in order g = 0..7.
__global__ __launch_bounds__(256) void k_colsum(const float* D, long long M, long long Nc, float* out) {
  __shared__ double part[8][32];
  const int c = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long long n = (long long)blockIdx.x * 32 + c;
  double s = 0.0;
  if (n < Nc)
    for (long long m = g; m < M; m += 8) s += (double)D[m * Nc + n];
  part[g][c] = s;
  __syncthreads();
  if (g == 0 && n < Nc) {
    double t = part[0][c];
#pragma unroll
    for (int q = 1; q < 8; ++q) t += part[q][c];
    out[n] = (float)t;
  }
}

// dxh = 2 (xh - x) / n and per-block partial sums of (xh - x)^2.
__global__ __launch_bounds__(256) void k_mse_partial(const float* xh, const float* x, long long n,
                                                     float* dxh, double* partial) {
  __shared__ double red[4];
  double s = 0.0;
  const float sc = (float)(2.0 / (double)n);
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const float e = xh[i] - x[i];
    if (dxh) dxh[i] = sc * e;
    s += (double)e * (double)e;
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

// loss = (sum of the partials) / n: 256 threads sum strided partials in order, then a
// fixed pairwise tree.
__global__ __launch_bounds__(256) void k_mse_final(const double* partial, int nb, long long n, float* loss) {
  __shared__ double red[256];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int i = t; i < nb; i += 256) s += partial[i];
  red[t] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (t < w) red[t] += red[t + w];
    __syncthreads();
  }
  if (t == 0) *loss = (float)(red[0] / (double)n);
}

// Adam (Kingma & Ba) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t.
__global__ void k_adam(float* p, const float* g, float* m, float* v, long long n, float lr, float b1,
                       float b2, float eps, float c1, float sqrt_c2) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float denom = sqrtf(vi) / sqrt_c2 + eps;
  p[i] = p[i] - (lr / c1) * mi / denom;
}

// Per-pixel statistics over H histograms in two passes: partial sums over row blocks,
// then per pixel the mean; partial sums of squared deviations, then the population std.
constexpr int kStatRows = 256;

template <typename T>
__global__ void k_stat_pass(const T* hist, long long H, long long hs, long long rs, int n_par, int N,
                            const double* mean, double* partial) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= N) return;
  const long long off = (long long)(e / n_par) * rs + (e % n_par);
  const long long h0 = (long long)blockIdx.y * kStatRows;
  const long long h1 = h0 + kStatRows < H ? h0 + kStatRows : H;
  double s = 0.0;
  const double mu = mean ? mean[e] : 0.0;
  for (long long h = h0; h < h1; ++h) {
    const double v = (double)hist[h * hs + off];
    const double d = mean ? v - mu : v;
    s += mean ? d * d : d;
  }
  partial[(long long)blockIdx.y * N + e] = s;
}

__global__ void k_stat_reduce(const double* partial, int nb, int N, long long H, double* out, int sq) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= N) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[(long long)b * N + e];
  out[e] = sq ? sqrt(s / (double)H) : s / (double)H;
}

__global__ __launch_bounds__(1024) void k_stat_final(const double* mean, const double* sd, int N,
                                                     double floor_rel, float* mo, float* so) {
  __shared__ double red[16];
  double mx = 0.0;
  for (int e = threadIdx.x; e < N; e += 1024) mx = fmax(mx, sd[e]);
  mx = wave_max(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  double m = red[0];
  for (int q = 1; q < 16; ++q) m = fmax(m, red[q]);
  for (int e = threadIdx.x; e < N; e += 1024) {
    mo[e] = (float)mean[e];
    so[e] = (float)fmax(sd[e], floor_rel * m);
  }
}

hipError_t launch_gemm(const float* A, long long sam, long long sak, const float* B, long long sbk,
                       long long sbn, float* C, long long scm, long long M, long long Nc, long long K,
                       float alpha, float beta, const float* bias, int relu, hipStream_t st, int bf16) {
  if (M <= 0 || Nc <= 0) return hipSuccess;
  dim3 grid((unsigned)((M + kGT - 1) / kGT), (unsigned)((Nc + kGT - 1) / kGT));
  if (bf16)
    hipLaunchKernelGGL(k_gemm<true>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, C, scm, M, Nc, K, alpha,
                       beta, bias, relu);
  else
    hipLaunchKernelGGL(k_gemm<false>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, C, scm, M, Nc, K, alpha,
                       beta, bias, relu);
  return hipGetLastError();
}

hipError_t launch_relu_mask(float* d, const float* h, long long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_relu_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, d, h, n);
  return hipGetLastError();
}

hipError_t launch_colsum(const float* D, long long M, long long Nc, float* out, hipStream_t st) {
  if (Nc <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_colsum, dim3((unsigned)((Nc + 31) / 32)), dim3(256), 0, st, D, M, Nc, out);
  return hipGetLastError();
}

size_t mse_ws_bytes() { return 1024 * sizeof(double); }

hipError_t launch_mse(const float* xh, const float* x, long long n, float* loss, float* dxh, void* ws,
                      hipStream_t st) {
  const int nb = (int)std::max<long long>(1, std::min<long long>(1024, (n + 255) / 256));
  hipLaunchKernelGGL(k_mse_partial, dim3(nb), dim3(256), 0, st, xh, x, n, dxh, (double*)ws);
  hipLaunchKernelGGL(k_mse_final, dim3(1), dim3(256), 0, st, (const double*)ws, nb, n, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, double lr, double b1,
                       double b2, double eps, long long step, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const double c1 = 1.0 - std::pow(b1, (double)step), c2 = 1.0 - std::pow(b2, (double)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, g, m, v, n, (float)lr,
                     (float)b1, (float)b2, (float)eps, (float)c1, (float)std::sqrt(c2));
  return hipGetLastError();
}

// out[r][c] = (x[r][c] - mean[c]) / sd[c] in FP32 (x rounded to FP32 first; mean NULL = 0):
// one thread per element, rows of ld elements.
template <typename T>
__global__ __launch_bounds__(256) void k_col_normalize(const T* x, long long rows, long long cols, long long ld,
                                                       const float* mean, const float* sd, float* out) {
  const long long n = rows * cols;
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const long long r = e / cols, c = e - r * cols;
    const float v = (float)x[r * ld + c];
    out[e] = __fdiv_rn(mean ? __fsub_rn(v, mean[c]) : v, sd[c]);
  }
}

hipError_t launch_col_normalize(const void* x, int dtype, long long rows, long long cols, long long ld,
                                const float* mean, const float* sd, float* out, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const long long n = rows * cols;
  const unsigned nb = (unsigned)std::min<long long>((n + 255) / 256, 65536);
  if (dtype == HCZ_F32)
    hipLaunchKernelGGL(k_col_normalize<float>, dim3(nb), dim3(256), 0, st, (const float*)x, rows, cols, ld, mean,
                       sd, out);
  else
    hipLaunchKernelGGL(k_col_normalize<double>, dim3(nb), dim3(256), 0, st, (const double*)x, rows, cols, ld,
                       mean, sd, out);
  return hipGetLastError();
}

size_t norm_stats_ws_bytes(long long H, int N) {
  const long long nb = (H + kStatRows - 1) / kStatRows;
  return (size_t)(nb * N + 2 * N) * sizeof(double);
}

hipError_t launch_norm_stats(const void* hist, int dtype, long long H, long long hs, long long rs, int n_par,
                             int N, float* mean, float* sd, void* ws, hipStream_t st) {
  const long long nb = (H + kStatRows - 1) / kStatRows;
  double* partial = (double*)ws;
  double* mu = partial + nb * N;
  double* sdd = mu + N;
  dim3 g1((unsigned)((N + 255) / 256), (unsigned)nb), g2((unsigned)((N + 255) / 256));
  for (int pass = 0; pass < 2; ++pass) {
    if (dtype == HCZ_F32)
      hipLaunchKernelGGL(k_stat_pass<float>, g1, dim3(256), 0, st, (const float*)hist, H, hs, rs, n_par, N,
                         pass ? (const double*)mu : nullptr, partial);
    else
      hipLaunchKernelGGL(k_stat_pass<double>, g1, dim3(256), 0, st, (const double*)hist, H, hs, rs, n_par, N,
                         pass ? (const double*)mu : nullptr, partial);
    hipLaunchKernelGGL(k_stat_reduce, g2, dim3(256), 0, st, (const double*)partial, (int)nb, N, H,
                       pass ? sdd : mu, pass);
  }
  hipLaunchKernelGGL(k_stat_final, dim3(1), dim3(1024), 0, st, (const double*)mu, (const double*)sdd, N, 1e-12,
                     mean, sd);
  return hipGetLastError();
}

}  // namespace hcz
