// Dense autoencoder evaluation on FP32 matrix cores (Section III Stages 2-3) and the
// product-quantizer encoder (Stage 3).
//
// Encoder: a workgroup takes a tile of 128 histograms and computes
//   H1 = relu(X W1^T + b1)   [128 x 128], K = N streamed in chunks of 32 through LDS,
//   z  = H1 W2^T + b2        [128 x 16] on the vector ALUs,
// where X = (f - mu) / sigma is formed while loading.  Each of the four waves owns a
// 64 x 64 block of H1 made of 2 x 2 v_mfma_f32_32x32x2f32 tiles.  LDS rows are stored
// with k permuted (k -> (k & 1) * 16 + k / 2) so that a lane's 16 operands for one chunk
// are contiguous (four ds_read_b128).
// Decoder: Zhat = C[codes] -> H3 = relu(Zhat W3^T + b3) (vector ALUs) ->
//   fhat = sigma (H3 W4^T + b4) + mu, with H3 in LDS (k permuted) and W4 pre-permuted in
//   device memory, output columns in blocks of 128.  The decoder's arithmetic does not
//   depend on the launch: compression and decompression run this same kernel and get the
//   same bits.
#include "hcz_internal.h"

namespace hcz {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;   // histograms per workgroup
constexpr int kKc = 32;      // encoder K chunk
constexpr int kPitch = 36;   // LDS pitch (floats) of an encoder operand row
constexpr int kHPitch = 132; // LDS pitch of H1 / H3 rows

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

template <typename TIn, bool CONTIG>
__global__ __launch_bounds__(256, 2) void k_encode(ModelDev M, const TIn* hist, long long H,
                                                   long long hs, long long rs, int n_par, float* z) {
  // union: {As, Bs} during the K loop, H1 afterwards
  __shared__ __attribute__((aligned(16))) float smem[kTile * kHPitch];
  __shared__ __attribute__((aligned(16))) float W2t[kHidden * kLatent];
  float* As = smem;
  float* Bs = smem + kTile * kPitch;
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h0 = (long long)blockIdx.x * kTile;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int li = l & 31, lh = l >> 5;
  for (int q = t; q < kHidden * kLatent; q += 256) {
    const int o = q / kHidden, c = q % kHidden;
    W2t[c * kLatent + o] = M.W2[q];
  }
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;

  const int lk = t & 31, lr = t >> 5;
  const int kp = (lk & 1) * 16 + (lk >> 1);
  float ra[16], rb[16];
  const int nchunk = M.kpad / kKc;
  auto gload = [&](int c) {
    const int k = c * kKc + lk;
    const bool kin = k < M.N;
    const float mu = kin ? M.mu[k] : 0.0f;
    const float rsd = kin ? M.rsd[k] : 0.0f;
    const long long koff = CONTIG ? (long long)k : (long long)(k / n_par) * rs + (k % n_par);
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      const int row = it * 8 + lr;
      const long long h = h0 + row;
      float v = 0.0f;
      if (kin && h < H) {
        float fv = (float)hist[h * hs + koff];
        if (!isfinite(fv)) fv = 0.0f;
        v = (fv - mu) * rsd;
      }
      ra[it] = v;
      rb[it] = M.W1p[(long long)row * M.kpad + k];
    }
  };
  gload(0);
  for (int c = 0; c < nchunk; ++c) {
#pragma unroll
    for (int it = 0; it < 16; ++it) {
      As[(it * 8 + lr) * kPitch + kp] = ra[it];
      Bs[(it * 8 + lr) * kPitch + kp] = rb[it];
    }
    __syncthreads();
    if (c + 1 < nchunk) gload(c + 1);
    f32x4 av[2][4], bv[2][4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const f32x4* pa = (const f32x4*)&As[(wr + q * 32 + li) * kPitch + lh * 16];
      const f32x4* pb = (const f32x4*)&Bs[(wc + q * 32 + li) * kPitch + lh * 16];
#pragma unroll
      for (int u = 0; u < 4; ++u) { av[q][u] = pa[u]; bv[q][u] = pb[u]; }
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = mfma32(av[a][s >> 2][s & 3], bv[b][s >> 2][s & 3], acc[a][b]);
    }
    __syncthreads();
  }
  // epilogue 1: H1 = relu(acc + b1) into LDS
  float* H1 = smem;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wc + b * 32 + li;
      const float bias = M.b1[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr + a * 32 + 8 * (r >> 2) + 4 * lh + (r & 3);
        H1[row * kHPitch + col] = fmaxf(acc[a][b][r] + bias, 0.0f);
      }
    }
  __syncthreads();
  // layer 2 on the vector ALUs: 8 latent outputs per thread
  const int row = t >> 1, o0 = (t & 1) * 8;
  float s[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) s[o] = M.b2[o0 + o];
  for (int c = 0; c < kHidden; ++c) {
    const float hv = H1[row * kHPitch + c];
    const f32x4 w0 = *(const f32x4*)&W2t[c * kLatent + o0];
    const f32x4 w1 = *(const f32x4*)&W2t[c * kLatent + o0 + 4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      s[o] = fmaf(hv, w0[o], s[o]);
      s[o + 4] = fmaf(hv, w1[o], s[o + 4]);
    }
  }
  const long long h = h0 + row;
  if (h < H) {
#pragma unroll
    for (int o = 0; o < 8; ++o) z[h * kLatent + o0 + o] = s[o];
  }
}

// Encoder for contiguous FP32 histograms without LDS staging in the K loop: lane
// (li, kh) of a wave owns rows wr + 32 q + li and feeds the matrix core the 16
// consecutive k = 32 c + 16 kh + s (s = 0..15) of chunk c, loaded straight from memory
// (one run of 64 bytes per row and operand), so each v_mfma_f32_32x32x2f32 step sums the
// pair k = 32 c + s, 32 c + 16 + s.  The next chunk's operands are loaded while the
// current one is multiplied; no barrier is needed until the epilogue.  mu and 1/sigma
// sit in LDS (zero beyond N), and a chunk reaching past N reads element by element.
typedef float f32x4u __attribute__((ext_vector_type(4), aligned(4)));

__global__ __launch_bounds__(256, 2) void k_encode_d(ModelDev M, const float* hist, long long H, long long hs,
                                                     float* z) {
  __shared__ __attribute__((aligned(16))) float smem[kTile * kHPitch];   // mu / rsd, then H1
  __shared__ __attribute__((aligned(16))) float W2t[kHidden * kLatent];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h0 = (long long)blockIdx.x * kTile;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int li = l & 31, kh = l >> 5;
  const int N = M.N, kpad = M.kpad;
  float* s_mu = smem;
  float* s_rsd = smem + kpad;
  for (int k = t; k < kpad; k += 256) {
    s_mu[k] = k < N ? M.mu[k] : 0.0f;
    s_rsd[k] = k < N ? M.rsd[k] : 0.0f;
  }
  for (int q = t; q < kHidden * kLatent; q += 256) {
    const int o = q / kHidden, c = q % kHidden;
    W2t[c * kLatent + o] = M.W2[q];
  }
  __syncthreads();
  const float* arow[2];
  const float* brow[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const long long r = min(h0 + wr + q * 32 + li, H - 1);     // rows past H repeat the last one
    arow[q] = hist + r * hs + kh * 16;
    brow[q] = M.W1p + (long long)(wc + q * 32 + li) * kpad + kh * 16;
  }
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
  const int nfull = N / kKc, nchunk = kpad / kKc;
  // two raw operand buffers: chunk c + 1 is loaded while chunk c is normalised and
  // multiplied (the loop takes chunks in pairs, so the buffers alternate by name)
  struct Raw {
    f32x4u a[2][4], b[2][4];
  };
  auto gload = [&](int c, Raw& R) {
    if (c < nfull) {
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          R.a[q][u] = *(const f32x4u*)(arow[q] + c * kKc + 4 * u);
          R.b[q][u] = *(const f32x4u*)(brow[q] + c * kKc + 4 * u);
        }
    } else {                              // k may reach N: element by element
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int k = c * kKc + kh * 16 + 4 * u + e;
            R.a[q][u][e] = k < N ? arow[q][c * kKc + 4 * u + e] : 0.0f;
          }
          R.b[q][u] = *(const f32x4u*)(brow[q] + c * kKc + 4 * u);
        }
    }
  };
  // (f - mu) / sigma with non-finite inputs as 0, formed right before the matrix core
  // takes it; the products and their order are those of a fully normalised chunk
  auto mma = [&](int c, const Raw& R) {
    const f32x4* pm = (const f32x4*)(s_mu + c * kKc + kh * 16);
    const f32x4* pr = (const f32x4*)(s_rsd + c * kKc + kh * 16);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f32x4 mu4 = pm[u], rs4 = pr[u];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float av[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          float fv = R.a[q][u][e];
          if (!isfinite(fv)) fv = 0.0f;
          av[q] = (fv - mu4[e]) * rs4[e];
        }
#pragma unroll
        for (int qa = 0; qa < 2; ++qa)
#pragma unroll
          for (int qb = 0; qb < 2; ++qb) acc[qa][qb] = mfma32(av[qa], R.b[qb][u][e], acc[qa][qb]);
      }
    }
  };
  Raw R0, R1;
  gload(0, R0);
  for (int c = 0; c < nchunk; c += 2) {
    if (c + 1 < nchunk) gload(c + 1, R1);
    mma(c, R0);
    if (c + 1 < nchunk) {
      if (c + 2 < nchunk) gload(c + 2, R0);
      mma(c + 1, R1);
    }
  }
  __syncthreads();
  // epilogue 1: H1 = relu(acc + b1) into LDS
  float* H1 = smem;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wc + b * 32 + li;
      const float bias = M.b1[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr + a * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        H1[row * kHPitch + col] = fmaxf(acc[a][b][r] + bias, 0.0f);
      }
    }
  __syncthreads();
  // layer 2 on the vector ALUs: 8 latent outputs per thread
  const int row = t >> 1, o0 = (t & 1) * 8;
  float sacc[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) sacc[o] = M.b2[o0 + o];
  for (int c = 0; c < kHidden; ++c) {
    const float hv = H1[row * kHPitch + c];
    const f32x4 w0 = *(const f32x4*)&W2t[c * kLatent + o0];
    const f32x4 w1 = *(const f32x4*)&W2t[c * kLatent + o0 + 4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      sacc[o] = fmaf(hv, w0[o], sacc[o]);
      sacc[o + 4] = fmaf(hv, w1[o], sacc[o + 4]);
    }
  }
  const long long h = h0 + row;
  if (h < H) {
#pragma unroll
    for (int o = 0; o < 8; ++o) z[h * kLatent + o0 + o] = sacc[o];
  }
}

__global__ __launch_bounds__(256, 2) void k_decode(ModelDev M, const uint8_t* codes,
                                                   const float* centroids, int kcb, long long H,
                                                   float* fhat) {
  __shared__ __attribute__((aligned(16))) float H3[kTile * kHPitch];
  __shared__ float Zh[kTile * kLatent];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h0 = (long long)blockIdx.x * kTile;
  const int li = l & 31, lh = l >> 5;
  for (int q = t; q < kTile * kLatent; q += 256) {
    const int row = q / kLatent, d = q % kLatent;
    const long long h = h0 + row;
    Zh[q] = (h < H) ? centroids[d * kcb + min((int)codes[h * kLatent + d], kcb - 1)] : 0.0f;
  }
  __syncthreads();
  // H3 = relu(Zhat W3^T + b3), stored with k permuted: c -> (c & 1) * 64 + c / 2
  {
    const int c = t & 127;
    float w3[kLatent];
#pragma unroll
    for (int d = 0; d < kLatent; ++d) w3[d] = M.W3[c * kLatent + d];
    const float b3 = M.b3[c];
    const int cp = (c & 1) * 64 + (c >> 1);
    for (int row = t >> 7; row < kTile; row += 2) {
      float s = b3;
#pragma unroll
      for (int d = 0; d < kLatent; ++d) s = fmaf(Zh[row * kLatent + d], w3[d], s);
      H3[row * kHPitch + cp] = fmaxf(s, 0.0f);
    }
  }
  __syncthreads();
  const int wr = (w >> 1) * 64;
  // the weights of the next (column block, quarter) step are loaded from memory while the
  // current one is multiplied; the H3 operands come from LDS
  f32x4 av[2][4], bv[2][4], bn[2][4];
  auto bload = [&](int nb, int quarter, f32x4 (&B)[2][4]) {
    const int wc = nb + (w & 1) * 64;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const f32x4* pb = (const f32x4*)&M.W4p[(long long)(wc + q * 32 + li) * kHidden + lh * 64 + quarter * 16];
#pragma unroll
      for (int u = 0; u < 4; ++u) B[q][u] = pb[u];
    }
  };
  bload(0, 0, bv);
  // b4, sigma and mu of the wave's two column tiles, loaded one column block ahead
  float ep[2][3], epn[2][3];
  auto epload = [&](int nb, float (&E)[2][3]) {
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int cc = min(nb + (w & 1) * 64 + b * 32 + li, M.N - 1);
      E[b][0] = M.b4[cc];
      E[b][1] = M.sd[cc];
      E[b][2] = M.mu[cc];
    }
  };
  epload(0, ep);
  const bool full = h0 + kTile <= H;       // every row of the tile is a histogram
  for (int nb = 0; nb < M.npad; nb += 128) {
    const int wc = nb + (w & 1) * 64;
    epload(min(nb + 128, M.npad - 128), epn);
    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
#pragma unroll 1
    for (int quarter = 0; quarter < 4; ++quarter) {
      if (quarter < 3 || nb + 128 < M.npad) bload(quarter < 3 ? nb : nb + 128, (quarter + 1) & 3, bn);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const f32x4* pa = (const f32x4*)&H3[(wr + q * 32 + li) * kHPitch + lh * 64 + quarter * 16];
#pragma unroll
        for (int u = 0; u < 4; ++u) av[q][u] = pa[u];
      }
#pragma unroll
      for (int s = 0; s < 16; ++s)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            acc[a][b] = mfma32(av[a][s >> 2][s & 3], bv[b][s >> 2][s & 3], acc[a][b]);
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int u = 0; u < 4; ++u) bv[q][u] = bn[q][u];
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int col = wc + b * 32 + li;
        if (col >= M.N) continue;
        const float b4 = ep[b][0], sd = ep[b][1], mu = ep[b][2];
        float* dst = fhat + (h0 + wr + a * 32 + 4 * lh) * M.N + col;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int rr = 8 * (r >> 2) + (r & 3);        // row within the tile, less 4 lh
          if (full || h0 + wr + a * 32 + 4 * lh + rr < H) dst[rr * M.N] = fmaf(sd, acc[a][b][r] + b4, mu);
        }
      }
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int e = 0; e < 3; ++e) ep[b][e] = epn[b][e];
  }
}

// ---- BF16 form --------------------------------------------------------------------------
// The two large products take bfloat16 operands on v_mfma_f32_32x32x16_bf16 with FP32
// accumulation: the encoder's x = (f - mu) * (1/sigma), formed in FP32 and rounded to
// nearest-even bfloat16, against W1 rounded at load; the decoder's h3 (the same FP32
// fused multiply-add chain as the FP32 form, then ReLU) rounded likewise, against W4.
// Operand layout of the 32x32x16 instruction: lane l supplies row (or column) l % 32 and
// eight consecutive k of the sixteen, starting at 8 (l / 32).  The encoder streams K in
// chunks of 32: lane half kh holds k in [32c + 16kh, 32c + 16kh + 16), the first eight for
// the chunk's first instruction and the rest for its second, read straight from memory.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
constexpr int kBPitch = 136;  // LDS pitch (bfloat16) of the decoder's H3 rows

__device__ __forceinline__ f32x16 mfma_bf16(bf16x8 a, bf16x8 b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// VEC: FP32 input with contiguous rows, loaded 16 bytes at a time.  Otherwise elements are
// loaded one by one through an LDS table of their offsets (FP64 input is rounded to FP32).
template <typename TIn, bool VEC>
__global__ __launch_bounds__(256, 2) void k_encode_b(ModelDev M, const TIn* hist, long long H, long long hs,
                                                     long long rs, int n_par, float* z) {
  __shared__ __attribute__((aligned(16))) float smem[kTile * kHPitch];   // mu / rsd / offsets, then H1
  __shared__ __attribute__((aligned(16))) float W2t[kHidden * kLatent];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h0 = (long long)blockIdx.x * kTile;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  const int li = l & 31, kh = l >> 5;
  const int N = M.N, kpad = M.kpad;
  float* s_mu = smem;
  float* s_rsd = smem + kpad;
  int* s_off = (int*)(smem + 2 * kpad);
  for (int k = t; k < kpad; k += 256) {
    s_mu[k] = k < N ? M.mu[k] : 0.0f;
    s_rsd[k] = k < N ? M.rsd[k] : 0.0f;
    if (!VEC) s_off[k] = k < N ? (int)((k / n_par) * rs + k % n_par) : 0;
  }
  for (int q = t; q < kHidden * kLatent; q += 256) {
    const int o = q / kHidden, c = q % kHidden;
    W2t[c * kLatent + o] = M.W2[q];
  }
  __syncthreads();
  const TIn* arow[2];
  const __bf16* brow[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const long long r = min(h0 + wr + q * 32 + li, H - 1);     // rows past H repeat the last one
    arow[q] = hist + r * hs;
    brow[q] = (const __bf16*)M.W1b + (long long)(wc + q * 32 + li) * kpad + kh * 16;
  }
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.0f;
  const int nfull = VEC ? N / kKc : 0, nchunk = kpad / kKc;
  float ra[2][16];
  bf16x8 rb[2][2];
  auto bload = [&](int c) {
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int s = 0; s < 2; ++s) rb[q][s] = *(const bf16x8*)(brow[q] + c * kKc + 8 * s);
  };
  auto gload = [&](int c) {               // 16 in-range k per row
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const f32x4u v = *(const f32x4u*)((const float*)arow[q] + c * kKc + kh * 16 + 4 * u);
#pragma unroll
        for (int e = 0; e < 4; ++e) ra[q][4 * u + e] = v[e];
      }
    bload(c);
  };
  auto gload_elem = [&](int c) {          // k may reach N, or rows are strided
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int k = c * kKc + kh * 16 + j;
        ra[q][j] = k < N ? (float)arow[q][VEC ? k : s_off[k]] : 0.0f;
      }
    bload(c);
  };
  if (nfull > 0) gload(0);
  else gload_elem(0);
  for (int c = 0; c < nchunk; ++c) {
    // this chunk's operands: (f - mu) / sigma in FP32, non-finite inputs as 0, to bfloat16
    bf16x8 a8[2][2], b8[2][2];
    const f32x4* pm = (const f32x4*)(s_mu + c * kKc + kh * 16);
    const f32x4* pr = (const f32x4*)(s_rsd + c * kKc + kh * 16);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const f32x4 mu4 = pm[u], rs4 = pr[u];
#pragma unroll
      for (int e = 0; e < 4; ++e)
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          float fv = ra[q][4 * u + e];
          if (!isfinite(fv)) fv = 0.0f;
          a8[q][u >> 1][4 * (u & 1) + e] = (__bf16)((fv - mu4[e]) * rs4[e]);
        }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q)
#pragma unroll
      for (int s = 0; s < 2; ++s) b8[q][s] = rb[q][s];
    if (c + 1 < nfull) gload(c + 1);
    else if (c + 1 < nchunk) gload_elem(c + 1);
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = mfma_bf16(a8[a][s], b8[b][s], acc[a][b]);
  }
  __syncthreads();
  // epilogue 1: H1 = relu(acc + b1) into LDS
  float* H1 = smem;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int col = wc + b * 32 + li;
      const float bias = M.b1[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wr + a * 32 + 8 * (r >> 2) + 4 * kh + (r & 3);
        H1[row * kHPitch + col] = fmaxf(acc[a][b][r] + bias, 0.0f);
      }
    }
  __syncthreads();
  // layer 2 on the vector ALUs in FP32: 8 latent outputs per thread
  const int row = t >> 1, o0 = (t & 1) * 8;
  float sacc[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) sacc[o] = M.b2[o0 + o];
  for (int c = 0; c < kHidden; ++c) {
    const float hv = H1[row * kHPitch + c];
    const f32x4 w0 = *(const f32x4*)&W2t[c * kLatent + o0];
    const f32x4 w1 = *(const f32x4*)&W2t[c * kLatent + o0 + 4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      sacc[o] = fmaf(hv, w0[o], sacc[o]);
      sacc[o + 4] = fmaf(hv, w1[o], sacc[o + 4]);
    }
  }
  const long long h = h0 + row;
  if (h < H) {
#pragma unroll
    for (int o = 0; o < 8; ++o) z[h * kLatent + o0 + o] = sacc[o];
  }
}

// BF16 encoder for FP32 input with contiguous rows.  Each wave owns 32 histograms and all
// 128 hidden units (four 32-column tiles).  Per K chunk of 32 a load instruction covers 8
// whole 128-byte row segments (lane l: row 8 i + l / 8, floats 4 (l % 8) .. + 3), the
// normalised bfloat16 values pass through a wave-private LDS tile into the matrix-core
// row layout, and the weights come pre-arranged in operand order (W1m: one contiguous
// 1 KB load per k-step and column tile).  The next chunk's loads are in flight while the
// current one is multiplied; no workgroup barrier inside the K loop.
constexpr int kSP = 40;   // LDS pitch (bfloat16) of a staged row of 32 k
__global__ __launch_bounds__(256, 2) void k_encode_b2(ModelDev M, const float* hist, long long H, long long hs,
                                                      float* z) {
  __shared__ __attribute__((aligned(16))) float smem[kTile * kHPitch];   // mu / rsd / staging, then H1
  __shared__ __attribute__((aligned(16))) float W2t[kHidden * kLatent];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h0 = (long long)blockIdx.x * kTile;
  const int li = l & 31, kh = l >> 5;
  const int N = M.N, kpad = M.kpad;
  float* s_mu = smem;
  float* s_rsd = smem + kpad;
  __bf16* stg = (__bf16*)(smem + 2 * kpad) + w * 32 * kSP;
  for (int k = t; k < kpad; k += 256) {
    s_mu[k] = k < N ? M.mu[k] : 0.0f;
    s_rsd[k] = k < N ? M.rsd[k] : 0.0f;
  }
  for (int q = t; q < kHidden * kLatent; q += 256) {
    const int o = q / kHidden, c = q % kHidden;
    W2t[c * kLatent + o] = M.W2[q];
  }
  __syncthreads();
  const int kq = l & 7, rsub = l >> 3;
  const float* arow[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const long long r = min(h0 + 32 * w + 8 * i + rsub, H - 1);
    arow[i] = hist + r * hs + 4 * kq;
  }
  const bf16x8* Wm = (const bf16x8*)M.W1m + l;
  f32x16 acc[4];
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[n][r] = 0.0f;
  const int nfull = N / kKc, nchunk = kpad / kKc;
  // two chunks of input in flight: ra holds chunk c, rn chunk c + 1
  f32x4u ra[4], rn[4];
  bf16x8 rb[2][4];
  auto aload = [&](int c, f32x4u (&dst)[4]) {
    if (c < nfull) {
#pragma unroll
      for (int i = 0; i < 4; ++i) dst[i] = *(const f32x4u*)(arow[i] + c * kKc);
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int e = 0; e < 4; ++e) dst[i][e] = (c * kKc + 4 * kq + e < N) ? arow[i][c * kKc + e] : 0.0f;
    }
  };
  auto bload = [&](int c) {
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int n = 0; n < 4; ++n) rb[s][n] = Wm[((2 * c + s) * 4 + n) * 64];
  };
  aload(0, ra);
  if (nchunk > 1) aload(1, rn);
  bload(0);
  for (int c = 0; c < nchunk; ++c) {
    const f32x4 mu4 = *(const f32x4*)(s_mu + c * kKc + 4 * kq);
    const f32x4 rs4 = *(const f32x4*)(s_rsd + c * kKc + 4 * kq);
    // normalise this chunk and stage it as bfloat16 rows
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
      bf16x4 v;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        float fv = ra[i][e];
        if (!isfinite(fv)) fv = 0.0f;
        v[e] = (__bf16)((fv - mu4[e]) * rs4[e]);
      }
      *(bf16x4*)(stg + (8 * i + rsub) * kSP + 4 * kq) = v;
    }
    bf16x8 b8[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int n = 0; n < 4; ++n) b8[s][n] = rb[s][n];
#pragma unroll
    for (int i = 0; i < 4; ++i) ra[i] = rn[i];
    if (c + 2 < nchunk) aload(c + 2, rn);
    if (c + 1 < nchunk) bload(c + 1);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    bf16x8 a8[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) a8[s] = *(const bf16x8*)(stg + li * kSP + 16 * s + 8 * kh);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int n = 0; n < 4; ++n) acc[n] = mfma_bf16(a8[s], b8[s][n], acc[n]);
  }
  __syncthreads();
  // epilogue 1: H1 = relu(acc + b1) into LDS (rows of this wave)
  float* H1 = smem;
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    const int col = 32 * n + li;
    const float bias = M.b1[col];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = 32 * w + 8 * (r >> 2) + 4 * kh + (r & 3);
      H1[row * kHPitch + col] = fmaxf(acc[n][r] + bias, 0.0f);
    }
  }
  __syncthreads();
  const int row = t >> 1, o0 = (t & 1) * 8;
  float sacc[8];
#pragma unroll
  for (int o = 0; o < 8; ++o) sacc[o] = M.b2[o0 + o];
  for (int c = 0; c < kHidden; ++c) {
    const float hv = H1[row * kHPitch + c];
    const f32x4 w0 = *(const f32x4*)&W2t[c * kLatent + o0];
    const f32x4 w1 = *(const f32x4*)&W2t[c * kLatent + o0 + 4];
#pragma unroll
    for (int o = 0; o < 4; ++o) {
      sacc[o] = fmaf(hv, w0[o], sacc[o]);
      sacc[o + 4] = fmaf(hv, w1[o], sacc[o + 4]);
    }
  }
  const long long h = h0 + row;
  if (h < H) {
#pragma unroll
    for (int o = 0; o < 8; ++o) z[h * kLatent + o0 + o] = sacc[o];
  }
}

// Decoder of the BF16 form, with row-contiguous stores: each wave owns 32 histograms and
// keeps their eight bfloat16 h3 operands in registers; per block of 64 output columns the
// weights come pre-arranged in operand order (W4m, 1 KB per load instruction, the next
// block in flight) and the results pass through a wave-private LDS tile so that each
// store instruction writes four 256-byte row segments.
constexpr int kOP = 68;   // LDS pitch (floats) of the output tile
__global__ __launch_bounds__(256, 2) void k_decode_b2(ModelDev M, const uint8_t* codes, const float* centroids,
                                                      int kcb, long long H, float* fhat) {
  __shared__ __attribute__((aligned(16))) __bf16 H3[kTile * kBPitch];
  __shared__ __attribute__((aligned(16))) float outs[4 * 32 * kOP];
  __shared__ float Zh[kTile * kLatent];
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long h0 = (long long)blockIdx.x * kTile;
  const int li = l & 31, kh = l >> 5;
  const int N = M.N;
  for (int q = t; q < kTile * kLatent; q += 256) {
    const int row = q / kLatent, d = q % kLatent;
    const long long h = h0 + row;
    Zh[q] = (h < H) ? centroids[d * kcb + min((int)codes[h * kLatent + d], kcb - 1)] : 0.0f;
  }
  __syncthreads();
  {
    const int c = t & 127;
    float w3[kLatent];
#pragma unroll
    for (int d = 0; d < kLatent; ++d) w3[d] = M.W3[c * kLatent + d];
    const float b3 = M.b3[c];
    for (int row = t >> 7; row < kTile; row += 2) {
      float s = b3;
#pragma unroll
      for (int d = 0; d < kLatent; ++d) s = fmaf(Zh[row * kLatent + d], w3[d], s);
      H3[row * kBPitch + c] = (__bf16)fmaxf(s, 0.0f);
    }
  }
  __syncthreads();
  bf16x8 a8[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) a8[s] = *(const bf16x8*)&H3[(32 * w + li) * kBPitch + 16 * s + 8 * kh];
  float* ot = outs + w * 32 * kOP;
  const bf16x8* Wm = (const bf16x8*)M.W4m + l;
  const int nblk = M.npad / 64;
  bf16x8 bv[2][8], bn[2][8];
  auto bload = [&](int nb, bf16x8 (&B)[2][8]) {
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int s = 0; s < 8; ++s) B[n][s] = Wm[((nb * 2 + n) * 8 + s) * 64];
  };
  bload(0, bv);
  // b4, sigma and mu of the lane's two columns, loaded one column block ahead
  float ep[2][3], epn[2][3];
  auto epload = [&](int nb, float (&E)[2][3]) {
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const int cc = min(64 * nb + 32 * n + li, N - 1);
      E[n][0] = M.b4[cc];
      E[n][1] = M.sd[cc];
      E[n][2] = M.mu[cc];
    }
  };
  epload(0, ep);
  // store mapping: lane -> row 4 i + l / 16 (i = 0..7), columns 4 (l % 16) .. + 3 of the block
  const int srow = l >> 4, scol = 4 * (l & 15);
  for (int nb = 0; nb < nblk; ++nb) {
    if (nb + 1 < nblk) bload(nb + 1, bn);
    epload(min(nb + 1, nblk - 1), epn);
    f32x16 acc[2];
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[n][r] = 0.0f;
#pragma unroll
    for (int s = 0; s < 8; ++s)
#pragma unroll
      for (int n = 0; n < 2; ++n) acc[n] = mfma_bf16(a8[s], bv[n][s], acc[n]);
#pragma unroll
    for (int n = 0; n < 2; ++n) {
      const float b4 = ep[n][0], sd = ep[n][1], mu = ep[n][2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = 8 * (r >> 2) + 4 * kh + (r & 3);
        ot[row * kOP + 32 * n + li] = fmaf(sd, acc[n][r] + b4, mu);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int c0 = 64 * nb + scol;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int row = 4 * i + srow;
      const long long h = h0 + 32 * w + row;
      const f32x4 v = *(const f32x4*)(ot + row * kOP + scol);
      if (h < H) {
        float* dst = fhat + h * N + c0;
        if (c0 + 3 < N) {
          *(f32x4u*)dst = v;
        } else {
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (c0 + e < N) dst[e] = v[e];
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int s = 0; s < 8; ++s) bv[n][s] = bn[n][s];
#pragma unroll
    for (int n = 0; n < 2; ++n)
#pragma unroll
      for (int e = 0; e < 3; ++e) ep[n][e] = epn[n][e];
  }
}

// code = #{c : (C_c + C_{c+1}) / 2 < z} with the midpoints in FP64: a lower bound search.
__global__ __launch_bounds__(256) void k_quantize(const float* z, long long n, int latent,
                                                  const float* centroids, int kcb, uint8_t* codes) {
  const long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  if (q >= n * latent) return;
  const int d = (int)(q % latent);
  const float* C = centroids + (long long)d * kcb;
  const double zv = (double)z[q];
  int lo = 0, hi = kcb - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double beta = ((double)C[mid] + (double)C[mid + 1]) * 0.5;
    if (beta < zv) lo = mid + 1;
    else hi = mid;
  }
  codes[q] = (uint8_t)lo;
}

// The same search over midpoints staged once per workgroup in LDS ([latent][kcb - 1] in
// FP64, formed exactly as above), the workgroup striding over the latents.
constexpr int kQuantLdsMax = 65536;   // bytes of staged midpoints this form takes
__global__ __launch_bounds__(256) void k_quantize_lds(const float* z, long long n, int latent,
                                                      const float* centroids, int kcb, uint8_t* codes) {
  extern __shared__ double beta[];
  const int nb = kcb - 1;
  for (int q = threadIdx.x; q < latent * nb; q += 256) {
    const int d = q / nb, c = q - d * nb;
    const float* C = centroids + (long long)d * kcb;
    beta[q] = ((double)C[c] + (double)C[c + 1]) * 0.5;
  }
  __syncthreads();
  const long long tot = n * latent;
  const long long stride = (long long)gridDim.x * 256;
  long long q = (long long)blockIdx.x * 256 + threadIdx.x;
  int d = (int)(q % latent);
  const int dstep = (int)(stride % latent);
  for (; q < tot; q += stride) {
    const double* B = beta + d * nb;
    const double zv = (double)z[q];
    int lo = 0, hi = kcb - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (B[mid] < zv) lo = mid + 1;
      else hi = mid;
    }
    codes[q] = (uint8_t)lo;
    d += dstep;
    if (d >= latent) d -= latent;
  }
}

// ---- FP64 form: every layer in FP64 on the vector ALUs, one workgroup per histogram ----
// Encoder: x = (f - mu) / sigma (non-finite inputs as 0) staged in LDS; thread c sums
// W1[c][k] x_k over k = 0..N-1 with fused multiply-adds, h1_c = max(0, sum + b1_c);
// threads o < latent sum W2[o][c] h1_c over c = 0..127, plus b2_o; z stored as FP32.
template <typename TIn>
__global__ __launch_bounds__(128) void k_encode64(ModelDev M, const TIn* hist, long long H, long long hs,
                                                  long long rs, int n_par, float* z) {
  extern __shared__ double xs[];          // x [N], then h1 [128]
  const long long h = blockIdx.x;
  const int t = threadIdx.x, N = M.N;
  const TIn* f = hist + h * hs;
  for (int e = t; e < N; e += 128) {
    const int j = e / n_par, i = e - j * n_par;
    double v = (double)f[(long long)j * rs + i];
    if (!isfinite(v)) v = 0.0;
    xs[e] = (v - M.mud[e]) / M.sdd[e];
  }
  __syncthreads();
  double s = 0.0;
  for (int k = 0; k < N; ++k) s = fma(M.W1t[(long long)k * kHidden + t], xs[k], s);
  double* h1 = xs + N;
  h1[t] = fmax(s + M.b1d[t], 0.0);
  __syncthreads();
  if (t < kLatent) {
    double a = 0.0;
    for (int c = 0; c < kHidden; ++c) a = fma(M.W2d[t * kHidden + c], h1[c], a);
    z[h * kLatent + t] = (float)(a + M.b2d[t]);
  }
}

// Decoder: zhat_d = C[d][code_d]; h3_c = max(0, sum_d W3[c][d] zhat_d + b3_c) over
// d = 0..15; fhat_n = sigma_n (sum_c W4[n][c] h3_c + b4_n) + mu_n over c = 0..127, stored
// as FP32.
__global__ __launch_bounds__(128) void k_decode64(ModelDev M, const uint8_t* codes, const float* centroids,
                                                  int kcb, long long H, float* fhat) {
  __shared__ double zh[kLatent], h3[kHidden];
  const long long h = blockIdx.x;
  const int t = threadIdx.x, N = M.N;
  if (t < kLatent) zh[t] = (double)centroids[t * kcb + min((int)codes[h * kLatent + t], kcb - 1)];
  __syncthreads();
  double s = 0.0;
  for (int d = 0; d < kLatent; ++d) s = fma(M.W3d[t * kLatent + d], zh[d], s);
  h3[t] = fmax(s + M.b3d[t], 0.0);
  __syncthreads();
  for (int n = t; n < N; n += 128) {
    double y = 0.0;
    for (int c = 0; c < kHidden; ++c) y = fma(M.W4t[(long long)c * N + n], h3[c], y);
    y = y + M.b4d[n];
    fhat[h * N + n] = (float)(M.sdd[n] * y + M.mud[n]);
  }
}

hipError_t launch_encode(const ModelDev& M, const void* hist, int dtype, long long H, long long hs,
                         long long rs, int n_par, float* z, hipStream_t st) {
  if (H <= 0) return hipSuccess;
  if (M.arch == HCZ_ARCH_CONV) return launch_conv_encode(M, hist, dtype, H, hs, rs, z, st);
  if (M.fp64) {
    const size_t lds = ((size_t)M.N + kHidden) * sizeof(double);
    if (dtype == HCZ_F32)
      hipLaunchKernelGGL(k_encode64<float>, dim3((unsigned)H), dim3(128), lds, st, M, (const float*)hist, H, hs, rs, n_par, z);
    else
      hipLaunchKernelGGL(k_encode64<double>, dim3((unsigned)H), dim3(128), lds, st, M, (const double*)hist, H, hs, rs, n_par, z);
    return hipGetLastError();
  }
  const bool contig = rs == n_par;
  dim3 grid((unsigned)((H + kTile - 1) / kTile)), block(256);
  if (M.bf16) {
    if (dtype == HCZ_F32 && contig)
      hipLaunchKernelGGL(k_encode_b2, grid, block, 0, st, M, (const float*)hist, H, hs, z);
    else if (dtype == HCZ_F32)
      hipLaunchKernelGGL((k_encode_b<float, false>), grid, block, 0, st, M, (const float*)hist, H, hs, rs, n_par, z);
    else
      hipLaunchKernelGGL((k_encode_b<double, false>), grid, block, 0, st, M, (const double*)hist, H, hs, rs, n_par, z);
  } else if (dtype == HCZ_F32) {
    if (contig && (size_t)M.kpad * 2 <= (size_t)kTile * kHPitch)
      hipLaunchKernelGGL(k_encode_d, grid, block, 0, st, M, (const float*)hist, H, hs, z);
    else if (contig) hipLaunchKernelGGL((k_encode<float, true>), grid, block, 0, st, M, (const float*)hist, H, hs, rs, n_par, z);
    else hipLaunchKernelGGL((k_encode<float, false>), grid, block, 0, st, M, (const float*)hist, H, hs, rs, n_par, z);
  } else {
    if (contig) hipLaunchKernelGGL((k_encode<double, true>), grid, block, 0, st, M, (const double*)hist, H, hs, rs, n_par, z);
    else hipLaunchKernelGGL((k_encode<double, false>), grid, block, 0, st, M, (const double*)hist, H, hs, rs, n_par, z);
  }
  return hipGetLastError();
}

hipError_t launch_decode(const ModelDev& M, const uint8_t* codes, const float* centroids, int bits,
                         long long H, float* fhat, hipStream_t st) {
  if (H <= 0) return hipSuccess;
  if (M.arch == HCZ_ARCH_CONV) return launch_conv_decode(M, codes, centroids, bits, H, fhat, st);
  if (M.fp64) {
    hipLaunchKernelGGL(k_decode64, dim3((unsigned)H), dim3(128), 0, st, M, codes, centroids, 1 << bits, H, fhat);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((H + kTile - 1) / kTile)), block(256);
  if (M.bf16) hipLaunchKernelGGL(k_decode_b2, grid, block, 0, st, M, codes, centroids, 1 << bits, H, fhat);
  else hipLaunchKernelGGL(k_decode, grid, block, 0, st, M, codes, centroids, 1 << bits, H, fhat);
  return hipGetLastError();
}

hipError_t launch_quantize(const float* z, long long n, int latent, const float* centroids,
                           int bits, uint8_t* codes, hipStream_t st) {
  const long long tot = n * latent;
  if (tot <= 0) return hipSuccess;
  const int kcb = 1 << bits;
  const size_t lds = (size_t)latent * (kcb - 1) * sizeof(double);
  if (kcb > 1 && lds <= (size_t)kQuantLdsMax) {
    const unsigned grid = (unsigned)std::min<long long>((tot + 255) / 256, 2048);
    hipLaunchKernelGGL(k_quantize_lds, dim3(grid), dim3(256), lds, st, z, n, latent, centroids, kcb, codes);
  } else {
    hipLaunchKernelGGL(k_quantize, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, z, n, latent,
                       centroids, kcb, codes);
  }
  return hipGetLastError();
}

}  // namespace hcz
