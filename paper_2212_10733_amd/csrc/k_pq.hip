// Product-quantizer codebook fit (Section III Stage 3, Section IV-E): per latent
// dimension, 1-D k-means on every `every`-th latent vector.
//
// In one dimension every cluster of Lloyd's algorithm is a contiguous run of the sorted
// sample, so the fit is: gather -> bitonic sort per dimension -> FP64 prefix sums ->
// Lloyd iterations where each iteration finds the k-1 run boundaries by binary search at
// the FP64 midpoints and takes each centroid as (prefix[end] - prefix[start]) / count.
// Initial centroids: sorted[(2c+1) n / (2k)]; stop when no boundary moves, at most 25
// updates; an empty run keeps its centroid.
#include "hcz_internal.h"

namespace hcz {

constexpr int kSortNT = 1024;
constexpr int kSortChunk = 8192;   // keys sorted per workgroup in LDS (32 KB)

static long long next_pow2(long long n) {
  long long p = 1;
  while (p < n) p <<= 1;
  return p;
}

__global__ void k_gather(const float* z, long long n, int latent, long long every, long long ns,
                         long long np2, float* keys) {
  const long long s = (long long)blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y;
  if (s >= np2) return;
  float v = INFINITY;
  if (s < ns) {
    v = z[s * every * latent + d];
    if (isnan(v)) v = INFINITY;
  }
  keys[(long long)d * np2 + s] = v;
}

__device__ __forceinline__ void cswap(float& a, float& b, bool up) {
  if ((a > b) == up) { const float x = a; a = b; b = x; }
}

// Bitonic stages with stride j < chunk for sequence sizes k in [k_lo, k_hi] (powers of 2),
// on a chunk of `chunk` keys held in LDS.  Direction from the global index.
__global__ __launch_bounds__(kSortNT) void k_sort_local(float* keys, long long np2, int chunk,
                                                        long long k_lo, long long k_hi) {
  __shared__ float s[kSortChunk];
  const int d = blockIdx.y;
  float* base = keys + (long long)d * np2 + (long long)blockIdx.x * chunk;
  const long long gbase = (long long)blockIdx.x * chunk;
  for (int i = threadIdx.x; i < chunk; i += kSortNT) s[i] = base[i];
  __syncthreads();
  for (long long k = k_lo; k <= k_hi; k <<= 1) {
    long long jstart = k >> 1;
    if (jstart >= chunk) jstart = chunk >> 1;
    for (long long j = jstart; j >= 1; j >>= 1) {
      for (int i = threadIdx.x; i < chunk; i += kSortNT) {
        const int p = i ^ (int)j;
        if (p > i) {
          const bool up = ((gbase + i) & k) == 0;
          float a = s[i], b = s[p];
          cswap(a, b, up);
          s[i] = a;
          s[p] = b;
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < chunk; i += kSortNT) base[i] = s[i];
}

__global__ __launch_bounds__(256) void k_sort_global(float* keys, long long np2, long long k, long long j) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  const int d = blockIdx.y;
  if (i >= np2) return;
  const long long p = i ^ j;
  if (p <= i) return;
  float* b = keys + (long long)d * np2;
  const bool up = (i & k) == 0;
  float a = b[i], c = b[p];
  cswap(a, c, up);
  b[i] = a;
  b[p] = c;
}

// Exclusive FP64 prefix sums of the first ns sorted keys of each dimension.
__global__ __launch_bounds__(1024) void k_prefix(const float* keys, long long np2, long long ns,
                                                 double* prefix) {
  __shared__ double sw[16];
  const int d = blockIdx.x, t = threadIdx.x, w = t >> 6, l = t & 63;
  const float* kk = keys + (long long)d * np2;
  double* pf = prefix + (long long)d * (ns + 1);
  double carry = 0.0;
  for (long long b0 = 0; b0 < ns; b0 += 1024) {
    const long long i = b0 + t;
    const double x = i < ns ? (double)kk[i] : 0.0;
    double v = x;
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
      const double o = __shfl_up(v, k, 64);
      if (l >= k) v = v + o;
    }
    if (l == 63) sw[w] = v;
    __syncthreads();
    double before = carry;
    for (int q = 0; q < w; ++q) before = before + sw[q];
    if (i < ns) pf[i] = before + (v - x);
    double tot = carry;
    for (int q = 0; q < 16; ++q) tot = tot + sw[q];
    __syncthreads();
    carry = tot;
  }
  if (t == 0) pf[ns] = carry;
}

// Lloyd iterations of one dimension; thread c owns centroid c.
__global__ __launch_bounds__(256) void k_lloyd(const float* keys, long long np2, long long ns,
                                               const double* prefix, int kcb, float* centroids) {
  __shared__ double C[256];
  __shared__ long long ends[256];
  const int d = blockIdx.x, c = threadIdx.x;
  const float* kk = keys + (long long)d * np2;
  const double* pf = prefix + (long long)d * (ns + 1);
  if (c < kcb) {
    const long long idx = ((long long)(2 * c + 1) * ns) / (2LL * kcb);
    C[c] = (double)kk[idx];
  }
  __syncthreads();
  long long prev_end = -1;
  for (int it = 0; it < 25; ++it) {
    // end of run c: #{s : key_s <= beta_c}, beta_c = (C_c + C_{c+1}) * 0.5
    long long e = ns;
    if (c < kcb - 1) {
      const double beta = (C[c] + C[c + 1]) * 0.5;
      long long lo = 0, hi = ns;
      while (lo < hi) {
        const long long mid = (lo + hi) >> 1;
        if ((double)kk[mid] <= beta) lo = mid + 1;
        else hi = mid;
      }
      e = lo;
    }
    const int moved = (c < kcb) && (e != prev_end);
    if (c < kcb) ends[c] = e;
    const int any = __syncthreads_or(moved);
    if (it > 0 && !any) break;
    if (c < kcb) {
      const long long st = c == 0 ? 0 : ends[c - 1];
      const long long cnt = e - st;
      if (cnt > 0) C[c] = (pf[e] - pf[st]) / (double)cnt;
    }
    prev_end = e;
    __syncthreads();
  }
  if (c < kcb) centroids[(long long)d * kcb + c] = (float)C[c];
}

size_t codebook_ws_bytes(long long n, int latent, long long every) {
  const long long ns = (n + every - 1) / every;
  const long long np2 = std::max<long long>(next_pow2(ns), 2);
  return (size_t)latent * np2 * 4 + (size_t)latent * (ns + 1) * 8 + 256;
}

hipError_t launch_codebook_fit(const float* z, long long n, int latent, long long every, int bits,
                               float* centroids, void* ws, hipStream_t st) {
  const long long ns = (n + every - 1) / every;
  const long long np2 = std::max<long long>(next_pow2(ns), 2);
  float* keys = (float*)ws;
  double* prefix = (double*)((uint8_t*)ws + (((size_t)latent * np2 * 4 + 255) / 256) * 256);
  hipLaunchKernelGGL(k_gather, dim3((unsigned)((np2 + 255) / 256), latent), dim3(256), 0, st, z, n,
                     latent, every, ns, np2, keys);
  const int chunk = (int)std::min<long long>(np2, kSortChunk);
  const dim3 lgrid((unsigned)(np2 / chunk), latent);
  hipLaunchKernelGGL(k_sort_local, lgrid, dim3(kSortNT), 0, st, keys, np2, chunk, 2LL, (long long)chunk);
  for (long long k = 2LL * chunk; k <= np2; k <<= 1) {
    for (long long j = k >> 1; j >= chunk; j >>= 1)
      hipLaunchKernelGGL(k_sort_global, dim3((unsigned)((np2 + 255) / 256), latent), dim3(256), 0, st,
                         keys, np2, k, j);
    hipLaunchKernelGGL(k_sort_local, lgrid, dim3(kSortNT), 0, st, keys, np2, chunk, k, k);
  }
  hipLaunchKernelGGL(k_prefix, dim3(latent), dim3(1024), 0, st, keys, np2, ns, prefix);
  hipLaunchKernelGGL(k_lloyd, dim3(latent), dim3(256), 0, st, keys, np2, ns, prefix, 1 << bits, centroids);
  return hipGetLastError();
}

}  // namespace hcz
