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
      // pair m joins keys i = 2 j (m / j) + m % j and i + j: every thread busy
      const int jj = (int)j;
      for (int m = threadIdx.x; m < chunk / 2; m += kSortNT) {
        const int i = ((m & ~(jj - 1)) << 1) | (m & (jj - 1)), p = i + jj;
        const bool up = ((gbase + i) & k) == 0;
        float a = s[i], b = s[p];
        cswap(a, b, up);
        s[i] = a;
        s[p] = b;
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

// Exclusive FP64 prefix sums of the first ns sorted keys of each dimension, in two
// passes over chunks of 1,024 keys.  k_prefix_local: each chunk's exclusive prefix sums
// (waves by shuffles, then the chunk's 16 wave totals in order) and the chunk total;
// k_prefix_add: each chunk adds the totals of the chunks before it, summed in order.
__global__ __launch_bounds__(1024) void k_prefix_local(const float* keys, long long np2, long long ns,
                                                       double* prefix, double* totals) {
  __shared__ double sw[16];
  const int b = blockIdx.x, d = blockIdx.y, t = threadIdx.x, w = t >> 6, l = t & 63;
  const long long i = (long long)b * 1024 + t;
  const double x = i < ns ? (double)keys[(long long)d * np2 + i] : 0.0;
  double v = x;
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const double o = __shfl_up(v, k, 64);
    if (l >= k) v = v + o;
  }
  if (l == 63) sw[w] = v;
  __syncthreads();
  double before = 0.0;
  for (int q = 0; q < w; ++q) before = before + sw[q];
  if (i < ns) prefix[(long long)d * (ns + 1) + i] = before + (v - x);
  if (t == 1023) totals[(long long)d * gridDim.x + b] = before + v;
}

__global__ __launch_bounds__(1024) void k_prefix_add(long long ns, double* prefix, const double* totals) {
  __shared__ double off_s;
  const int b = blockIdx.x, d = blockIdx.y, t = threadIdx.x;
  const double* tot = totals + (long long)d * gridDim.x;
  if (t == 0) {
    double o = 0.0;
    for (int q = 0; q < b; ++q) o = o + tot[q];
    off_s = o;
  }
  __syncthreads();
  const double off = off_s;
  const long long i = (long long)b * 1024 + t;
  double* pf = prefix + (long long)d * (ns + 1);
  if (i < ns) pf[i] = off + pf[i];
  if (b == (int)gridDim.x - 1 && t == 0) pf[ns] = off + tot[b];
}

// Lloyd iterations of one dimension; thread c owns centroid c.  Every stride-th sorted key
// sits in LDS (at most kLloydSamples of them), so each run boundary's binary search takes
// its first steps there and only the last log2(stride) in memory; the count it finds is
// the one a search over all keys finds.
constexpr int kLloydSamples = 8192;
__global__ __launch_bounds__(256) void k_lloyd(const float* keys, long long np2, long long ns,
                                               const double* prefix, int kcb, float* centroids) {
  __shared__ double C[256];
  __shared__ long long ends[256];
  __shared__ float smp[kLloydSamples];
  const int d = blockIdx.x, c = threadIdx.x;
  const float* kk = keys + (long long)d * np2;
  const double* pf = prefix + (long long)d * (ns + 1);
  long long stride = 1;
  while ((ns + stride - 1) / stride > kLloydSamples) stride <<= 1;
  const int nsmp = (int)((ns + stride - 1) / stride);      // samples kk[q stride], q < nsmp
  for (int q = c; q < nsmp; q += 256) smp[q] = kk[(long long)q * stride];
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
      // q = #{samples <= beta}: key (q - 1) stride is <= beta and key q stride (if any) is
      // not, so the count lies in ((q - 1) stride, q stride]
      int qlo = 0, qhi = nsmp;
      while (qlo < qhi) {
        const int mid = (qlo + qhi) >> 1;
        if ((double)smp[mid] <= beta) qlo = mid + 1;
        else qhi = mid;
      }
      long long lo = qlo == 0 ? 0 : (long long)(qlo - 1) * stride + 1;
      long long hi = min((long long)qlo * stride, ns);
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

// Workspace: the keys [latent][np2] (FP32), the prefix sums [latent][ns + 1] and the chunk
// totals [latent][ceil(ns / 1024)] (FP64), each part 256-byte aligned.
static size_t align_up256(size_t x) { return (x + 255) / 256 * 256; }
size_t codebook_ws_bytes(long long n, int latent, long long every) {
  const long long ns = (n + every - 1) / every;
  const long long np2 = std::max<long long>(next_pow2(ns), 2);
  const long long nch = (ns + 1023) / 1024;
  return align_up256((size_t)latent * np2 * 4) + align_up256((size_t)latent * (ns + 1) * 8) +
         (size_t)latent * nch * 8;
}

hipError_t launch_codebook_fit(const float* z, long long n, int latent, long long every, int bits,
                               float* centroids, void* ws, hipStream_t st) {
  const long long ns = (n + every - 1) / every;
  const long long np2 = std::max<long long>(next_pow2(ns), 2);
  const long long nch = (ns + 1023) / 1024;
  float* keys = (float*)ws;
  double* prefix = (double*)((uint8_t*)ws + align_up256((size_t)latent * np2 * 4));
  double* totals = (double*)((uint8_t*)prefix + align_up256((size_t)latent * (ns + 1) * 8));
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
  hipLaunchKernelGGL(k_prefix_local, dim3((unsigned)nch, latent), dim3(1024), 0, st, keys, np2, ns, prefix, totals);
  hipLaunchKernelGGL(k_prefix_add, dim3((unsigned)nch, latent), dim3(1024), 0, st, ns, prefix, totals);
  hipLaunchKernelGGL(k_lloyd, dim3(latent), dim3(256), 0, st, keys, np2, ns, prefix, 1 << bits, centroids);
  return hipGetLastError();
}

}  // namespace hcz
