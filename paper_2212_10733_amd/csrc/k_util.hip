// Stream assembly: exclusive scan of record sizes into offsets, compaction of the staged
// records into the residual stream (in histogram order), and the run statistics.
#include "hcz_internal.h"

namespace hcz {

constexpr int kScanNT = 1024;
constexpr int kScanItems = 4;
constexpr long long kScanTile = (long long)kScanNT * kScanItems;

// Inclusive scan of one value per thread over the block; returns the block total.
__device__ uint64_t block_incl_scan(uint64_t& v, uint64_t* sw) {
  const int t = threadIdx.x, w = t >> 6, l = t & 63;
#pragma unroll
  for (int k = 1; k < 64; k <<= 1) {
    const uint64_t o = __shfl_up(v, k, 64);
    if (l >= k) v += o;
  }
  if (l == 63) sw[w] = v;
  __syncthreads();
  if (w == 0) {
    uint64_t x = (l < kScanNT / 64) ? sw[l] : 0;
#pragma unroll
    for (int k = 1; k < 64; k <<= 1) {
      const uint64_t o = __shfl_up(x, k, 64);
      if (l >= k) x += o;
    }
    if (l < kScanNT / 64) sw[l] = x;
  }
  __syncthreads();
  const uint64_t total = sw[kScanNT / 64 - 1];
  if (w > 0) v += sw[w - 1];
  __syncthreads();
  return total;
}

__global__ __launch_bounds__(kScanNT) void k_scan_reduce(const uint64_t* sizes, long long H,
                                                         uint64_t* partial) {
  __shared__ uint64_t sw[kScanNT / 64];
  const long long base = blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < H) s += sizes[base + k];
  const uint64_t total = block_incl_scan(s, sw);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of the per-tile totals, in one block, tile by tile with a carry.
__global__ __launch_bounds__(kScanNT) void k_scan_partials(uint64_t* partial, long long nb) {
  __shared__ uint64_t sw[kScanNT / 64];
  uint64_t carry = 0;
  for (long long b0 = 0; b0 < nb; b0 += kScanNT) {
    const long long i = b0 + threadIdx.x;
    uint64_t v = i < nb ? partial[i] : 0;
    const uint64_t x = v;
    const uint64_t total = block_incl_scan(v, sw);
    if (i < nb) partial[i] = carry + v - x;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[nb] = carry;
}

__global__ __launch_bounds__(kScanNT) void k_scan_final(const uint64_t* sizes, long long H,
                                                        const uint64_t* partial, long long nb,
                                                        uint64_t* offsets) {
  __shared__ uint64_t sw[kScanNT / 64];
  const long long base = blockIdx.x * kScanTile + (long long)threadIdx.x * kScanItems;
  uint64_t v[kScanItems];
  uint64_t s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = (base + k < H) ? sizes[base + k] : 0;
    s += v[k];
  }
  uint64_t incl = s;
  block_incl_scan(incl, sw);
  uint64_t run = partial[blockIdx.x] + incl - s;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < H) offsets[base + k] = run;
    run += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) offsets[H] = partial[nb];
}

size_t scan_partial_elems(long long H) { return (size_t)((H + kScanTile - 1) / kScanTile) + 1; }

hipError_t launch_scan(const uint64_t* sizes, uint64_t* offsets, long long H, uint64_t* partial,
                       hipStream_t st) {
  const long long nb = (H + kScanTile - 1) / kScanTile;
  if (nb == 0) {
    hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanNT), 0, st, partial, 0LL);
    hipLaunchKernelGGL(k_scan_final, dim3(1), dim3(kScanNT), 0, st, sizes, 0LL, partial, 0LL, offsets);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanNT), 0, st, sizes, H, partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kScanNT), 0, st, partial, nb);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nb), dim3(kScanNT), 0, st, sizes, H, partial, nb, offsets);
  return hipGetLastError();
}

// One wave per record: copy the staged record to its offset in the stream as 32-bit words
// (record sizes and offsets are multiples of 4).  Records that would end past the
// capacity are not written.
__global__ __launch_bounds__(256) void k_compact(const uint8_t* slots, long long slot_stride,
                                                 const uint64_t* offsets, const uint64_t* sizes,
                                                 long long H, uint8_t* out, uint64_t capacity) {
  const long long h = (long long)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int l = threadIdx.x & 63;
  if (h >= H) return;
  const uint64_t sz = sizes[h], off = offsets[h];
  if (sz == 0 || off + sz > capacity) return;
  const uint32_t* __restrict__ src = (const uint32_t*)(slots + h * slot_stride);
  uint32_t* __restrict__ dst = (uint32_t*)(out + off);
  const uint64_t nw = sz >> 2;
  // eight words per lane in flight at a time: the loads are clamped to the record's last
  // word so that all of them issue together, the stores past the end are skipped (slot
  // and stream never overlap)
  for (uint64_t k0 = l; k0 < nw; k0 += 512) {
    uint32_t v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = src[min(k0 + 64 * j, nw - 1)];
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (k0 + 64 * j < nw) dst[k0 + 64 * j] = v[j];
  }
}

hipError_t launch_compact(const uint8_t* slots, long long slot_stride, const uint64_t* offsets,
                          const uint64_t* sizes, long long H, uint8_t* out, uint64_t capacity,
                          hipStream_t st) {
  if (H <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_compact, dim3((unsigned)((H + 3) / 4)), dim3(256), 0, st, slots, slot_stride,
                     offsets, sizes, H, out, capacity);
  return hipGetLastError();
}

__global__ void k_stats_zero(hcz_stats* s) {
  uint64_t* p = (uint64_t*)s;
  for (int i = threadIdx.x; i < (int)(sizeof(hcz_stats) / 8); i += blockDim.x) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_stats(const uint8_t* flags, const uint8_t* kstar,
                                               const uint16_t* iters, const uint64_t* offsets,
                                               long long H, uint64_t capacity, hcz_stats* s) {
  __shared__ unsigned long long c[3 + 64 + 48 + 2];
  for (int i = threadIdx.x; i < 3 + 64 + 48 + 2; i += 256) c[i] = 0;
  __syncthreads();
  for (long long h = (long long)blockIdx.x * 256 + threadIdx.x; h < H; h += (long long)gridDim.x * 256) {
    const int fl = flags[h];
    if (fl & HCZ_FLAG_CODED) atomicAdd(&c[0], 1ull);
    if (fl & HCZ_FLAG_ROUND2) atomicAdd(&c[1], 1ull);
    if (fl & HCZ_FLAG_RAW) atomicAdd(&c[2], 1ull);
    const int it = iters[h];
    atomicAdd(&c[3 + min(it, 63)], 1ull);
    if (kstar[h] != 0xff) atomicAdd(&c[3 + 64 + min((int)kstar[h], 47)], 1ull);
    atomicAdd(&c[3 + 64 + 48], (unsigned long long)it);
    atomicMax(&c[3 + 64 + 48 + 1], (unsigned long long)it);
  }
  __syncthreads();
  unsigned long long* g = (unsigned long long*)s;
  if (threadIdx.x < 3) {
    if (c[threadIdx.x]) atomicAdd(&g[1 + threadIdx.x], c[threadIdx.x]);
  } else if (threadIdx.x < 3 + 64 + 48) {
    const int k = threadIdx.x - 3;
    if (c[threadIdx.x]) atomicAdd(&g[8 + k], c[threadIdx.x]);
  } else if (threadIdx.x == 3 + 64 + 48) {
    atomicAdd(&g[7], c[3 + 64 + 48]);
    atomicMax(&g[6], c[3 + 64 + 48 + 1]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    s->n_hist = (uint64_t)H;
    s->stream_bytes = offsets[H];
    s->overflow = offsets[H] > capacity ? 1 : 0;
  }
}

hipError_t launch_stats(const uint8_t* flags, const uint8_t* kstar, const uint16_t* iters,
                        const uint64_t* offsets, long long H, uint64_t capacity, hcz_stats* stats,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_stats_zero, dim3(1), dim3(256), 0, st, stats);
  const long long nb = H <= 0 ? 1 : std::min<long long>((H + 255) / 256, 1024);
  hipLaunchKernelGGL(k_stats, dim3((unsigned)nb), dim3(256), 0, st, flags, kstar, iters, offsets, H,
                     capacity, stats);
  return hipGetLastError();
}


// ---- batches of subdomains -----------------------------------------------------------------

// tau_hist[h] = seg_tau[s] with s the last segment whose start is <= h (starts clamped)
__global__ __launch_bounds__(256) void k_segment_tau(const int64_t* start, const double* tau, int nseg,
                                                     long long H, double* out) {
  const long long h = (long long)blockIdx.x * 256 + threadIdx.x;
  if (h >= H) return;
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= h) lo = mid;
    else hi = mid - 1;
  }
  out[h] = tau[lo];
}

// one workgroup per segment: the maximum of t over its histograms
__global__ __launch_bounds__(256) void k_segment_max(const int64_t* start, long long H, const uint64_t* t,
                                                     uint64_t* out) {
  __shared__ uint64_t red[256];
  const int s = blockIdx.x;
  const long long lo = min(max(start[s], (int64_t)0), (int64_t)H);
  const long long hi = min(max(start[s + 1], (int64_t)lo), (int64_t)H);
  uint64_t m = 0;
  for (long long h = lo + threadIdx.x; h < hi; h += 256) m = max(m, t[h]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = max(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[s] = red[0];
}

__global__ void k_timestamp(uint64_t* dst) { *dst = wall_clock64(); }

hipError_t launch_segment_tau(const int64_t* start, const double* tau, int nseg, long long H, double* out,
                              hipStream_t st) {
  if (H <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_segment_tau, dim3((unsigned)((H + 255) / 256)), dim3(256), 0, st, start, tau, nseg, H, out);
  return hipGetLastError();
}

hipError_t launch_segment_max(const int64_t* start, int nseg, long long H, const uint64_t* t, uint64_t* out,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_segment_max, dim3((unsigned)nseg), dim3(256), 0, st, start, H, t, out);
  return hipGetLastError();
}

hipError_t launch_timestamp(uint64_t* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_timestamp, dim3(1), dim3(1), 0, st, dst);
  return hipGetLastError();
}

}  // namespace hcz
