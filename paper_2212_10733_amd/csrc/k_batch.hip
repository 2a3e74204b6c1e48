// The persistent batch form of the residual stage (Section III Stages 4-5) for subdomains
// on several grids at once (the paper's per-rank subdomains, Section III-A): one launch of
// two workgroups per CU that take work items from a device counter until the list is
// empty.  The list is the concatenation of the segments' items: four histograms of a
// wave-per-histogram grid (the 39 x 39 compiled shape or run-time slot tables) or one
// histogram of a grid beyond one wave, served by a team of four waves.  Each item stages
// its grid's tables like the per-grid launches do, so the records, flags and multipliers
// are those of the per-grid kernels bit for bit.  This translation unit also compiles the
// wave and wave-team kernels it calls.
#include "k_wave.hip"
#include "k_team.hip"

namespace hcz {

__global__ void k_zero_u64(unsigned long long* p) { *p = 0ull; }

template <typename TIn, bool UVOL>
__global__ __launch_bounds__(256, 2) void k_residual_batch(BatchArgs B) {
  extern __shared__ double smem[];
  __shared__ long long s_item;
  for (;;) {
    __syncthreads();                            // the previous item is done with LDS and s_item
    if (threadIdx.x == 0) s_item = (long long)atomicAdd(B.counter, 1ull);
    __syncthreads();
    const long long item = s_item;
    if (item >= B.nitems) break;                // every thread read the same item: a uniform exit
    int s = 0;
#pragma unroll
    for (int q = 1; q < kBatchSeg; ++q)
      if (q < B.nseg && item >= B.s[q].item0) s = q;
    const GridDev& G = B.s[s].G;
    const ResidualArgs& a = B.s[s].a;
    const long long t0 = item - B.s[s].item0;
    const int kind = B.s[s].kind;
    if (kind == kBatchTeam4) {
      Team<4> T = setup_team<4>(G, smem);
      T.sync();
      residual_t_hist<TIn, UVOL, 4>(G, a, T, t0);
    } else {
      const int wv = threadIdx.x >> 6;
      const long long h = t0 * kWPB + wv;
      PreRows<TIn, ShapeDyn> P;
      const WaveLds L = setup_lds(G, smem, wv);
      __syncthreads();
      if (h < a.H) residual_w_hist<TIn, UVOL, ShapeDyn>(G, a, L, h, P);
    }
  }
}

// LDS of a segment's kernel body.
size_t batch_lds_bytes(const BatchSeg& S) {
  return S.kind == kBatchTeam4 ? lds_bytes_t<4>(S.G) : lds_bytes_w(S.G);
}

hipError_t launch_residual_batch(BatchArgs B, int dtype, bool uvol, int grid, hipStream_t st) {
  long long items = 0;
  size_t lds = 0;
  for (int s = 0; s < B.nseg; ++s) {
    B.s[s].item0 = items;
    items += B.s[s].kind == kBatchTeam4 ? B.s[s].a.H : (B.s[s].a.H + kWPB - 1) / kWPB;
    lds = std::max(lds, batch_lds_bytes(B.s[s]));
  }
  B.nitems = items;
  if (items <= 0) return hipSuccess;
  const void* fn = dtype == HCZ_F32 ? (uvol ? (const void*)k_residual_batch<float, true> : (const void*)k_residual_batch<float, false>)
                                    : (uvol ? (const void*)k_residual_batch<double, true> : (const void*)k_residual_batch<double, false>);
  if (grid <= 0) {
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, lds)) != hipSuccess) return e;
    grid = std::max(1, cus * std::max(1, per_cu));
  }
  grid = (int)std::min<long long>(grid, items);
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, B.counter);
  const dim3 g((unsigned)grid), b(256);
  if (dtype == HCZ_F32) {
    if (uvol) hipLaunchKernelGGL((k_residual_batch<float, true>), g, b, lds, st, B);
    else hipLaunchKernelGGL((k_residual_batch<float, false>), g, b, lds, st, B);
  } else {
    if (uvol) hipLaunchKernelGGL((k_residual_batch<double, true>), g, b, lds, st, B);
    else hipLaunchKernelGGL((k_residual_batch<double, false>), g, b, lds, st, B);
  }
  return hipGetLastError();
}

}  // namespace hcz
