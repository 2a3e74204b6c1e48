// Internal declarations of libhcz: device-side grid tables, kernel argument blocks,
// block reductions and the launch functions each kernel file exports to the host API.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <cfloat>

#include "../../include/hcz.h"

#pragma clang fp contract(off)

namespace hcz {

constexpr int kMaxDim = 128;        // largest n_par / n_perp of a grid
constexpr int kMaxN = 4608;         // largest n_par * n_perp (keeps per-block LDS < 64 KB)
constexpr int kMaxLev = 9;          // L + 1 for n <= 128 is at most 8
constexpr int kLadder = 41;         // quantisation ladder k = 0..40
constexpr int kWaveSlots = 26;     // slots of 64 nodes a wave-per-histogram kernel holds
constexpr int kTeamSlots2 = 22;    // slots of 128 nodes a team of two waves holds
constexpr int kTeamSlots4 = 20;    // slots of 256 nodes a team of four waves holds
constexpr int kHidden = 128;
constexpr int kLatent = 16;

// Selection / feasibility margin 1 - 2^-20 and ladder margin 2 (1 - 2^-19).
constexpr double kSelMargin = 1.0 - 0x1p-20;
constexpr double kLadderMargin = 2.0 * (1.0 - 0x1p-19);
constexpr double kQMax = 1073741824.0;   // 2^30: larger integer coefficients go verbatim
constexpr double kGTol = 1e-13;          // Newton stopping rule
constexpr double kPivTol = 1e-14;        // Cholesky pivot test relative to trace(H)
constexpr double kArmijoC = 1e-4;
constexpr int kArmijoHalvings = 40;

// Device copy of the grid: moment basis and the multilevel node layout.
struct GridDev {
  int n_par, n_perp, N, L, nlev, hdr_bytes, uniform_vol;
  int gstart[kMaxLev + 1];     // coefficient groups in packing order, coarsest first
  double vol0;                 // the cell volume when uniform
  double sqrtN;                // sqrt(N)
  double den;                  // sqrt(N) * (L + 1)
  double Vpar, Vperp, mass;
  const double* vol;           // [N] cell volumes (natural order e = j * n_par + i)
  const double* apar;          // [n_par]  v_par / V_par
  const double* cperp;         // [n_perp] (v_perp / V_perp)^2
  const uint32_t* node_ij;     // [N] packing order -> i | j << 16
  const uint8_t* lev_par;      // [n_par] finest level whose node set holds i (L at the ends)
  const uint8_t* a_par;        // [n_par] lower bracket of i at level lev + 1
  const uint8_t* b_par;        // [n_par] upper bracket
  const double* s_par;         // [n_par] (i - a) / (b - a)
  const uint8_t* lev_perp;
  const uint8_t* a_perp;
  const uint8_t* b_perp;
  const double* s_perp;
  // Wave-per-histogram layout: the nodes split into nslots slots of 64 (one node per
  // lane), each slot within one coefficient group except slot 0, which holds the
  // ncoarse coarsest groups in order.  Within a group, nodes with linear interpolation
  // come before bilinear ones.  nslots = 0: grid too large for the wave kernels.
  int nslots, ncoarse, nw;
  int8_t slot_group[kWaveSlots];     // -1 for the multi-group slot 0
  uint32_t slot_bil;                 // bit s: slot s uses the four-corner form
  uint32_t slot_sync;                // bit s: the next slot belongs to a later group
  uint32_t slot_keep;                // bit s: later groups read slot s (not the finest group)
  uint32_t slot_half;                // bit s: every weight of slot s is exactly 1/2
  const uint32_t* slot_meta;         // [nslots * 64][3], see make_slots()
  const uint16_t* slot_rank;         // [nslots * 64] packing rank of each entry within its group
  const double* wtab;                // [nw] distinct interpolation weights, wtab[0] = 0
  // Wave-team layout (a team of W waves per histogram, for grids beyond one wave): the same
  // scheme with slots of 64 W nodes, index 0 for W = 2 and 1 for W = 4; tnslots[k] = 0
  // where the grid does not fit that team.
  int tnslots[2], tncoarse[2], tnw[2];
  uint32_t tslot_bil[2], tslot_sync[2], tslot_keep[2];
  const uint32_t* tslot_meta[2];     // [tnslots * 64 W][3]
  const uint16_t* tslot_rank[2];     // [tnslots * 64 W]
  const double* twtab[2];            // [tnw]
};

struct ModelDev {
  int N, hidden, latent, kpad;     // kpad: N rounded up to the encoder's K chunk
  const float* W1p;                // [hidden][kpad] zero padded
  const float* b1;
  const float* W2;                 // [latent][hidden]
  const float* b2;
  const float* W3;                 // [hidden][latent]
  const float* b3;
  const float* W4p;                // [npad][hidden] rows >= N zero, k permuted for MFMA
  const float* b4;                 // [N]
  const float* mu;                 // [N]
  const float* rsd;                // [N] 1 / sigma (encoder side)
  const float* sd;                 // [N] sigma (decoder side)
  int npad;
  int bf16;                        // 1: the BF16 form (W1b, W1m, W4m below)
  const uint16_t* W1b;             // [hidden][kpad] bfloat16 of W1, zero padded
  const uint16_t* W1m;             // bfloat16 of W1 in matrix-core operand order (see k_encode_b2)
  const uint16_t* W4m;             // bfloat16 of W4 in matrix-core operand order (see k_decode_b2)
  int fp64;                        // 1: the FP64 form (the FP64 copies below)
  const double* W1t;               // [N][hidden], W1 transposed
  const double* b1d;
  const double* W2d;               // [latent][hidden]
  const double* b2d;
  const double* W3d;               // [hidden][latent]
  const double* b3d;
  const double* W4t;               // [hidden][N], W4 transposed
  const double* b4d;
  const double* mud;               // [N]
  const double* sdd;               // [N]
  // convolutional model (39 x 39 grids), arch == HCZ_ARCH_CONV
  int arch;
  const float* c1w;                // [32][9]
  const float* c1b;                // [32]
  const uint16_t* c2w;             // bfloat16 [tap][64 out][32 in]
  const float* c2b;                // [64]
  const float* fw;                 // [16][6400]
  const float* fb;                 // [16]
  const float* dw;                 // [6400][16]
  const float* db;                 // [6400]
  const uint16_t* t1w;             // bfloat16 [tap][32 out][64 in]
  const float* t1b;                // [32]
  const float* t2w;                // [32][9]
  const float* t2b;                // [1]
  float* scratch;                  // [kConvChunk][6400] FP32, owned by the model
};
constexpr int kConvChunk = 16384;  // histograms per pass of the convolutional model

struct ResidualArgs {
  const void* hist;
  int dtype;
  long long hs, rs, H;
  const float* fhat;           // [H][N] or null
  double tau;
  int tau_mode;
  double newton_s;
  int max_iter, max_iter2, fallback;
  void* lambda;                // [H][4] FP64, or FP32 when lambda_fp32
  int lambda_fp32;
  int no_positivity;           // 1: projection onto {A x = b} only (flag HCZ_FLAG_NOCLIP)
  int kl;                      // 1: KL correction where it keeps the bound (flag HCZ_FLAG_KL)
  int lambda_bits;             // 0, or stored multipliers rounded to this many mantissa bits
  int ub_k;                    // -1: search the ladder; 0..40: this ladder step, no search
  int k_start;                 // -1: bisection over [0, 41); else the exponential search's first probe
  int variant;                 // HCZ_VARIANT_*: kernel family and shape of the launch
  uint8_t* flags;              // [H]
  uint64_t* sizes;             // [H] record bytes
  uint8_t* slots;              // [H][slot_stride] staging
  long long slot_stride;
  uint8_t* kstar;              // [H] 0xff if not coded
  uint16_t* iters;             // [H]
  const double* lam0;          // [H][4] warm start or null
  int analytic;                // 1: warm start (A A^T)^-1 (A ft - b), formed in the kernel
  const double* tau_hist;      // [H] per-histogram tau, or null (tau for all)
  unsigned long long* t_done;  // [H] wall clock at the end of each histogram, or null
};

// One grid's share of the persistent batch launch of the residual stage.
constexpr int kBatchSeg = 4;                   // grids per batch launch
enum { kBatchWave = 0, kBatchTeam4 = 1 };
struct BatchSeg {
  GridDev G;
  ResidualArgs a;
  int kind;                    // kBatchWave (4 histograms per item), kBatchTeam4 (1)
  long long item0;             // first work item of the segment in the batch's list
};
struct BatchArgs {
  BatchSeg s[kBatchSeg];
  int nseg;
  long long nitems;
  unsigned long long* counter; // the work counter (device), zeroed by the launch itself
};

struct DecompressArgs {
  const uint8_t* flags;
  const void* lambda;          // FP64, or FP32 when lambda_fp32
  int lambda_fp32;
  const uint64_t* offsets;
  const uint8_t* stream;
  int in_dtype;
  long long H;
  const float* fhat;           // [H][N] or null
  void* out;
  int out_dtype;
  uint64_t capacity;           // bytes of `stream`; records ending past it decode to NaN
};

// v rounded to `bits` explicit mantissa bits (nearest, ties to even); bits = 0 or >= 52
// keeps v.  A carry out of the mantissa moves into the exponent, as it should.
__host__ __device__ inline double round_mantissa(double v, int bits) {
  if (bits <= 0 || bits >= 52) return v;
  unsigned long long u;
  __builtin_memcpy(&u, &v, 8);
  const int drop = 52 - bits;
  const unsigned long long half = (1ull << (drop - 1)) - 1ull + ((u >> drop) & 1ull);
  u = (u + half) & ~((1ull << drop) - 1ull);
  __builtin_memcpy(&v, &u, 8);
  return v;
}

// Quantised coefficient Dk * q, q = rint(d / Dk) taken as an integer: rint of a small
// negative value is -0, which the integer turns into +0.
__device__ __forceinline__ double qdelta(double Dk, double d, double inv) {
  return __dmul_rn(Dk, __dadd_rn(rint(__dmul_rn(d, inv)), 0.0));
}

// ---- double-double accumulation (exact TwoSum error terms) --------------------------
struct dd { double hi, lo; };

__device__ __forceinline__ dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double err = (a - (s - bb)) + (b - bb);
  return {s, err};
}
__device__ __forceinline__ dd dd_add_d(dd a, double b) {
  dd s = two_sum(a.hi, b);
  s.lo += a.lo;
  double hi = s.hi + s.lo;
  double lo = s.lo - (hi - s.hi);
  return {hi, lo};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  s.lo += (a.lo + b.lo);
  double hi = s.hi + s.lo;
  double lo = s.lo - (hi - s.hi);
  return {hi, lo};
}

// ---- wave / block reductions ----------------------------------------------------------
// Butterflies with xor partners: each stage adds x_l + x_{l^k}, which both partners
// compute identically (addition commutes exactly), so every lane ends with the same
// bits and the order is fixed, i.e. results are run-to-run deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) v = v + __shfl_xor(v, k, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) v = fmax(v, __shfl_xor(v, k, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) v = fmin(v, __shfl_xor(v, k, 64));
  return v;
}
__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, k, 64));
  return v;
}
__device__ __forceinline__ dd wave_dd(dd v) {
#pragma unroll
  for (int k = 32; k >= 1; k >>= 1) {
    dd o{__shfl_xor(v.hi, k, 64), __shfl_xor(v.lo, k, 64)};
    v = dd_add(v, o);
  }
  return v;
}

// Sum K doubles over the block; every thread gets the same result.  `red` needs
// NT/64 * K doubles of LDS.  Contains two barriers.
template <int NT, int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double* red) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (l == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) red[w * K + k] = v[k];
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = red[k];
#pragma unroll
    for (int q = 1; q < NW; ++q) s = s + red[q * K + k];
    v[k] = s;
  }
  __syncthreads();
}

template <int NT>
__device__ __forceinline__ double block_max(double v, double* red) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  v = wave_max(v);
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) s = fmax(s, red[q]);
  __syncthreads();
  return s;
}

template <int NT>
__device__ __forceinline__ dd block_dd(dd v, double* red) {
  constexpr int NW = NT / 64;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  v = wave_dd(v);
  if (l == 0) { red[2 * w] = v.hi; red[2 * w + 1] = v.lo; }
  __syncthreads();
  dd s{red[0], red[1]};
#pragma unroll
  for (int q = 1; q < NW; ++q) s = dd_add(s, dd{red[2 * q], red[2 * q + 1]});
  __syncthreads();
  return s;
}

// ---- multilevel interpolation ----------------------------------------------------------
// Per node of the decomposition: the four corner offsets of its interpolation cell and
// the weights s (along v_par) and t (along v_perp).  A node on a coarse line has the two
// corners of that line repeated and weight 0 across it; the bilinear formula then
// reduces exactly to the linear one.
struct Interp {
  uint16_t e00, e10, e01, e11;
  double s, t;
};

__device__ __forceinline__ Interp make_interp(const GridDev& G, int i, int j) {
  const int li = G.lev_par[i], lj = G.lev_perp[j];
  int ia = i, ib = i, ja = j, jb = j;
  double s = 0.0, t = 0.0;
  if (li <= lj) { ia = G.a_par[i]; ib = G.b_par[i]; s = G.s_par[i]; }
  if (lj <= li) { ja = G.a_perp[j]; jb = G.b_perp[j]; t = G.s_perp[j]; }
  Interp r;
  r.e00 = (uint16_t)(ja * G.n_par + ia);
  r.e10 = (uint16_t)(ja * G.n_par + ib);
  r.e01 = (uint16_t)(jb * G.n_par + ia);
  r.e11 = (uint16_t)(jb * G.n_par + ib);
  r.s = s;
  r.t = t;
  return r;
}

// p0 = y00 + s (y10 - y00), p1 = y01 + s (y11 - y01), P = p0 + t (p1 - p0), unfused.
__device__ __forceinline__ double predict(const double* y, const Interp& c) {
  const double y00 = y[c.e00], y10 = y[c.e10], y01 = y[c.e01], y11 = y[c.e11];
  const double p0 = __dadd_rn(y00, __dmul_rn(c.s, __dsub_rn(y10, y00)));
  const double p1 = __dadd_rn(y01, __dmul_rn(c.s, __dsub_rn(y11, y01)));
  return __dadd_rn(p0, __dmul_rn(c.t, __dsub_rn(p1, p0)));
}

// 2^(m/4), m = 0..3, correctly rounded.
__device__ __forceinline__ double ladder_c(int m) {
  return m == 0 ? 1.0 : (m == 1 ? 0x1.306fe0a31b715p+0 : (m == 2 ? 0x1.6a09e667f3bcdp+0 : 0x1.ae89f995ad3adp+0));
}
__device__ __forceinline__ double ladder(double d0, int k) {
  return __dmul_rn(ldexp(d0, k >> 2), ladder_c(k & 3));
}

// The bound search over the ladder, uniform across the threads that run it: a bisection
// of [lo, hi), optionally preceded by an exponential search from k_start that brackets the
// feasibility boundary (probe k_start; climb +1, +3, +7, ... while feasible, or descend
// -1, -3, ... while infeasible).  next() gives the next probe or -1 when k* = lo is found.
struct LadderSearch {
  int lo, hi, step, phase, k0;   // phase 0: first probe, 1: climbing, 2: descending, 3: bisection
  __device__ __forceinline__ void init(int ub_k, int k_start) {
    step = 1;
    k0 = k_start;
    lo = 0;
    hi = kLadder;
    phase = k_start < 0 ? 3 : 0;
    if (ub_k >= 0) { lo = ub_k; hi = ub_k + 1; phase = 3; }
  }
  __device__ __forceinline__ int next() {
    if (phase == 1 && lo + step >= kLadder) phase = 3;
    if (phase == 2 && hi - step <= 0) { lo = 0; phase = 3; }
    if (phase == 0) return k0;
    if (phase == 1) return lo + step;
    if (phase == 2) return hi - step;
    return hi - lo > 1 ? (lo + hi) >> 1 : -1;
  }
  __device__ __forceinline__ void result(int t, bool ok) {
    if (phase == 0) {
      if (ok) { lo = t; phase = 1; } else { hi = t; phase = 2; }
    } else if (phase == 1) {
      if (ok) { lo = t; step <<= 1; } else { hi = t; phase = 3; }
    } else if (phase == 2) {
      if (ok) { lo = t; phase = 3; } else { hi = t; step <<= 1; }
    } else {
      if (ok) lo = t; else hi = t;
    }
  }
};

// Per-cell constraint coefficients vol * phi_k and the correction A^T lambda, in one
// fixed order shared by compression and decompression.
struct Aphi { double a0, a1, a2, a3; };
__device__ __forceinline__ Aphi make_aphi(const GridDev& G, int e, int i, int j) {
  const double v = G.uniform_vol ? G.vol0 : G.vol[e];
  const double ap = G.apar[i];
  Aphi r;
  r.a0 = v;
  r.a1 = __dmul_rn(v, ap);
  r.a2 = __dmul_rn(v, G.cperp[j]);
  r.a3 = __dmul_rn(r.a1, ap);
  return r;
}
__device__ __forceinline__ double correction(const Aphi& A, const double (&lam)[4]) {
  double c = __dmul_rn(lam[0], A.a0);
  c = __dadd_rn(c, __dmul_rn(lam[1], A.a1));
  c = __dadd_rn(c, __dmul_rn(lam[2], A.a2));
  return __dadd_rn(c, __dmul_rn(lam[3], A.a3));
}

// ---- launch functions (defined in the kernel files) -----------------------------------
hipError_t launch_qoi(const GridDev& G, const void* hist, int dtype, long long H, long long hs,
                      long long rs, double* b, double* qoi, double* norm, hipStream_t st);
hipError_t launch_residual(const GridDev& G, const ResidualArgs& a, hipStream_t st);
bool wave_path(const GridDev& G);
bool wave_fixed_path(const GridDev& G);
hipError_t launch_residual_w(const GridDev& G, const ResidualArgs& a, hipStream_t st);
hipError_t launch_decompress_w(const GridDev& G, const DecompressArgs& a, hipStream_t st);
hipError_t launch_decompress(const GridDev& G, const DecompressArgs& a, hipStream_t st);
hipError_t launch_scan(const uint64_t* sizes, uint64_t* offsets, long long H, uint64_t* partial,
                       hipStream_t st);
size_t scan_partial_elems(long long H);
hipError_t launch_compact(const uint8_t* slots, long long slot_stride, const uint64_t* offsets,
                          const uint64_t* sizes, long long H, uint8_t* out, uint64_t capacity,
                          hipStream_t st);
// Records msg as the calling thread's last error and returns s.
hcz_status set_error(hcz_status s, const char* msg);

hipError_t launch_segment_tau(const int64_t* start, const double* tau, int nseg, long long H, double* out,
                              hipStream_t st);
hipError_t launch_segment_max(const int64_t* start, int nseg, long long H, const uint64_t* t, uint64_t* out,
                              hipStream_t st);
hipError_t launch_timestamp(uint64_t* dst, hipStream_t st);
hipError_t launch_stats(const uint8_t* flags, const uint8_t* kstar, const uint16_t* iters,
                        const uint64_t* offsets, long long H, uint64_t capacity, hcz_stats* stats,
                        hipStream_t st);
hipError_t launch_encode(const ModelDev& M, const void* hist, int dtype, long long H, long long hs,
                         long long rs, int n_par, float* z, hipStream_t st);
hipError_t launch_decode(const ModelDev& M, const uint8_t* codes, const float* centroids, int bits,
                         long long H, float* fhat, hipStream_t st);
hipError_t launch_conv_encode(const ModelDev& M, const void* hist, int dtype, long long H, long long hs,
                              long long rs, float* z, hipStream_t st);
hipError_t launch_conv_decode(const ModelDev& M, const uint8_t* codes, const float* centroids, int bits,
                              long long H, float* fhat, hipStream_t st);
hipError_t launch_residual_t(const GridDev& G, const ResidualArgs& a, int W, hipStream_t st);
// Fills B's item0 and nitems from the segments' kinds and H; grid <= 0: as many workgroups
// as stay resident on the device.
hipError_t launch_residual_batch(BatchArgs B, int dtype, bool uvol, int grid, hipStream_t st);
bool team_path(const GridDev& G, int W);
hipError_t launch_cv_fwd(const float* in, int C, int n, int relu_in, const float* w, const float* bias, float* out,
                         int O, int m, long long B, hipStream_t st, int bf);
hipError_t launch_cvt_fwd(const float* in, int C, int n, int relu_in, const float* w, const float* bias, float* out,
                          int O, int m, long long B, hipStream_t st, int bf);
hipError_t launch_cv_wgrad(const float* coarse, int Cc, int m, int relu_c, const float* fine, int Cf, int n,
                           int relu_f, long long B, float* G, hipStream_t st, int bf);
hipError_t launch_chsum(const float* d, int C, int P, long long B, float* out, hipStream_t st);
hipError_t launch_relu_copy(const float* a, float* h, long long n, hipStream_t st);
hipError_t launch_quantize(const float* z, long long n, int latent, const float* centroids,
                           int bits, uint8_t* codes, hipStream_t st);
size_t codebook_ws_bytes(long long n, int latent, long long every);
hipError_t launch_gemm(const float* A, long long sam, long long sak, const float* B, long long sbk,
                       long long sbn, float* C, long long scm, long long M, long long Nc, long long K,
                       float alpha, float beta, const float* bias, int relu, hipStream_t st, int bf16 = 0);
hipError_t launch_relu_mask(float* d, const float* h, long long n, hipStream_t st);
hipError_t launch_colsum(const float* D, long long M, long long Nc, float* out, hipStream_t st);
size_t mse_ws_bytes();
hipError_t launch_mse(const float* xh, const float* x, long long n, float* loss, float* dxh, void* ws,
                      hipStream_t st);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, long long n, double lr, double b1,
                       double b2, double eps, long long step, hipStream_t st);
int mlp_param_count();
hipError_t launch_mlp_infer(const float* params, const double* scale, const uint8_t* codes,
                            const float* centroids, int bits, long long H, double* lam0, hipStream_t st);
hipError_t launch_dequant(const uint8_t* codes, long long n, int latent, const float* centroids, int bits,
                          float* z, hipStream_t st);
size_t norm_stats_ws_bytes(long long H, int N);
hipError_t launch_col_normalize(const void* x, int dtype, long long rows, long long cols, long long ld,
                                const float* mean, const float* sd, float* out, hipStream_t st);
hipError_t launch_norm_stats(const void* hist, int dtype, long long H, long long hs, long long rs, int n_par,
                             int N, float* mean, float* sd, void* ws, hipStream_t st);
hipError_t launch_codebook_fit(const float* z, long long n, int latent, long long every, int bits,
                               float* centroids, void* ws, hipStream_t st);

}  // namespace hcz
