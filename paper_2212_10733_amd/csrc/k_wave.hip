// Wave-per-histogram residual coding, Newton projection and decompression (Section III
// Stages 4-5 and decompression), for grids whose nodes fit in kWaveSlots slots of 64.
//
// Each 64-lane wave owns one histogram; a workgroup of four waves shares only the small
// per-grid tables in LDS, so after the first barrier no block-wide synchronisation is
// needed.  Lane l holds, per slot, one node of the multilevel decomposition (residual r
// and coefficient d in registers, interpolation cell in packed form).  A per-wave FP64
// buffer in LDS carries the values the recomposition reads from coarser groups; since a
// wave's LDS operations complete in order, a compiler fence between groups is all the
// ordering needed.  Reductions are DPP butterflies within the wave with the result taken
// from lane 63, so every lane sees the same bits and runs repeat bitwise.
// The Newton projection runs in natural element order (lane l, elements l + 64 m).
#include "hcz_internal.h"

namespace hcz {

constexpr int kWPB = 4;   // waves (histograms) per workgroup

// ---- wave-level primitives -------------------------------------------------------------

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const int lo2 = __builtin_amdgcn_update_dpp(0, lo, CTRL, ROWS, 0xF, false);
  const int hi2 = __builtin_amdgcn_update_dpp(0, hi, CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi2, lo2);
}

__device__ __forceinline__ double lane63(double v) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
  return __hiloint2double(hi, lo);
}

// quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror, then
// row_bcast:15 into rows 1 and 3 and row_bcast:31 into rows 2 and 3: lane 63 ends with
// the total.
#define HCZ_WAVE_REDUCE(v, OP)                                    \
  do {                                                            \
    v = OP(v, dpp_d<0xB1, 0xF>(v));                               \
    v = OP(v, dpp_d<0x4E, 0xF>(v));                               \
    v = OP(v, dpp_d<0x141, 0xF>(v));                              \
    v = OP(v, dpp_d<0x140, 0xF>(v));                              \
    v = OP(v, dpp_d<0x142, 0xA>(v));                              \
    v = OP(v, dpp_d<0x143, 0xC>(v));                              \
  } while (0)

__device__ __forceinline__ double op_add(double a, double b) { return a + b; }
__device__ __forceinline__ double op_max(double a, double b) { return fmax(a, b); }

__device__ __forceinline__ double wsum(double v) {
  HCZ_WAVE_REDUCE(v, op_add);
  return lane63(v);
}
__device__ __forceinline__ double lane_d(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

__device__ __forceinline__ double wmax(double v) {
  // a masked-out row of a row_bcast reads 0, which must not enter a max of possibly
  // negative values: reduce within rows by DPP, then across the four rows by readlane
  v = fmax(v, dpp_d<0xB1, 0xF>(v));
  v = fmax(v, dpp_d<0x4E, 0xF>(v));
  v = fmax(v, dpp_d<0x141, 0xF>(v));
  v = fmax(v, dpp_d<0x140, 0xF>(v));
  const double r0 = lane_d(v, 15);
  const double r1 = lane_d(v, 31), r2 = lane_d(v, 47), r3 = lane_d(v, 63);
  return fmax(fmax(r0, r1), fmax(r2, r3));
}

__device__ __forceinline__ uint32_t wumax(uint32_t v) {
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false));
  v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false));
  return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ dd wdd(dd v) {
#define HCZ_DD_STEP(C, R) v = dd_add(v, dd{dpp_d<C, R>(v.hi), dpp_d<C, R>(v.lo)})
  HCZ_DD_STEP(0xB1, 0xF);
  HCZ_DD_STEP(0x4E, 0xF);
  HCZ_DD_STEP(0x141, 0xF);
  HCZ_DD_STEP(0x140, 0xF);
  HCZ_DD_STEP(0x142, 0xA);
  HCZ_DD_STEP(0x143, 0xC);
#undef HCZ_DD_STEP
  return dd{lane63(v.hi), lane63(v.lo)};
}

// ---- node arithmetic --------------------------------------------------------------------

struct Node {
  uint32_t w0, w1;
};
__device__ __forceinline__ int n_e(const Node& n) { return n.w0 & 0x1fff; }
__device__ __forceinline__ int n_g(const Node& n) { return (n.w0 >> 13) & 0xf; }
__device__ __forceinline__ bool n_bil(const Node& n) { return (n.w0 >> 17) & 1u; }
__device__ __forceinline__ bool n_valid(const Node& n) { return (n.w0 >> 18) & 1u; }

// Interpolated value at a node from y, in the fixed unfused order of the coder.
__device__ __forceinline__ double predict_n(const double* y, const double* wt, const Node& n, int np) {
  const int a = n.w1 & 0x7f, b = (n.w1 >> 7) & 0x7f, aj = (n.w1 >> 14) & 0x7f, bj = (n.w1 >> 21) & 0x7f;
  const double s = wt[(n.w0 >> 19) & 0x3f];
  if (!n_bil(n)) {
    const double y0 = y[aj * np + a], y1 = y[bj * np + b];
    return __dadd_rn(y0, __dmul_rn(s, __dsub_rn(y1, y0)));
  }
  const double y00 = y[aj * np + a], y10 = y[aj * np + b], y01 = y[bj * np + a], y11 = y[bj * np + b];
  const double t = wt[(n.w0 >> 25) & 0x3f];
  const double p0 = __dadd_rn(y00, __dmul_rn(s, __dsub_rn(y10, y00)));
  const double p1 = __dadd_rn(y01, __dmul_rn(s, __dsub_rn(y11, y01)));
  return __dadd_rn(p0, __dmul_rn(t, __dsub_rn(p1, p0)));
}

// Hide a value from loop-invariant code motion: without this the compiler hoists every
// node's decoded corners and weights out of the bisection and Newton loops, which
// multiplies the live registers and spills.
__device__ __forceinline__ Node opaque(Node n) {
  asm volatile("" : "+v"(n.w0), "+v"(n.w1));
  return n;
}
__device__ __forceinline__ int opaque_i(int v) {
  asm volatile("" : "+v"(v));
  return v;
}

// y = dq + P (or dq on the coarsest group), stored at the node's offset.
__device__ __forceinline__ double recompose_node(double* y, const double* wt, const Node& n, double dq, int np) {
  const double v = n_g(n) == 0 ? dq : __dadd_rn(dq, predict_n(y, wt, n, np));
  y[n_e(n)] = v;
  return v;
}

// Correction A^T lam at one cell: vol * (lam0 + lam1 a + lam2 c + lam3 a^2), one fixed
// order for compression and decompression.
__device__ __forceinline__ double corr_cell(const double (&lam)[4], double vol, double a, double c) {
  double p = fma(lam[3], a, lam[1]);
  p = fma(p, a, lam[0]);
  p = fma(lam[2], c, p);
  return vol * p;
}

// Recompose every node at step Dk (1/Dk = inv) into y; returns sum (r - y)^2 over the
// histogram (same value in all lanes).  Slots after the first are independent within a
// group; a fence separates groups.
template <int NS>
__device__ __forceinline__ double recompose_all(const GridDev& G, double* y, const double* wt, const uint2* meta,
                                const int* ssync, const double (&dm)[NS], const double (&rm)[NS], double Dk,
                                double inv) {
  const int lane = threadIdx.x & 63;
  auto nd_at = [&](int s) { const uint2 v = meta[s * 64 + lane]; return Node{v.x, v.y}; };
  double acc = 0.0;
  for (int g = 0; g < G.ncoarse; ++g) {
    const Node n0 = nd_at(0);
    if (n_valid(n0) && n_g(n0) == g) {
      const double v = recompose_node(y, wt, n0, __dmul_rn(Dk, rint(__dmul_rn(dm[0], inv))), G.n_par);
      const double e = rm[0] - v;
      acc = fma(e, e, acc);
    }
    wave_sync();
  }
  // Slots of one group read only coarser groups, so the stores of a batch of slots can
  // wait until every load of the batch is issued; batches end at group boundaries.
  constexpr int BATCH = 4;
#pragma unroll
  for (int s0 = 1; s0 < NS; s0 += BATCH) {
    double v[BATCH];
    int ev[BATCH];
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int s = s0 + q;
      ev[q] = -1;
      v[q] = 0.0;
      const Node n = (s < NS && s < G.nslots) ? nd_at(s) : Node{0u, 0u};
      if (n_valid(n)) {
        const double dq = __dmul_rn(Dk, rint(__dmul_rn(dm[s], inv)));
        v[q] = __dadd_rn(dq, predict_n(y, wt, n, G.n_par));
        ev[q] = n_e(n);
      }
      // a group boundary inside the batch: store what is computed so far first
      if (s < NS && s < G.nslots && ssync[s]) {
#pragma unroll
        for (int r = 0; r <= q; ++r)
          if (ev[r] >= 0) { y[ev[r]] = v[r]; ev[r] = -2 - ev[r]; }
        wave_sync();
      }
    }
#pragma unroll
    for (int q = 0; q < BATCH; ++q) {
      const int s = s0 + q;
      if (s < NS && s < G.nslots) {
        if (ev[q] >= 0) y[ev[q]] = v[q];
        if (ev[q] != -1) {
          const double e = rm[s] - v[q];
          acc = fma(e, e, acc);
        }
      }
    }
  }
  return wsum(acc);
}

// Newton statistics at lam over the lane's natural-order elements (uniform vol factored
// out: v[0..3] = sum phi_k x, v[4] = sum |phi_1| x, v[5..14] = sum_{x>0} phi_k phi_l,
// v[15] = ||x - ft||^2; all scaled back by vol / vol^2 before return).
__device__ __forceinline__ void newton_stats(const GridDev& G, const double* ft, const double* s_a, const double* s_c,
                             const double (&lam)[4], double (&v)[16]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = 0.0;
  int i = lane % G.n_par, j = lane / G.n_par;
  const int di = 64 % G.n_par, dj = 64 / G.n_par;
#pragma unroll 2
  for (int e = lane; e < G.N; e += 64) {
    const double a = s_a[i], c = s_c[j];
    const double vol = G.uniform_vol ? G.vol0 : G.vol[e];
    const double fte = ft[e];
    const double x = fmax(0.0, fte - corr_cell(lam, vol, a, c));
    const double w = G.uniform_vol ? 1.0 : vol;
    const double wx = w * x;
    const double ax = a * wx;
    v[0] += wx;
    v[1] += ax;
    v[2] = fma(c, wx, v[2]);
    v[3] = fma(a, ax, v[3]);
    v[4] = fma(fabs(a), wx, v[4]);
    if (x > 0.0) {
      const double w2 = w * w;
      const double wa = w2 * a, wc = w2 * c, wa2 = wa * a;
      v[5] += w2;
      v[6] += wa;
      v[7] += wc;
      v[8] += wa2;
      v[9] += wa2;
      v[10] = fma(wa, c, v[10]);
      v[11] = fma(wa2, a, v[11]);
      v[12] = fma(wc, c, v[12]);
      v[13] = fma(wa2, c, v[13]);
      v[14] = fma(wa2, a * a, v[14]);
    }
    const double dx = x - fte;
    v[15] = fma(dx, dx, v[15]);
    i += di;
    j += dj;
    if (i >= G.n_par) { i -= G.n_par; ++j; }
  }
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = wsum(v[k]);
  if (G.uniform_vol) {
    const double s1 = G.vol0, s2 = G.vol0 * G.vol0;
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] *= s1;
#pragma unroll
    for (int k = 5; k < 15; ++k) v[k] *= s2;
  }
}

__device__ __forceinline__ double theta_w(const double (&v)[16], const double (&lam)[4], const double (&b)[4]) {
  double t = 0.5 * v[15];
#pragma unroll
  for (int k = 0; k < 4; ++k) t = t + lam[k] * (v[k] - b[k]);
  return t;
}

__device__ __forceinline__ bool chol4(const double (&v)[16], const double (&g)[4], double (&d)[4]) {
  double Hm[4][4];
  Hm[0][0] = v[5]; Hm[0][1] = v[6]; Hm[0][2] = v[7]; Hm[0][3] = v[8];
  Hm[1][1] = v[9]; Hm[1][2] = v[10]; Hm[1][3] = v[11];
  Hm[2][2] = v[12]; Hm[2][3] = v[13]; Hm[3][3] = v[14];
  Hm[1][0] = Hm[0][1]; Hm[2][0] = Hm[0][2]; Hm[3][0] = Hm[0][3];
  Hm[2][1] = Hm[1][2]; Hm[3][1] = Hm[1][3]; Hm[3][2] = Hm[2][3];
  const double tr = ((Hm[0][0] + Hm[1][1]) + Hm[2][2]) + Hm[3][3];
  double Lm[4][4] = {};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double piv = Hm[k][k];
#pragma unroll
    for (int q = 0; q < k; ++q) piv = piv - Lm[k][q] * Lm[k][q];
    if (!(piv > kPivTol * tr)) return false;
    Lm[k][k] = sqrt(piv);
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      double s = Hm[i][k];
#pragma unroll
      for (int q = 0; q < k; ++q) s = s - Lm[i][q] * Lm[k][q];
      Lm[i][k] = s / Lm[k][k];
    }
  }
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = g[i];
#pragma unroll
    for (int q = 0; q < i; ++q) s = s - Lm[i][q] * y[q];
    y[i] = s / Lm[i][i];
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int q = i + 1; q < 4; ++q) s = s - Lm[q][i] * d[q];
    d[i] = s / Lm[i][i];
  }
  return true;
}

// Both Newton rounds in one loop with a single pass site (the unrolled pass is large):
// round 1 takes fixed steps s1 for up to max1 updates; if it does not converge, round 2
// continues from its multipliers with fixed steps s2 or, with armijo2, Armijo
// backtracking on theta, for up to max2 updates.  An accepted Armijo candidate's pass is
// also the next iterate's pass (same multipliers, same values).  Returns 0 (round 1
// converged), 1 (round 2 converged) or 2 (failed); *upd counts the updates.
__device__ __forceinline__ int newton_w(const GridDev& G, const double* ft, const double* s_a, const double* s_c,
                        const double (&b)[4], double (&lam)[4], double s1, int max1, double s2, int max2,
                        bool armijo2, int* upd, bool have_init, const double (&lam_init)[4], bool* rejected) {
  int round = 0, it = 0, total = 0, halvings = 0;
  bool trial = false;
  // warm start: lam begins at lam_init; it is dropped (cold restart) if round 1 allows no
  // update, if the Cholesky step at it fails, or if that first step makes the scaled
  // residual max_k |g_k| / s_k grow
  bool warm = have_init && max1 >= 1;
  double r_warm0 = 0.0;
  *rejected = false;
  if (have_init) {
    bool fin = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) fin = fin && isfinite(lam_init[k]);
    if (!warm || !fin) { warm = false; *rejected = true; }
#pragma unroll
    for (int k = 0; k < 4; ++k) lam[k] = warm ? lam_init[k] : 0.0;
  }
  double cand[4] = {lam[0], lam[1], lam[2], lam[3]};
  double d[4] = {0.0, 0.0, 0.0, 0.0};
  double t0 = 0.0, gd = 0.0, step = 1.0;
  double v[16];
  for (;;) {
    newton_stats(G, ft, s_a, s_c, cand, v);
    const bool armijo = round == 1 && armijo2;
    if (trial) {
      if (theta_w(v, cand, b) >= t0 + kArmijoC * step * gd) {
#pragma unroll
        for (int k = 0; k < 4; ++k) lam[k] = cand[k];
        trial = false;
        ++it;
        ++total;
      } else {
        if (++halvings >= kArmijoHalvings) break;
        step *= 0.5;
#pragma unroll
        for (int k = 0; k < 4; ++k) cand[k] = lam[k] + step * d[k];
        continue;
      }
    }
    // v holds the pass at lam
    double g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = v[k] - b[k];
    const double sc[4] = {v[0], v[4], v[2], v[3]};
    bool conv = true;
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      conv = conv && (fabs(g[k]) <= kGTol * (sc[k] + 1e-300));
      rs = fmax(rs, fabs(g[k]) / (sc[k] + 1e-300));
    }
    if (warm && round == 0 && it == 1 && total == 1) {
      warm = false;
      if (rs > r_warm0) {          // the warm start's first step made things worse
        *rejected = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) { lam[k] = 0.0; cand[k] = 0.0; }
        it = 0;
        total = 0;
        continue;
      }
    }
    if (warm && round == 0 && it == 0) r_warm0 = rs;
    *upd = total;
    if (conv) return round;
    const int cap = round == 0 ? max1 : max2;
    bool fail_round = it == cap || !chol4(v, g, d);
    if (fail_round && warm && round == 0 && it == 0) {
      warm = false;                // no usable step at the warm start
      *rejected = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) { lam[k] = 0.0; cand[k] = 0.0; }
      continue;
    }
    if (fail_round) {
      if (round == 1) break;
      round = 1;                 // round 2 starts from round 1's multipliers
      it = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) cand[k] = lam[k];
      // the pass at lam is v already: redo the checks for round 2 without a new pass
      const int cap2 = max2;
      if (it == cap2 || !chol4(v, g, d)) break;
    }
    if (round == 1 && armijo2) {
      t0 = theta_w(v, lam, b);
      gd = ((g[0] * d[0] + g[1] * d[1]) + g[2] * d[2]) + g[3] * d[3];
      step = 1.0;
      halvings = 0;
      trial = true;
#pragma unroll
      for (int k = 0; k < 4; ++k) cand[k] = lam[k] + d[k];
    } else {
      const double sk = round == 0 ? s1 : s2;
#pragma unroll
      for (int k = 0; k < 4; ++k) lam[k] = lam[k] + sk * d[k];
#pragma unroll
      for (int k = 0; k < 4; ++k) cand[k] = lam[k];
      ++it;
      ++total;
    }
    (void)armijo;
  }
  *upd = total;
  return 2;
}

// Dynamic LDS of the wave kernels, in doubles: s_a [kMaxDim], s_c [kMaxDim], s_w [64],
// then (compression only) the node metadata, nslots * 64 entries of two words = one
// double each, then one N-double buffer per wave.  Kernels and launchers both take the
// offsets from here.
constexpr int kLdsTables = 2 * kMaxDim + 64;
__host__ __device__ __forceinline__ size_t lds_meta_doubles(int nslots) { return (size_t)nslots * 64; }

// Per-grid scalars that are indexed at run time go to LDS (indexing them inside the
// by-value kernel argument would force a private copy of the whole argument).
__device__ __forceinline__ void load_small_tables(const GridDev& G, int* gs, int* sg, int* ss) {
  const int t = threadIdx.x;
  if (t <= kMaxLev) gs[t] = t <= G.nlev ? G.gstart[t] : G.N;
  if (t < kWaveSlots) {
    sg[t] = G.slot_group[t];
    ss[t] = G.slot_sync[t];
  }
}

// ---- compression ------------------------------------------------------------------------

template <typename TIn, int NS>
__global__ __launch_bounds__(256, 2) void k_residual_w(GridDev G, ResidualArgs a) {
  extern __shared__ double smem[];
  __shared__ uint32_t s_gmax[kWPB][kMaxLev], s_width[kWPB][kMaxLev], s_base[kWPB][kMaxLev];
  __shared__ int s_gstart[kMaxLev + 1];
  __shared__ int s_sgroup[kWaveSlots], s_ssync[kWaveSlots];
  double* s_a = smem;                    // [128]
  double* s_c = smem + kMaxDim;          // [128]
  double* s_w = smem + 2 * kMaxDim;      // [64]
  uint2* meta = (uint2*)(smem + kLdsTables);                       // [nslots * 64]
  const int N = G.N;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* y = smem + kLdsTables + lds_meta_doubles(G.nslots) + (size_t)N * wv;
  uint32_t* words = (uint32_t*)y;        // payload words reuse the buffer once ft is read
  for (int k = threadIdx.x; k < G.n_par; k += 256) s_a[k] = G.apar[k];
  for (int k = threadIdx.x; k < G.n_perp; k += 256) s_c[k] = G.cperp[k];
  for (int k = threadIdx.x; k < G.nw; k += 256) s_w[k] = G.wtab[k];
  for (int k = threadIdx.x; k < G.nslots * 64; k += 256)
    meta[k] = make_uint2(G.slot_meta[2 * k], G.slot_meta[2 * k + 1]);
  load_small_tables(G, s_gstart, s_sgroup, s_ssync);
  __syncthreads();
  const long long h = (long long)blockIdx.x * kWPB + wv;
  if (h >= a.H) return;
  const TIn* f = (const TIn*)a.hist + h * a.hs;
  const float* fhp = a.fhat ? a.fhat + h * (long long)N : nullptr;

  // ---- natural-order pass: residual into LDS, moments, norms, range ----
  dd ff{0.0, 0.0};
  double rr = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, fmx = -INFINITY, fmnn = -INFINITY;
  bool bad = false;
  {
    // issue every load of the histogram before using any (one round trip of latency)
    TIn fr[NS];
    float hr[NS];
    {
      int i = lane % G.n_par, j = lane / G.n_par;
      const int di = 64 % G.n_par, dj = 64 / G.n_par;
#pragma unroll
      for (int m = 0; m < NS; ++m) {
        const int e = lane + 64 * m;
        fr[m] = (TIn)0;
        hr[m] = 0.0f;
        if (e < N) {
          fr[m] = f[(long long)j * a.rs + i];
          if (fhp) hr[m] = fhp[e];
        }
        i += di;
        j += dj;
        if (i >= G.n_par) { i -= G.n_par; ++j; }
      }
    }
    int i = lane % G.n_par, j = lane / G.n_par;
    const int di = 64 % G.n_par, dj = 64 / G.n_par;
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int e = lane + 64 * m;
      if (e < N) {
        const double fv = (double)fr[m];
        const double r = fv - (double)hr[m];
        y[e] = r;
        ff = dd_add_d(ff, fv * fv);
        rr = fma(r, r, rr);
        const double w = G.uniform_vol ? fv : G.vol[e] * fv;
        const double av = s_a[i];
        const double wa = w * av;
        m0 += w;
        m1 += wa;
        m2 = fma(s_c[j], w, m2);
        m3 = fma(av, wa, m3);
        bad |= !isfinite(fv);
        fmx = fmax(fmx, fv);
        fmnn = fmax(fmnn, -fv);
      }
      i += di;
      j += dj;
      if (i >= G.n_par) { i -= G.n_par; ++j; }
    }
  }
  ff = wdd(ff);
  rr = wsum(rr);
  double b[4] = {wsum(m0), wsum(m1), wsum(m2), wsum(m3)};
  if (G.uniform_vol) {
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] *= G.vol0;
  }
  fmx = wmax(fmx);
  fmnn = wmax(fmnn);
  bad = __ballot(bad) != 0;
  const double tau_h = (a.tau_mode == HCZ_TAU_NRMSE) ? (a.tau * G.sqrtN) * (fmx - (-fmnn))
                                                     : a.tau * sqrt(ff.hi + ff.lo);
  const double thr = kSelMargin * tau_h;
  const double thr2 = thr * thr;
  bool raw = bad || !(b[0] > 0.0);
  const bool coded = rr > thr2;
  if (coded && !(tau_h > 0.0)) raw = true;
  wave_sync();

  int kst = 0xff;
  uint32_t rec_bytes = 0;
  // ft = fhat + rhat (rhat = 0 when not coded), written over the buffer in natural order
  bool ft_ready = false;
  auto load_ft = [&](bool with_r) {
    float hr[NS];
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int e = lane + 64 * m;
      hr[m] = (fhp && e < N) ? fhp[e] : 0.0f;
    }
#pragma unroll
    for (int m = 0; m < NS; ++m) {
      const int e = lane + 64 * m;
      if (e < N) y[e] = (double)hr[m] + (with_r ? y[e] : 0.0);
    }
    wave_sync();
  };
  auto nd_at = [&](int s) { const uint2 v = meta[s * 64 + lane]; return Node{v.x, v.y}; };
  if (coded && !raw) {
    double dm[NS], rm[NS];
    double mx = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      dm[s] = 0.0;
      rm[s] = 0.0;
      const Node n = s < G.nslots ? nd_at(s) : Node{0u, 0u};
      if (n_valid(n)) {
        rm[s] = y[n_e(n)];
        dm[s] = n_g(n) == 0 ? rm[s] : __dsub_rn(rm[s], predict_n(y, s_w, n, G.n_par));
        mx = fmax(mx, fabs(dm[s]));
      }
    }
    mx = wmax(mx);
    wave_sync();
    const double d0 = (kLadderMargin * tau_h) / G.den;
    if (mx * (1.0 / d0) >= kQMax) raw = true;
    if (!raw) {
      int lo = 0, hi = kLadder;
      while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        const double Dk = ladder(d0, mid);
        const double e2 = recompose_all<NS>(G, y, s_w, meta, s_ssync, dm, rm, Dk, 1.0 / Dk);
        if (e2 <= thr2) lo = mid;
        else hi = mid;
      }
      kst = lo;
      const double Dk = ladder(d0, kst);
      const double inv = 1.0 / Dk;
      // zigzag integers, per-group widths (packing first: the payload words borrow the
      // buffer, which the final recomposition then fills with rhat)
      if (lane < kMaxLev) s_gmax[wv][lane] = 0u;
      wave_sync();
      auto zz = [&](double d) -> uint32_t {
        const int q = (int)rint(__dmul_rn(d, inv));
        return ((uint32_t)q << 1) ^ (uint32_t)(q >> 31);
      };
      // slot 0 may mix groups: reduce each of its groups separately
      const Node nd0 = nd_at(0);
      const uint32_t u0 = n_valid(nd0) ? zz(dm[0]) : 0u;
      for (int g = 0; g < G.ncoarse; ++g) {
        const uint32_t v = wumax((n_valid(nd0) && n_g(nd0) == g) ? u0 : 0u);
        if (lane == 0) s_gmax[wv][g] = max(s_gmax[wv][g], v);
      }
      uint32_t cur = 0u;
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        if (s < G.nslots) {
          if (n_valid(nd_at(s))) cur = max(cur, zz(dm[s]));
          if (s_ssync[s]) {
            const uint32_t v = wumax(cur);
            if (lane == 0) {
              const int g = s_sgroup[s];
              s_gmax[wv][g] = max(s_gmax[wv][g], v);
            }
            cur = 0u;
          }
        }
      }
      wave_sync();
      uint32_t nbits = 0;
      for (int g = 0; g < G.nlev; ++g) {
        const uint32_t mxu = s_gmax[wv][g];
        const uint32_t wdt = mxu ? 32u - (uint32_t)__clz(mxu) : 0u;
        if (lane == 0) { s_width[wv][g] = wdt; s_base[wv][g] = nbits; }
        nbits += (uint32_t)(s_gstart[g + 1] - s_gstart[g]) * wdt;
      }
      const uint32_t nwords = (nbits + 31u) >> 5;
      for (uint32_t k = lane; k < nwords; k += 64) words[k] = 0u;
      wave_sync();
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const Node n = s < G.nslots ? nd_at(s) : Node{0u, 0u};
        if (n_valid(n)) {
          const int g = n_g(n);
          const uint32_t wdt = s_width[wv][g];
          if (wdt != 0) {
            const int p = G.slot_pos[(size_t)s * 64 + lane];
            const uint32_t pos = s_base[wv][g] + (uint32_t)(p - s_gstart[g]) * wdt;
            const uint64_t v = (uint64_t)zz(dm[s]) << (pos & 31u);
            atomicOr(&words[pos >> 5], (uint32_t)v);
            if ((pos & 31u) + wdt > 32u) atomicOr(&words[(pos >> 5) + 1], (uint32_t)(v >> 32));
          }
        }
      }
      wave_sync();
      uint8_t* slot = a.slots + h * a.slot_stride;
      if (lane == 0) {
        uint64_t* hp = (uint64_t*)slot;
        hp[0] = (uint64_t)__double_as_longlong(Dk);
        uint64_t w1 = (uint64_t)(uint32_t)kst | ((uint64_t)(uint32_t)G.nlev << 8);
        uint64_t w2 = 0;
        for (int g = 0; g < G.nlev; ++g) {
          const int byte = 10 + g;
          if (byte < 16) w1 |= (uint64_t)s_width[wv][g] << (8 * (byte - 8));
          else w2 |= (uint64_t)s_width[wv][g] << (8 * (byte - 16));
        }
        hp[1] = w1;
        if (G.hdr_bytes > 16) hp[2] = w2;
      }
      uint32_t* pw = (uint32_t*)(slot + G.hdr_bytes);
      for (uint32_t k = lane; k < nwords; k += 64) pw[k] = words[k];
      rec_bytes = (uint32_t)G.hdr_bytes + 4u * nwords;
      wave_sync();
      recompose_all<NS>(G, y, s_w, meta, s_ssync, dm, rm, Dk, inv);   // rhat at k* now in y
      wave_sync();
      load_ft(true);                                          // ft = fhat + rhat
      ft_ready = true;
    }
  }

  // ---- Newton projection in natural order ----
  double lam[4] = {0.0, 0.0, 0.0, 0.0};
  int flags = 0, total_upd = 0;
  if (!raw) {
    if (!ft_ready) load_ft(false);
    const bool paper = a.fallback == HCZ_FALLBACK_PAPER;
    double l0[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.lam0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) l0[k] = a.lam0[h * 4 + k];
    }
    bool rejected = false;
    const int st = newton_w(G, y, s_a, s_c, b, lam, a.newton_s, a.max_iter, paper ? 0.01 : 1.0,
                            a.max_iter2, !paper, &total_upd, a.lam0 != nullptr, l0, &rejected);
    if (rejected) flags |= HCZ_FLAG_WARM_REJECTED;
    if (st >= 1) flags |= HCZ_FLAG_ROUND2;
    if (st == 2) raw = true;
  }

  uint64_t size = 0;
  if (raw) {
    flags = (flags & (HCZ_FLAG_ROUND2 | HCZ_FLAG_WARM_REJECTED)) | HCZ_FLAG_RAW;
    TIn* dst = (TIn*)(a.slots + h * a.slot_stride);
    int i = lane % G.n_par, j = lane / G.n_par;
    const int di = 64 % G.n_par, dj = 64 / G.n_par;
    for (int e = lane; e < N; e += 64) {
      dst[e] = f[(long long)j * a.rs + i];
      i += di;
      j += dj;
      if (i >= G.n_par) { i -= G.n_par; ++j; }
    }
    size = (uint64_t)N * sizeof(TIn);
    kst = 0xff;
  } else if (coded) {
    flags |= HCZ_FLAG_CODED;
    size = rec_bytes;
  }
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) a.lambda[h * 4 + k] = raw ? 0.0 : lam[k];
    a.flags[h] = (uint8_t)flags;
    a.sizes[h] = size;
    a.kstar[h] = (uint8_t)kst;
    a.iters[h] = (uint16_t)min(total_upd, 65535);
  }
}

// ---- decompression ----------------------------------------------------------------------

__device__ __forceinline__ uint32_t ld32w(const uint8_t* p) { return *(const uint32_t*)p; }

template <typename TIn, typename TOut, int NS>
__global__ __launch_bounds__(256, 2) void k_decompress_w(GridDev G, DecompressArgs a) {
  extern __shared__ double smem[];
  __shared__ uint32_t s_width[kWPB][kMaxLev], s_base[kWPB][kMaxLev];
  __shared__ int s_gstart[kMaxLev + 1];
  __shared__ int s_sgroup[kWaveSlots], s_ssync[kWaveSlots];
  double* s_a = smem;
  double* s_c = smem + kMaxDim;
  double* s_w = smem + 2 * kMaxDim;
  const int N = G.N;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* y = smem + kLdsTables + (size_t)N * wv;
  for (int k = threadIdx.x; k < G.n_par; k += 256) s_a[k] = G.apar[k];
  for (int k = threadIdx.x; k < G.n_perp; k += 256) s_c[k] = G.cperp[k];
  for (int k = threadIdx.x; k < G.nw; k += 256) s_w[k] = G.wtab[k];
  load_small_tables(G, s_gstart, s_sgroup, s_ssync);
  __syncthreads();
  const long long h = (long long)blockIdx.x * kWPB + wv;
  if (h >= a.H) return;
  const int fl = a.flags[h];
  const uint8_t* rec = a.stream + a.offsets[h];
  TOut* out = (TOut*)a.out + h * (long long)N;
  if ((fl & (HCZ_FLAG_RAW | HCZ_FLAG_CODED)) &&
      (a.offsets[h + 1] > a.capacity || a.offsets[h + 1] < a.offsets[h] ||
       a.offsets[h + 1] - a.offsets[h] < (uint64_t)G.hdr_bytes)) {
    for (int e = lane; e < N; e += 64) out[e] = (TOut)NAN;
    return;
  }
  if (fl & HCZ_FLAG_RAW) {
    if (sizeof(TIn) == 8) {
      const uint32_t* s32 = (const uint32_t*)rec;
      for (int e = lane; e < N; e += 64) {
        const uint64_t lo = s32[2 * e], hi = s32[2 * e + 1];
        out[e] = (TOut)__longlong_as_double((long long)(lo | (hi << 32)));
      }
    } else {
      const float* src = (const float*)rec;
      for (int e = lane; e < N; e += 64) out[e] = (TOut)src[e];
    }
    return;
  }
  const float* fhp = a.fhat ? a.fhat + h * (long long)N : nullptr;
  const bool coded = (fl & HCZ_FLAG_CODED) != 0;
  if (coded) {
    const uint64_t lo = ld32w(rec), hi = ld32w(rec + 4);
    const double Delta = __longlong_as_double((long long)(lo | (hi << 32)));
    if (lane == 0) {
      uint32_t nb = 0;
      for (int g = 0; g < G.nlev; ++g) {
        const uint32_t wdt = rec[10 + g];
        s_width[wv][g] = wdt;
        s_base[wv][g] = nb;
        nb += (uint32_t)(s_gstart[g + 1] - s_gstart[g]) * wdt;
      }
    }
    wave_sync();
    const uint8_t* payload = rec + G.hdr_bytes;
    Node nd[NS];
    double dq[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      nd[s] = Node{0u, 0u};
      dq[s] = 0.0;
      if (s < G.nslots) {
        const uint32_t* mp = G.slot_meta + ((size_t)s * 64 + lane) * 2;
        nd[s] = Node{mp[0], mp[1]};
        if (n_valid(nd[s])) {
          const int g = n_g(nd[s]);
          const uint32_t wdt = s_width[wv][g];
          uint32_t u = 0;
          if (wdt) {
            const int p = G.slot_pos[(size_t)s * 64 + lane];
            const uint32_t pos = s_base[wv][g] + (uint32_t)(p - s_gstart[g]) * wdt;
            const uint32_t wi = pos >> 5, sh = pos & 31u;
            uint64_t v = ld32w(payload + 4 * wi);
            if (sh + wdt > 32u) v |= (uint64_t)ld32w(payload + 4 * (wi + 1)) << 32;
            u = (uint32_t)((v >> sh) & ((wdt == 32u) ? 0xffffffffull : ((1ull << wdt) - 1ull)));
          }
          const int q = (int)((u >> 1) ^ (0u - (u & 1u)));
          dq[s] = __dmul_rn(Delta, (double)q);
        }
      }
    }
    // recomposition in the compressor's order
    for (int g = 0; g < G.ncoarse; ++g) {
      if (n_valid(nd[0]) && n_g(nd[0]) == g) recompose_node(y, s_w, nd[0], dq[0], G.n_par);
      wave_sync();
    }
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      if (s < G.nslots) {
        if (n_valid(nd[s])) recompose_node(y, s_w, nd[s], dq[s], G.n_par);
        if (s_ssync[s]) wave_sync();
      }
    }
  }
  double lam[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) lam[k] = a.lambda[h * 4 + k];
  float hr[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int e = lane + 64 * m;
    hr[m] = (fhp && e < N) ? fhp[e] : 0.0f;
  }
  int i = lane % G.n_par, j = lane / G.n_par;
  const int di = 64 % G.n_par, dj = 64 / G.n_par;
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const int e = lane + 64 * m;
    if (e < N) {
      const double ft = (double)hr[m] + (coded ? y[e] : 0.0);
      const double vol = G.uniform_vol ? G.vol0 : G.vol[e];
      out[e] = (TOut)fmax(0.0, ft - corr_cell(lam, vol, s_a[i], s_c[j]));
    }
    i += di;
    j += dj;
    if (i >= G.n_par) { i -= G.n_par; ++j; }
  }
}

// ---- launchers ----------------------------------------------------------------------------

static size_t lds_bytes(const GridDev& G, bool with_meta) {
  const size_t meta = with_meta ? lds_meta_doubles(G.nslots) : 0;
  return (kLdsTables + meta + (size_t)G.N * kWPB) * sizeof(double);
}

bool wave_path(const GridDev& G) { return G.nslots > 0 && G.nslots <= kWaveSlots; }

hipError_t launch_residual_w(const GridDev& G, const ResidualArgs& a, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.H + kWPB - 1) / kWPB)), block(64 * kWPB);
  const size_t lds = lds_bytes(G, true);
  if (a.dtype == HCZ_F32)
    hipLaunchKernelGGL((k_residual_w<float, kWaveSlots>), grid, block, lds, st, G, a);
  else
    hipLaunchKernelGGL((k_residual_w<double, kWaveSlots>), grid, block, lds, st, G, a);
  return hipGetLastError();
}

hipError_t launch_decompress_w(const GridDev& G, const DecompressArgs& a, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.H + kWPB - 1) / kWPB)), block(64 * kWPB);
  const size_t lds = lds_bytes(G, false);
#define HCZ_DW(TI, TO) hipLaunchKernelGGL((k_decompress_w<TI, TO, kWaveSlots>), grid, block, lds, st, G, a)
  if (a.in_dtype == HCZ_F32) {
    if (a.out_dtype == HCZ_F64) HCZ_DW(float, double); else HCZ_DW(float, float);
  } else {
    if (a.out_dtype == HCZ_F64) HCZ_DW(double, double); else HCZ_DW(double, float);
  }
#undef HCZ_DW
  return hipGetLastError();
}

}  // namespace hcz
