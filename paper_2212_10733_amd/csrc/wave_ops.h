// Wave-level building blocks shared by the residual kernels that keep a histogram in LDS
// and reduce across lanes with DPP: butterflies, the 4x4 Cholesky solve, the dual
// objective and the two-round Newton driver of the Stage-5 projection (Section III Stage
// 5, Eq. 6).  Included by the wave-per-histogram and the wave-team kernels.
#pragma once
#include "hcz_internal.h"

namespace hcz {

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

// Sixteen wave sums at once, by a transposed butterfly: each step pairs every value a lane
// carries with a partner lane and keeps half of the values, so the lanes end with one
// total each instead of sixteen.  Steps: lanes l, l ^ 32 (permlane32 swap; values k and
// k + 8), l, l ^ 16 (permlane16 swap; k and k + 4), l, l ^ 15 (row_mirror; k and k + 2,
// by bit 3), l, l ^ 7 (row_half_mirror; k and k + 1, by bit 2), then l ^ 1 and l ^ 2.  Lane
// 4 i .. 4 i + 3 ends with the total of v[i]; every lane reads all sixteen from those lanes,
// so all hold the same bits.
__device__ __forceinline__ double swap_add32(double p, double q) {
  const auto rl = __builtin_amdgcn_permlane32_swap((unsigned)__double2loint(p), (unsigned)__double2loint(q), false,
                                                   false);
  const auto rh = __builtin_amdgcn_permlane32_swap((unsigned)__double2hiint(p), (unsigned)__double2hiint(q), false,
                                                   false);
  return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
}
__device__ __forceinline__ double swap_add16(double p, double q) {
  const auto rl = __builtin_amdgcn_permlane16_swap((unsigned)__double2loint(p), (unsigned)__double2loint(q), false,
                                                   false);
  const auto rh = __builtin_amdgcn_permlane16_swap((unsigned)__double2hiint(p), (unsigned)__double2hiint(q), false,
                                                   false);
  return __hiloint2double((int)rh[0], (int)rl[0]) + __hiloint2double((int)rh[1], (int)rl[1]);
}
__device__ __forceinline__ void wsum16(const double (&v)[16], double (&out)[16]) {
  const int lane = threadIdx.x & 63;
  double u[8], w[4], z[2];
#pragma unroll
  for (int k = 0; k < 8; ++k) u[k] = swap_add32(v[k], v[k + 8]);       // lane half: k + 8 b5
#pragma unroll
  for (int k = 0; k < 4; ++k) w[k] = swap_add16(u[k], u[k + 4]);       // row parity: + 4 b4
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double keep = b3 ? w[k + 2] : w[k], send = b3 ? w[k] : w[k + 2];
    z[k] = keep + dpp_d<0x140, 0xF>(send);                                 // + 2 b3
  }
  double t;
  {
    const double keep = b2 ? z[1] : z[0], send = b2 ? z[0] : z[1];
    t = keep + dpp_d<0x141, 0xF>(send);                                    // + b2
  }
  t = t + dpp_d<0xB1, 0xF>(t);
  t = t + dpp_d<0x4E, 0xF>(t);
#pragma unroll
  for (int i = 0; i < 16; ++i) out[i] = lane_d(t, 4 * i);
}

__device__ __forceinline__ double theta_w(const double (&v)[16], const double (&lam)[4], const double (&b)[4]) {
  double t = 0.5 * v[15];
#pragma unroll
  for (int k = 0; k < 4; ++k) t = t + lam[k] * (v[k] - b[k]);
  return t;
}
// The KL reading's dual D(lam) = -sum_j x_j - lam^T b (v[15] = sum_j x_j), concave with the
// same gradient A x - b.
__device__ __forceinline__ double theta_kl(const double (&v)[16], const double (&lam)[4], const double (&b)[4]) {
  double t = -v[15];
#pragma unroll
  for (int k = 0; k < 4; ++k) t = t - lam[k] * b[k];
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
  double rl[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double piv = Hm[k][k];
#pragma unroll
    for (int q = 0; q < k; ++q) piv = piv - Lm[k][q] * Lm[k][q];
    if (!(piv > kPivTol * tr)) return false;
    rl[k] = rsqrt(piv);                 // 1 / L_kk: the only form the solves use
#pragma unroll
    for (int i = k + 1; i < 4; ++i) {
      double s = Hm[i][k];
#pragma unroll
      for (int q = 0; q < k; ++q) s = s - Lm[i][q] * Lm[k][q];
      Lm[i][k] = s * rl[k];
    }
  }
  double y[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double s = g[i];
#pragma unroll
    for (int q = 0; q < i; ++q) s = s - Lm[i][q] * y[q];
    y[i] = s * rl[i];
  }
#pragma unroll
  for (int i = 3; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int q = i + 1; q < 4; ++q) s = s - Lm[q][i] * d[q];
    d[i] = s * rl[i];
  }
  return true;
}

// Both Newton rounds in one loop with a single pass site: round 1 takes fixed steps s1
// for up to max1 updates; if it does not converge, round 2 continues from its
// multipliers with fixed steps s2 or, with armijo2, Armijo backtracking on theta, for up
// to max2 updates.  An accepted Armijo candidate's pass is also the next iterate's pass
// (same multipliers, same values).  Returns 0 (round 1 converged), 1 (round 2
// converged) or 2 (failed); *upd counts the updates.
// pass(theta, lam, v, sc) evaluates the iterate lam: v[0..3] = A x, v[15] = ||x - ft||^2
// when theta, sc the stopping rule's scales; hess(v) fills the Hessian entries v[5..14]
// of the last pass.
template <class PASS, class HESS, bool KL = false>
__device__ __forceinline__ int newton_core(PASS pass, HESS hess, const double (&b)[4], double (&lam)[4], double s1,
                                           int max1, double s2, int max2, bool armijo2, int* upd, bool have_init,
                                           const double (&lam_init)[4], bool* rejected) {
  auto theta = [&](const double (&v)[16], const double (&l)[4]) { return KL ? theta_kl(v, l, b) : theta_w(v, l, b); };
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
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = 0.0;
  double sc[4];
  auto hessian = [&]() { hess(v); };
  for (;;) {
    pass(round == 1 && armijo2, cand, v, sc);
    if (trial) {
      if (theta(v, cand) >= t0 + kArmijoC * step * gd) {
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
    bool conv = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) conv = conv && (fabs(g[k]) <= kGTol * (sc[k] + 1e-300));
    // the scaled residual max_k |g_k| / s_k, formed only while a warm start is judged
    auto scaled_res = [&]() {
      double rs = 0.0;
#pragma unroll
      for (int k = 0; k < 4; ++k) rs = fmax(rs, fabs(g[k]) / (sc[k] + 1e-300));
      return rs;
    };
    if (warm && round == 0 && it == 1 && total == 1) {
      warm = false;
      if (scaled_res() > r_warm0) {          // the warm start's first step made things worse
        *rejected = true;
#pragma unroll
        for (int k = 0; k < 4; ++k) { lam[k] = 0.0; cand[k] = 0.0; }
        it = 0;
        total = 0;
        continue;
      }
    }
    if (warm && round == 0 && it == 0) r_warm0 = scaled_res();
    *upd = total;
    if (conv) return round;
    const int cap = round == 0 ? max1 : max2;
    bool fail_round = it == cap;
    if (!fail_round) {
      hessian();
      fail_round = !chol4(v, g, d);
    }
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
      if (armijo2) continue;     // round 2 needs theta at lam: one pass with it
      if (it == max2) break;
      hessian();
      if (!chol4(v, g, d)) break;
    }
    if (round == 1 && armijo2) {
      t0 = theta(v, lam);
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
  }
  *upd = total;
  return 2;
}

}  // namespace hcz
