// Per-histogram FP64 kernels: moments/QoIs (Eq. 1-4), residual selection and the
// multilevel coder with its bound search (Section III Stage 4), the Newton projection
// restoring the four moments (Stage 5, Eq. 6), and decompression (Section III, end).
//
// One workgroup of NT threads owns one histogram.  A first pass streams the histogram
// in natural order (coalesced) into LDS as FP64 residuals; afterwards thread t owns the
// nodes p = t + NT m of the coefficient order (coarsest group first), keeping their
// residual, coefficient, interpolation cell and reconstruction in registers.  LDS then
// holds one FP64 array that the recomposition rewrites group by group, with one barrier
// per group.  Every reduction is a fixed xor-butterfly plus an ordered sum over waves,
// so results are bitwise repeatable.
#include "hcz_internal.h"

namespace hcz {

template <typename T>
__device__ __forceinline__ double to_d(T v) { return (double)v; }

// Index of the coefficient group holding packing position p.
__device__ __forceinline__ int group_of(const GridDev& G, int p) {
  int g = 0;
#pragma unroll
  for (int q = 1; q < kMaxLev; ++q)
    if (q < G.nlev && p >= G.gstart[q]) g = q;
  return g;
}

// Recompose the reconstruction of all owned nodes for step size Dk (1/Dk = inv) into buf
// (natural order) and return the block-wide sum of (r - y)^2.
template <int NT, int NPT>
__device__ double recompose_err(const GridDev& G, double* buf, double* red, const int (&gm)[NPT],
                                const int (&em)[NPT], const Interp (&cm)[NPT],
                                const double (&dm)[NPT], const double (&rm)[NPT], double Dk,
                                double inv) {
  for (int g = 0; g < G.nlev; ++g) {
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      if (gm[m] == g) {
        const double dq = qdelta(Dk, dm[m], inv);
        buf[em[m]] = (g == 0) ? dq : __dadd_rn(dq, predict(buf, cm[m]));
      }
    }
    __syncthreads();
  }
  double s[1] = {0.0};
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    if (em[m] >= 0) {
      const double e = rm[m] - buf[em[m]];
      s[0] = fma(e, e, s[0]);
    }
  }
  block_sum<NT, 1>(s, red);
  return s[0];
}

// Newton statistics of one pass at multipliers lam: v[0..3] = A x, v[4] = sum |A_1| x,
// v[5..14] = A diag(x > 0) A^T (upper triangle, row-major), v[15] = ||x - ft||^2.
// With pos = false (the projection onto {A x = b} alone) x may be negative: v[16..18]
// then hold sum A_k |x| for k = 0, 2, 3 and v[4] sum |A_1| |x|, the stopping rule's scales.
constexpr int kNv = 19;
// ft: the reconstruction f^ + r^ in LDS, natural order; thread t takes cells t, t + NT, ...
// kl: the KL reading, x = max(ft, 0) exp(-A^T lam), Hessian weights x, v[15] = sum_j x_j.
template <int NT>
__device__ void newton_pass(const GridDev& G, const double* ft, const double (&lam)[4], double (&v)[kNv],
                            double* red, bool pos, bool kl = false) {
#pragma unroll
  for (int k = 0; k < kNv; ++k) v[k] = 0.0;
  int i = (int)threadIdx.x % G.n_par, j = (int)threadIdx.x / G.n_par;
  const int di = NT % G.n_par, dj = NT / G.n_par;
  for (int e = threadIdx.x; e < G.N; e += NT) {
    const Aphi A = make_aphi(G, e, i, j);
    const double fte = ft[e];
    i += di;
    j += dj;
    if (i >= G.n_par) { i -= G.n_par; ++j; }
    double x;
    if (kl) {
      x = fte > 0.0 ? fte * exp(-correction(A, lam)) : 0.0;
    } else {
      const double y = fte - correction(A, lam);
      x = pos ? fmax(0.0, y) : y;
    }
    const double xa = fabs(x);
    v[0] = fma(A.a0, x, v[0]);
    v[1] = fma(A.a1, x, v[1]);
    v[2] = fma(A.a2, x, v[2]);
    v[3] = fma(A.a3, x, v[3]);
    v[4] = fma(fabs(A.a1), xa, v[4]);
    v[16] = fma(A.a0, xa, v[16]);
    v[17] = fma(A.a2, xa, v[17]);
    v[18] = fma(A.a3, xa, v[18]);
    if (kl) {
      const double p0 = x * A.a0, p1 = x * A.a1, p2 = x * A.a2, p3 = x * A.a3;
      v[5] = fma(p0, A.a0, v[5]);
      v[6] = fma(p0, A.a1, v[6]);
      v[7] = fma(p0, A.a2, v[7]);
      v[8] = fma(p0, A.a3, v[8]);
      v[9] = fma(p1, A.a1, v[9]);
      v[10] = fma(p1, A.a2, v[10]);
      v[11] = fma(p1, A.a3, v[11]);
      v[12] = fma(p2, A.a2, v[12]);
      v[13] = fma(p2, A.a3, v[13]);
      v[14] = fma(p3, A.a3, v[14]);
    } else if (!pos || x > 0.0) {
      v[5] = fma(A.a0, A.a0, v[5]);
      v[6] = fma(A.a0, A.a1, v[6]);
      v[7] = fma(A.a0, A.a2, v[7]);
      v[8] = fma(A.a0, A.a3, v[8]);
      v[9] = fma(A.a1, A.a1, v[9]);
      v[10] = fma(A.a1, A.a2, v[10]);
      v[11] = fma(A.a1, A.a3, v[11]);
      v[12] = fma(A.a2, A.a2, v[12]);
      v[13] = fma(A.a2, A.a3, v[13]);
      v[14] = fma(A.a3, A.a3, v[14]);
    }
    if (kl) {
      v[15] += x;
    } else {
      const double dx = x - fte;
      v[15] = fma(dx, dx, v[15]);
    }
  }
  block_sum<NT, kNv>(v, red);
}

// Scales sum_j |A_kj| x_j of the stopping rule from a pass.
__device__ __forceinline__ void pass_scales(const double (&v)[kNv], bool pos, double (&sc)[4]) {
  sc[0] = pos ? v[0] : v[16];
  sc[1] = v[4];
  sc[2] = pos ? v[2] : v[17];
  sc[3] = pos ? v[3] : v[18];
}

// theta(lam) = 1/2 ||x - ft||^2 + lam^T (A x - b) from a pass's statistics; in the KL
// reading the dual D(lam) = -sum_j x_j - lam^T b.  Both are concave with gradient A x - b.
__device__ __forceinline__ double theta_of(const double (&v)[kNv], const double (&lam)[4],
                                           const double (&b)[4], bool kl = false) {
  if (kl) {
    double t = -v[15];
#pragma unroll
    for (int k = 0; k < 4; ++k) t = t - lam[k] * b[k];
    return t;
  }
  double t = 0.5 * v[15];
#pragma unroll
  for (int k = 0; k < 4; ++k) t = t + lam[k] * (v[k] - b[k]);
  return t;
}

// Solve H d = g by Cholesky; false if a pivot is not > kPivTol * trace(H).
__device__ __forceinline__ bool chol_solve4(const double (&v)[kNv], const double (&g)[4],
                                            double (&d)[4]) {
  double Hm[4][4];
  Hm[0][0] = v[5]; Hm[0][1] = v[6]; Hm[0][2] = v[7]; Hm[0][3] = v[8];
  Hm[1][1] = v[9]; Hm[1][2] = v[10]; Hm[1][3] = v[11];
  Hm[2][2] = v[12]; Hm[2][3] = v[13]; Hm[3][3] = v[14];
  Hm[1][0] = Hm[0][1]; Hm[2][0] = Hm[0][2]; Hm[3][0] = Hm[0][3];
  Hm[2][1] = Hm[1][2]; Hm[3][1] = Hm[1][3]; Hm[3][2] = Hm[2][3];
  const double tr = ((Hm[0][0] + Hm[1][1]) + Hm[2][2]) + Hm[3][3];
  double Lm[4][4] = {};
  double rl[4];                         // 1 / L_kk: the only form the solves use
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    double piv = Hm[k][k];
#pragma unroll
    for (int q = 0; q < k; ++q) piv = piv - Lm[k][q] * Lm[k][q];
    if (!(piv > kPivTol * tr)) return false;
    rl[k] = rsqrt(piv);
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

// One Newton round (Eq. 6).  armijo = false: lam += s d; true: backtracking on theta.
// Returns true when the stopping rule holds; *upd counts the updates made.
template <int NT>
__device__ bool newton_round(const GridDev& G, const double* ft, const double (&b)[4], double (&lam)[4],
                             double s, int max_iter, bool armijo, double* red, int* upd, bool pos,
                             bool kl = false) {
  double v[kNv];
  for (int it = 0; it <= max_iter; ++it) {
    newton_pass<NT>(G, ft, lam, v, red, pos, kl);
    double g[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) g[k] = v[k] - b[k];
    double sc[4];
    pass_scales(v, pos, sc);
    bool conv = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) conv = conv && (fabs(g[k]) <= kGTol * (sc[k] + 1e-300));
    *upd = it;
    if (conv) return true;
    if (it == max_iter) return false;
    double d[4];
    if (!chol_solve4(v, g, d)) return false;
    if (!armijo) {
#pragma unroll
      for (int k = 0; k < 4; ++k) lam[k] = lam[k] + s * d[k];
    } else {
      const double t0 = theta_of(v, lam, b, kl);
      const double gd = ((g[0] * d[0] + g[1] * d[1]) + g[2] * d[2]) + g[3] * d[3];
      double step = 1.0;
      bool ok = false;
      double cand[4];
      for (int q = 0; q < kArmijoHalvings; ++q) {
#pragma unroll
        for (int k = 0; k < 4; ++k) cand[k] = lam[k] + step * d[k];
        double w[kNv];
        newton_pass<NT>(G, ft, cand, w, red, pos, kl);
        if (theta_of(w, cand, b, kl) >= t0 + kArmijoC * step * gd) { ok = true; break; }
        step *= 0.5;
      }
      if (!ok) return false;
#pragma unroll
      for (int k = 0; k < 4; ++k) lam[k] = cand[k];
    }
  }
  return false;
}

template <int NT>
__device__ __forceinline__ uint32_t block_umax(uint32_t v, double* red) {
  constexpr int NW = NT / 64;
  uint32_t* r = (uint32_t*)red;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  v = wave_umax(v);
  if (l == 0) r[w] = v;
  __syncthreads();
  uint32_t s = r[0];
#pragma unroll
  for (int q = 1; q < NW; ++q) s = max(s, r[q]);
  __syncthreads();
  return s;
}

template <int NT, int NPT, typename TIn>
__global__ __launch_bounds__(NT) void k_residual(GridDev G, ResidualArgs a) {
  extern __shared__ double smem[];
  const int N = G.N;
  double* buf = smem;                                  // [N] residual, then reconstruction
  float* fh = (float*)(smem + N);                      // [N] reconstruction, then payload words
  uint32_t* words = (uint32_t*)fh;
  double* red = smem + N + (N + 1) / 2;                // [NT/64 * kNv]
  __shared__ uint32_t s_width[kMaxLev], s_base[kMaxLev];
  const int t = threadIdx.x;
  const long long h = blockIdx.x;
  const TIn* f = (const TIn*)a.hist + h * a.hs;
  const float* fhp = a.fhat ? a.fhat + h * (long long)N : nullptr;

  // ---- pass over the histogram in natural order ----------------------------------
  dd ff{0.0, 0.0};
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};    // ||r||^2, b0..b3, non-finite count
  double fmx = -INFINITY, fmnn = -INFINITY;           // max f, max(-f)
  {
    int i = t % G.n_par, j = t / G.n_par;
    const int di = NT % G.n_par, dj = NT / G.n_par;
    for (int e = t; e < N; e += NT) {
      const double fv = to_d(f[(long long)j * a.rs + i]);
      const float fhv = fhp ? fhp[e] : 0.0f;
      const double r = fv - (double)fhv;
      buf[e] = r;
      fh[e] = fhv;
      ff = dd_add_d(ff, fv * fv);
      acc[0] = fma(r, r, acc[0]);
      const Aphi A = make_aphi(G, e, i, j);
      acc[1] = fma(A.a0, fv, acc[1]);
      acc[2] = fma(A.a1, fv, acc[2]);
      acc[3] = fma(A.a2, fv, acc[3]);
      acc[4] = fma(A.a3, fv, acc[4]);
      acc[5] += isfinite(fv) ? 0.0 : 1.0;
      fmx = fmax(fmx, fv);
      fmnn = fmax(fmnn, -fv);
      i += di;
      j += dj;
      if (i >= G.n_par) { i -= G.n_par; ++j; }
    }
  }
  block_sum<NT, 6>(acc, red);
  ff = block_dd<NT>(ff, red);
  fmx = block_max<NT>(fmx, red);
  fmnn = block_max<NT>(fmnn, red);
  const double b[4] = {acc[1], acc[2], acc[3], acc[4]};
  const double tau = a.tau_hist ? a.tau_hist[h] : a.tau;
  const double tau_h = (a.tau_mode == HCZ_TAU_NRMSE) ? (tau * G.sqrtN) * (fmx - (-fmnn))
                                                     : tau * sqrt(ff.hi + ff.lo);
  const double thr = kSelMargin * tau_h;
  const double thr2 = thr * thr;
  bool raw = (acc[5] > 0.0) || !(b[0] > 0.0) || !(tau >= 0.0 && tau <= DBL_MAX);
  const bool coded = acc[0] > thr2;
  if (coded && !(tau_h > 0.0)) raw = true;

  // ---- owned nodes ---------------------------------------------------------------
  int em[NPT], gm[NPT];
  Interp cm[NPT];
  double rm[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int p = t + NT * m;
    em[m] = -1;
    gm[m] = 99;
    rm[m] = 0.0;
    if (p < N) {
      const uint32_t ij = G.node_ij[p];
      const int i = ij & 0xffff, j = ij >> 16;
      em[m] = j * G.n_par + i;
      gm[m] = group_of(G, p);
      cm[m] = make_interp(G, i, j);
      rm[m] = buf[em[m]];
    }
  }

  int kst = 0xff;
  uint32_t rec_bytes = 0;
  bool have_y = false;          // buf holds the recomposition at ladder index kst
  double dm[NPT];
  if (coded && !raw) {
    double mx = 0.0;
#pragma unroll
    for (int m = 0; m < NPT; ++m) {
      dm[m] = 0.0;
      if (em[m] >= 0) {
        dm[m] = (gm[m] == 0) ? rm[m] : __dsub_rn(rm[m], predict(buf, cm[m]));
        mx = fmax(mx, fabs(dm[m]));
      }
    }
    mx = block_max<NT>(mx, red);      // its barriers also end every read of the residuals
    const double d0 = (kLadderMargin * tau_h) / G.den;
    if (mx * (1.0 / d0) >= kQMax) raw = true;
    if (!raw) {
      // the bound search over the ladder, or the user's step (an empty search)
      LadderSearch S;
      S.init(a.ub_k, a.k_start);
      int at = -1;
      for (int t = S.next(); t >= 0; t = S.next()) {
        const double Dk = ladder(d0, t);
        const double e2 = recompose_err<NT, NPT>(G, buf, red, gm, em, cm, dm, rm, Dk, 1.0 / Dk);
        at = t;
        S.result(t, e2 <= thr2);
      }
      kst = S.lo;
      if (at != kst) {
        const double Dk = ladder(d0, kst);
        recompose_err<NT, NPT>(G, buf, red, gm, em, cm, dm, rm, Dk, 1.0 / Dk);
      }
      have_y = true;
    }
  }

  // ft = f^ + r^ (r^ = 0 without a record) in natural order, before the record's words reuse
  // the f^ array
  for (int e = t; e < N; e += NT) buf[e] = (double)fh[e] + (have_y ? buf[e] : 0.0);
  __syncthreads();

  if (have_y) {
    {
      // ---- record: header + zigzag integers, group widths, LSB-first bit packing ----
      const double d0 = (kLadderMargin * tau_h) / G.den;
      const double Dk = ladder(d0, kst);
      const double inv = 1.0 / Dk;
      uint32_t um[NPT];
#pragma unroll
      for (int m = 0; m < NPT; ++m) {
        um[m] = 0;
        if (em[m] >= 0) {
          const int q = (int)rint(__dmul_rn(dm[m], inv));
          um[m] = ((uint32_t)q << 1) ^ (uint32_t)(q >> 31);
        }
      }
      for (int g = 0; g < G.nlev; ++g) {
        uint32_t mxu = 0;
#pragma unroll
        for (int m = 0; m < NPT; ++m)
          if (gm[m] == g) mxu = max(mxu, um[m]);
        mxu = block_umax<NT>(mxu, red);
        if (t == 0) s_width[g] = mxu ? 32u - (uint32_t)__clz(mxu) : 0u;
      }
      __syncthreads();
      uint32_t nbits = 0;
      for (int g = 0; g < G.nlev; ++g) {
        const uint32_t wdt = s_width[g];
        if (t == 0) s_base[g] = nbits;
        nbits += (uint32_t)(G.gstart[g + 1] - G.gstart[g]) * wdt;
      }
      const uint32_t nwords = (nbits + 31u) >> 5;
      for (uint32_t k = t; k < nwords; k += NT) words[k] = 0u;
      __syncthreads();
#pragma unroll
      for (int m = 0; m < NPT; ++m) {
        if (em[m] < 0) continue;
        const int g = gm[m];
        const uint32_t wdt = s_width[g];
        if (wdt == 0) continue;
        const uint32_t pos = s_base[g] + (uint32_t)(t + NT * m - G.gstart[g]) * wdt;
        const uint64_t v = (uint64_t)um[m] << (pos & 31u);
        atomicOr(&words[pos >> 5], (uint32_t)v);
        if ((pos & 31u) + wdt > 32u) atomicOr(&words[(pos >> 5) + 1], (uint32_t)(v >> 32));
      }
      __syncthreads();
      uint8_t* slot = a.slots + h * a.slot_stride;
      if (t == 0) {
        uint64_t* hp = (uint64_t*)slot;
        hp[0] = (uint64_t)__double_as_longlong(Dk);
        uint64_t w1 = (uint64_t)(uint32_t)kst | ((uint64_t)(uint32_t)G.nlev << 8);
        uint64_t w2 = 0;
        for (int g = 0; g < G.nlev; ++g) {
          const int byte = 10 + g;
          if (byte < 16) w1 |= (uint64_t)s_width[g] << (8 * (byte - 8));
          else w2 |= (uint64_t)s_width[g] << (8 * (byte - 16));
        }
        hp[1] = w1;
        if (G.hdr_bytes > 16) hp[2] = w2;
      }
      uint32_t* pw = (uint32_t*)(slot + G.hdr_bytes);
      for (uint32_t k = t; k < nwords; k += NT) pw[k] = words[k];
      rec_bytes = (uint32_t)G.hdr_bytes + 4u * nwords;
    }
  }

  // ---- Newton projection onto A x = b, x >= 0 --------------------------------------
  double lam[4] = {0.0, 0.0, 0.0, 0.0};
  int flags = 0, total_upd = 0;
  if (!raw) {
    const double* ft = buf;
    if (a.lam0 || a.analytic) {
      // warm start: keep it unless round 1 allows no update, its Cholesky step fails, or
      // that step makes max_k |g_k| / s_k grow
      double l0[4], v[kNv], g[4], d[4];
      const bool pos = !a.no_positivity;
      bool ok0 = a.max_iter >= 1;
      if (a.analytic) {
        // (A A^T)^-1 (A ft - b): one Newton step at lam = 0 with every cell active
        const double zero[4] = {0.0, 0.0, 0.0, 0.0};
        newton_pass<NT>(G, ft, zero, v, red, false);
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = v[k] - b[k];
        if (!chol_solve4(v, g, l0)) {
#pragma unroll
          for (int k = 0; k < 4; ++k) l0[k] = NAN;
        }
      } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) l0[k] = a.lam0[h * 4 + k];
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) ok0 = ok0 && isfinite(l0[k]);
      if (ok0) {
        newton_pass<NT>(G, ft, l0, v, red, pos);
        double r0 = 0.0;
        bool conv = true;
        double sc[4];
        pass_scales(v, pos, sc);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          g[k] = v[k] - b[k];
          conv = conv && (fabs(g[k]) <= kGTol * (sc[k] + 1e-300));
          r0 = fmax(r0, fabs(g[k]) / (sc[k] + 1e-300));
        }
        if (!conv) {
          ok0 = chol_solve4(v, g, d);
          if (ok0) {
            double l1[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) l1[k] = l0[k] + a.newton_s * d[k];
            newton_pass<NT>(G, ft, l1, v, red, pos);
            double sc1[4];
            pass_scales(v, pos, sc1);
            double r1 = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) r1 = fmax(r1, fabs(v[k] - b[k]) / (sc1[k] + 1e-300));
            ok0 = r1 <= r0;
          }
        }
      }
      if (ok0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) lam[k] = l0[k];
      } else {
        flags |= HCZ_FLAG_WARM_REJECTED;
      }
    }
    bool kl_kept = false;
    if (a.kl) {
      // KL reading first; kept only where it keeps the bound ||f - x|| <= thr (the KL
      // correction is not non-expansive), otherwise the L2 projection below
      double lk[4] = {0.0, 0.0, 0.0, 0.0};
      int k1 = 0, k2 = 0;
      bool okk = newton_round<NT>(G, ft, b, lk, a.newton_s, a.max_iter, false, red, &k1, true, true);
      const bool kl_r2 = !okk;
      if (!okk) {
        const bool paper = a.fallback == HCZ_FALLBACK_PAPER;
        okk = newton_round<NT>(G, ft, b, lk, paper ? 0.01 : 1.0, a.max_iter2, !paper, red, &k2, true, true);
      }
      total_upd = k1 + k2;
      if (okk) {
        double e2[1] = {0.0};
        int i = t % G.n_par, j = t / G.n_par;
        const int di = NT % G.n_par, dj = NT / G.n_par;
        for (int e = t; e < N; e += NT) {
          const Aphi A = make_aphi(G, e, i, j);
          const double fte = ft[e];
          const double x = fte > 0.0 ? fte * exp(-correction(A, lk)) : 0.0;
          const double d = to_d(f[(long long)j * a.rs + i]) - x;
          e2[0] = fma(d, d, e2[0]);
          i += di;
          j += dj;
          if (i >= G.n_par) { i -= G.n_par; ++j; }
        }
        block_sum<NT, 1>(e2, red);
        if (e2[0] <= thr2) {
          kl_kept = true;
          if (kl_r2) flags |= HCZ_FLAG_ROUND2;
#pragma unroll
          for (int k = 0; k < 4; ++k) lam[k] = lk[k];
        }
      }
    }
    int u1 = 0;
    bool ok = kl_kept || newton_round<NT>(G, ft, b, lam, a.newton_s, a.max_iter, false, red, &u1, !a.no_positivity);
    if (!kl_kept) total_upd = u1;
    if (!ok) {
      flags |= HCZ_FLAG_ROUND2;
      int u2 = 0;
      const bool paper = a.fallback == HCZ_FALLBACK_PAPER;
      ok = newton_round<NT>(G, ft, b, lam, paper ? 0.01 : 1.0, a.max_iter2, !paper, red, &u2, !a.no_positivity);
      total_upd += u2;
      if (!ok) raw = true;
    }
    if (!raw && a.no_positivity) flags |= HCZ_FLAG_NOCLIP;
    if (!raw && kl_kept) flags |= HCZ_FLAG_KL;
  }

  uint64_t size = 0;
  if (raw) {
    flags = (flags & (HCZ_FLAG_ROUND2 | HCZ_FLAG_WARM_REJECTED)) | HCZ_FLAG_RAW;
    TIn* dst = (TIn*)(a.slots + h * a.slot_stride);
    int i = t % G.n_par, j = t / G.n_par;
    const int di = NT % G.n_par, dj = NT / G.n_par;
    for (int e = t; e < N; e += NT) {
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
  if (t == 0) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double lv = raw ? 0.0 : round_mantissa(lam[k], a.lambda_bits);
      if (a.lambda_fp32) ((float*)a.lambda)[h * 4 + k] = (float)lv;
      else ((double*)a.lambda)[h * 4 + k] = lv;
    }
    a.flags[h] = (uint8_t)flags;
    a.sizes[h] = size;
    a.kstar[h] = (uint8_t)kst;
    a.iters[h] = (uint16_t)min(total_upd, 65535);
    if (a.t_done) a.t_done[h] = wall_clock64();
  }
}

// ---- moments / QoIs -------------------------------------------------------------------
template <int NT, typename TIn>
__global__ __launch_bounds__(NT) void k_qoi(GridDev G, const TIn* hist, long long hs, long long rs,
                                           double* bo, double* qo, double* no) {
  __shared__ double red[NT / 64 * 16];
  const int t = threadIdx.x;
  const long long h = blockIdx.x;
  const TIn* f = hist + h * hs;
  dd ff{0.0, 0.0};
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int i = t % G.n_par, j = t / G.n_par;
  const int di = NT % G.n_par, dj = NT / G.n_par;
  for (int e = t; e < G.N; e += NT) {
    const double fv = to_d(f[(long long)j * rs + i]);
    ff = dd_add_d(ff, fv * fv);
    const Aphi A = make_aphi(G, e, i, j);
    acc[0] = fma(A.a0, fv, acc[0]);
    acc[1] = fma(A.a1, fv, acc[1]);
    acc[2] = fma(A.a2, fv, acc[2]);
    acc[3] = fma(A.a3, fv, acc[3]);
    i += di;
    j += dj;
    if (i >= G.n_par) { i -= G.n_par; ++j; }
  }
  block_sum<NT, 4>(acc, red);
  ff = block_dd<NT>(ff, red);
  if (t == 0) {
    if (bo) for (int k = 0; k < 4; ++k) bo[h * 4 + k] = acc[k];
    if (qo) {
      const double n = acc[0];
      const double u = G.Vpar * acc[1] / n;
      qo[h * 4 + 0] = n;
      qo[h * 4 + 1] = u;
      qo[h * 4 + 2] = 0.5 * G.mass * (G.Vperp * G.Vperp) * acc[2] / n;
      qo[h * 4 + 3] = 0.5 * G.mass * ((G.Vpar * G.Vpar) * acc[3] / n - u * u);
    }
    if (no) no[h] = sqrt(ff.hi + ff.lo);
  }
}

// ---- decompression ---------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld32(const uint8_t* p) { return *(const uint32_t*)p; }

template <int NT, int NPT, typename TIn, typename TOut>
__global__ __launch_bounds__(NT) void k_decompress(GridDev G, DecompressArgs a) {
  extern __shared__ double smem[];
  const int N = G.N;
  double* buf = smem;
  __shared__ uint32_t s_width[kMaxLev], s_base[kMaxLev];
  __shared__ int s_corrupt;
  const int t = threadIdx.x;
  const long long h = blockIdx.x;
  const int fl = a.flags[h];
  const uint8_t* rec = a.stream + a.offsets[h];
  TOut* out = (TOut*)a.out + h * (long long)N;
  if ((fl & (HCZ_FLAG_RAW | HCZ_FLAG_CODED)) &&
      (a.offsets[h + 1] > a.capacity || a.offsets[h + 1] < a.offsets[h] ||
       a.offsets[h + 1] - a.offsets[h] < (uint64_t)G.hdr_bytes)) {
    for (int e = t; e < N; e += NT) out[e] = (TOut)NAN;   // record missing from the stream
    return;
  }
  if (fl & HCZ_FLAG_RAW) {
    // a verbatim record holds exactly the N input values; any other size decodes to NaN
    if (a.offsets[h + 1] - a.offsets[h] != (uint64_t)N * sizeof(TIn)) {
      for (int e = t; e < N; e += NT) out[e] = (TOut)NAN;
      return;
    }
    const TIn* src = (const TIn*)rec;   // records start 4-byte aligned
    if (sizeof(TIn) == 8) {
      const uint32_t* s32 = (const uint32_t*)rec;
      for (int e = t; e < N; e += NT) {
        const uint64_t lo = s32[2 * e], hi = s32[2 * e + 1];
        out[e] = (TOut)__longlong_as_double((long long)(lo | (hi << 32)));
      }
    } else {
      for (int e = t; e < N; e += NT) out[e] = (TOut)src[e];
    }
    return;
  }
  const float* fhp = a.fhat ? a.fhat + h * (long long)N : nullptr;
  double Delta = 0.0;
  const bool coded = (fl & HCZ_FLAG_CODED) != 0;
  if (coded) {
    const uint64_t lo = ld32(rec), hi = ld32(rec + 4);
    Delta = __longlong_as_double((long long)(lo | (hi << 32)));
    if (t < G.nlev) s_width[t] = rec[10 + t];
    __syncthreads();
    if (t == 0) {
      uint32_t nb = 0;
      bool corrupt = false;
      for (int g = 0; g < G.nlev; ++g) {
        s_base[g] = nb;
        nb += (uint32_t)(G.gstart[g + 1] - G.gstart[g]) * s_width[g];
        corrupt = corrupt || s_width[g] > 32u;
      }
      // a header that does not fit its record decodes to NaN rather than reading past it
      s_corrupt = corrupt || (uint64_t)G.hdr_bytes + 4ull * (((uint64_t)nb + 31u) >> 5) >
                                 a.offsets[h + 1] - a.offsets[h];
    }
    __syncthreads();
    if (s_corrupt) {
      for (int e = t; e < N; e += NT) out[e] = (TOut)NAN;
      return;
    }
  }
  const uint8_t* payload = rec + G.hdr_bytes;
  double lam[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    lam[k] = a.lambda_fp32 ? (double)((const float*)a.lambda)[h * 4 + k] : ((const double*)a.lambda)[h * 4 + k];
  const bool clip = (fl & HCZ_FLAG_NOCLIP) == 0;
  const bool kl = (fl & HCZ_FLAG_KL) != 0;
  int em[NPT], gm[NPT];
  Interp cm[NPT];
  double dq[NPT], ym[NPT];
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    const int p = t + NT * m;
    em[m] = -1;
    gm[m] = 99;
    dq[m] = 0.0;
    ym[m] = 0.0;
    if (p < N) {
      const uint32_t ij = G.node_ij[p];
      const int i = ij & 0xffff, j = ij >> 16;
      em[m] = j * G.n_par + i;
      gm[m] = group_of(G, p);
      cm[m] = make_interp(G, i, j);
      if (coded) {
        const uint32_t w = s_width[gm[m]];
        uint32_t u = 0;
        if (w) {
          const uint32_t pos = s_base[gm[m]] + (uint32_t)(p - G.gstart[gm[m]]) * w;
          const uint32_t wi = pos >> 5, sh = pos & 31u;
          uint64_t v = ld32(payload + 4 * wi);
          if (sh + w > 32u) v |= (uint64_t)ld32(payload + 4 * (wi + 1)) << 32;
          u = (uint32_t)((v >> sh) & ((w == 32u) ? 0xffffffffull : ((1ull << w) - 1ull)));
        }
        const int q = (int)((u >> 1) ^ (0u - (u & 1u)));
        dq[m] = __dmul_rn(Delta, (double)q);
      }
    }
  }
  if (coded) {
    for (int g = 0; g < G.nlev; ++g) {
#pragma unroll
      for (int m = 0; m < NPT; ++m) {
        if (gm[m] == g) {
          const double y = (g == 0) ? dq[m] : __dadd_rn(dq[m], predict(buf, cm[m]));
          buf[em[m]] = y;
          ym[m] = y;
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int m = 0; m < NPT; ++m) {
    if (em[m] < 0) continue;
    const int e = em[m];
    const int i = e % G.n_par, j = e / G.n_par;
    const float fv = fhp ? fhp[e] : 0.0f;
    const double ft = (double)fv + ym[m];
    const Aphi A = make_aphi(G, e, i, j);
    if (kl) {
      ym[m] = ft > 0.0 ? ft * exp(-correction(A, lam)) : 0.0;
    } else {
      const double y = ft - correction(A, lam);
      ym[m] = clip ? fmax(0.0, y) : y;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < NPT; ++m)
    if (em[m] >= 0) buf[em[m]] = ym[m];
  __syncthreads();
  for (int e = t; e < N; e += NT) out[e] = (TOut)buf[e];
}

// ---- launchers -------------------------------------------------------------------------
static int pick_nt(int N) { return N <= 1536 ? 256 : (N <= 3072 ? 512 : 1024); }

hipError_t launch_residual(const GridDev& G, const ResidualArgs& a, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  const int v = a.variant;
  const bool wave_v = v == HCZ_VARIANT_AUTO || v == HCZ_VARIANT_WAVE_FIXED || v == HCZ_VARIANT_WAVE;
  if (wave_path(G) && wave_v) return launch_residual_w(G, a, st);
  if ((v == HCZ_VARIANT_TEAM2 || v == HCZ_VARIANT_TEAM4) && !a.kl)
    return launch_residual_t(G, a, v == HCZ_VARIANT_TEAM2 ? 2 : 4, st);
  if (v == HCZ_VARIANT_AUTO && !a.kl && !wave_path(G) && (team_path(G, 2) || team_path(G, 4)))
    return launch_residual_t(G, a, team_path(G, 2) ? 2 : 4, st);
  // threads x nodes per thread: the variant's, else the smallest that holds the grid
  // (256 x 6 up to 1536 nodes, then 512 x 5 (2560) and 512 x 9 (4608))
  int shape = v;
  if (wave_v) shape = G.N <= 1536 ? HCZ_VARIANT_BLOCK_256x6 : (G.N <= 2560 ? HCZ_VARIANT_BLOCK_512x5 : HCZ_VARIANT_BLOCK_512x9);
  const int nt = shape == HCZ_VARIANT_BLOCK_256x6 ? 256 : 512;
  const size_t lds = (size_t)G.N * 8 + (size_t)((G.N + 1) / 2) * 8 + (size_t)(nt / 64) * kNv * 8;
  dim3 grid((unsigned)a.H), block(nt);
#define HCZ_RES(NT, NPT, T) hipLaunchKernelGGL((k_residual<NT, NPT, T>), grid, block, lds, st, G, a)
#define HCZ_RES_T(T)                                                      \
  do {                                                                    \
    if (shape == HCZ_VARIANT_BLOCK_256x6) HCZ_RES(256, 6, T);             \
    else if (shape == HCZ_VARIANT_BLOCK_512x5) HCZ_RES(512, 5, T);        \
    else HCZ_RES(512, 9, T);                                              \
  } while (0)
  if (a.dtype == HCZ_F32) HCZ_RES_T(float);
  else HCZ_RES_T(double);
#undef HCZ_RES_T
#undef HCZ_RES
  return hipGetLastError();
}

hipError_t launch_qoi(const GridDev& G, const void* hist, int dtype, long long H, long long hs,
                      long long rs, double* b, double* qoi, double* norm, hipStream_t st) {
  if (H <= 0) return hipSuccess;
  dim3 grid((unsigned)H), block(256);
  if (dtype == HCZ_F32)
    hipLaunchKernelGGL((k_qoi<256, float>), grid, block, 0, st, G, (const float*)hist, hs, rs, b, qoi, norm);
  else
    hipLaunchKernelGGL((k_qoi<256, double>), grid, block, 0, st, G, (const double*)hist, hs, rs, b, qoi, norm);
  return hipGetLastError();
}

hipError_t launch_decompress(const GridDev& G, const DecompressArgs& a, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  if (wave_path(G)) return launch_decompress_w(G, a, st);
  const int nt = pick_nt(G.N);
  const size_t lds = (size_t)G.N * 8;
  dim3 grid((unsigned)a.H), block(nt);
#define HCZ_DEC(NT, TI, TO) hipLaunchKernelGGL((k_decompress<NT, 6, TI, TO>), grid, block, lds, st, G, a)
#define HCZ_DEC_NT(TI, TO) \
  do { if (nt == 256) HCZ_DEC(256, TI, TO); else if (nt == 512) HCZ_DEC(512, TI, TO); else HCZ_DEC(1024, TI, TO); } while (0)
  if (a.in_dtype == HCZ_F32) {
    if (a.out_dtype == HCZ_F64) HCZ_DEC_NT(float, double); else HCZ_DEC_NT(float, float);
  } else {
    if (a.out_dtype == HCZ_F64) HCZ_DEC_NT(double, double); else HCZ_DEC_NT(double, float);
  }
#undef HCZ_DEC_NT
#undef HCZ_DEC
  return hipGetLastError();
}

}  // namespace hcz
