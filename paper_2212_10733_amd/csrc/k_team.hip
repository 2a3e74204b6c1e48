// Residual coding and Newton projection (Section III Stages 4-5) for grids too large for
// one wave: a team of W waves (W = 2 or 4) owns one histogram, one workgroup per team.
//
// The layout is the wave kernels' (k_wave.hip) widened to 64 W lanes: the histogram sits
// in an FP64 LDS buffer in natural order plus one zero cell; per slot, team lane t holds
// one node of the multilevel decomposition (slots of 64 W nodes, one coefficient group
// each except slot 0, which holds the coarsest groups), its residual and coefficient in
// registers and its interpolation corners as byte offsets into the buffer.  The slot
// entries are read from global memory once per histogram, so LDS holds only the buffer,
// the weights and the reduction scratch, and two teams share a SIMD.  A workgroup barrier
// closes every coefficient group (later groups read what earlier ones wrote) and every
// cross-wave reduction; every wave of a team computes the same reduced bits, so the
// team's control flow stays uniform and the barriers match.  The column passes (loading,
// moments, ft, Newton) split each grid column into row chunks so that every wave works.
// Records, flags and k* are those of the other kernel families, byte for byte.
#include "wave_ops.h"

namespace hcz {

constexpr int kTR = 20;                 // values one wave contributes to a team reduction
constexpr int kTeamLdsFixed = 64 + 2 * kMaxDim;

template <int W>
__host__ __device__ __forceinline__ size_t lds_bytes_t(const GridDev& G) {
  return (kTeamLdsFixed + 2 * W * kTR + (size_t)(G.N + 1)) * sizeof(double);
}

template <int W>
struct Team {
  static constexpr int NT = 64 * W;
  static constexpr int K = W == 2 ? 0 : 1;       // index of the team's slot tables
  double* s_w;
  double* s_cc;
  double* red;                                  // [2][W][kTR]
  char* yb;
  int buf;                                      // reduction buffer in use (alternates)

  __device__ __forceinline__ void sync() const { __syncthreads(); }

  // Sum each of the first N values over the team: wave butterflies, then the W wave totals
  // in wave order.  The two buffers alternate, so the next reduction's writes cannot meet
  // this one's reads (its own barrier lies between them).
  template <int N, int M>
  __device__ __forceinline__ void sum(double (&v)[M]) {
    static_assert(N <= kTR && N <= M, "reduction too wide");
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wsum(v[k]);
    double* r = red + buf * W * kTR;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < N; ++k) r[wv * kTR + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = r[k];
#pragma unroll
      for (int w = 1; w < W; ++w) s = s + r[w * kTR + k];
      v[k] = s;
    }
    buf ^= 1;
  }
  template <int N, int M>
  __device__ __forceinline__ void max(double (&v)[M]) {
#pragma unroll
    for (int k = 0; k < N; ++k) v[k] = wmax(v[k]);
    double* r = red + buf * W * kTR;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int k = 0; k < N; ++k) r[wv * kTR + k] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < N; ++k) {
      double s = r[k];
#pragma unroll
      for (int w = 1; w < W; ++w) s = fmax(s, r[w * kTR + k]);
      v[k] = s;
    }
    buf ^= 1;
  }
  __device__ __forceinline__ uint32_t umax(uint32_t u) {
    double v[1] = {(double)wumax(u)};            // exact: u < 2^32
    double* r = red + buf * W * kTR;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) r[wv * kTR] = v[0];
    __syncthreads();
    double s = r[0];
#pragma unroll
    for (int w = 1; w < W; ++w) s = fmax(s, r[w * kTR]);
    buf ^= 1;
    return (uint32_t)s;
  }
  __device__ __forceinline__ dd sum_dd(dd v) {
    v = wdd(v);
    double* r = red + buf * W * kTR;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
      r[wv * kTR] = v.hi;
      r[wv * kTR + 1] = v.lo;
    }
    __syncthreads();
    dd s{r[0], r[1]};
#pragma unroll
    for (int w = 1; w < W; ++w) s = dd_add(s, dd{r[w * kTR], r[w * kTR + 1]});
    buf ^= 1;
    return s;
  }
  __device__ __forceinline__ bool any(bool b) {
    double v[1] = {__ballot(b) != 0 ? 1.0 : 0.0};
    max<1>(v);
    return v[0] != 0.0;
  }
};

// The team's slot tables (one set per team width).
struct TeamTabs {
  int nslots, ncoarse;
  uint32_t bil, sync;
  const uint32_t* meta;
  const uint16_t* rank;
  const double* wtab;
  int nw;
};
template <int W>
__device__ __forceinline__ TeamTabs team_tabs(const GridDev& G) {
  constexpr int k = Team<W>::K;
  return TeamTabs{G.tnslots[k], G.tncoarse[k], G.tslot_bil[k], G.tslot_sync[k], G.tslot_meta[k],
                  G.tslot_rank[k], G.twtab[k], G.tnw[k]};
}

template <int W>
__device__ __forceinline__ Team<W> setup_team(const GridDev& G, double* smem) {
  Team<W> T;
  T.s_w = smem;
  T.s_cc = smem + 64;
  T.red = smem + kTeamLdsFixed;
  double* y = smem + kTeamLdsFixed + 2 * W * kTR;
  T.yb = (char*)y;
  T.buf = 0;
  const int t = threadIdx.x;
  const TeamTabs tb = team_tabs<W>(G);
  for (int k = t; k < tb.nw; k += Team<W>::NT) T.s_w[k] = tb.wtab[k];
  for (int k = t; k < G.n_perp; k += Team<W>::NT) {
    const double c = G.cperp[k];
    T.s_cc[2 * k] = c;
    T.s_cc[2 * k + 1] = c * c;
  }
  if (t == 0) y[G.N] = 0.0;
  return T;
}

__device__ __forceinline__ double ldt(const char* yb, uint32_t off) { return *(const double*)(yb + off); }
__device__ __forceinline__ void stt(char* yb, uint32_t off, double v) { *(double*)(yb + off) = v; }

// Interpolated value of a node from its corners (entry words m, m2), in the coder's fixed
// unfused order: the two-corner form unless FOUR.
template <bool FOUR, int W>
__device__ __forceinline__ double predict_t(const Team<W>& T, uint2 m, uint32_t m2) {
  const double y00 = ldt(T.yb, m.x >> 16), y10 = ldt(T.yb, m.y & 0xffffu);
  const double s = T.s_w[(m2 >> 16) & 63u];
  const double p0 = __dadd_rn(y00, __dmul_rn(s, __dsub_rn(y10, y00)));
  if (!FOUR) return p0;
  const double y01 = ldt(T.yb, m.y >> 16), y11 = ldt(T.yb, m2 & 0xffffu);
  const double tt = T.s_w[(m2 >> 22) & 63u];
  const double p1 = __dadd_rn(y01, __dmul_rn(s, __dsub_rn(y11, y01)));
  return __dadd_rn(p0, __dmul_rn(tt, __dsub_rn(p1, p0)));
}

// Slot s >= 1 of a team table: four-corner form, and whether a later group starts after it.
__device__ __forceinline__ bool tbit(uint32_t mask, int s) { return (mask >> s) & 1u; }
__device__ __forceinline__ int tgroup_of_slot(const TeamTabs& tb, int s) {
  return tb.ncoarse + __popc(tb.sync & ((1u << s) - 1u) & ~1u);
}

template <int NS>
struct TeamSlots {
  uint2 m[NS];
  uint32_t m2[NS];
};
// Entry words hidden from loop-invariant code motion (as in the wave kernels: otherwise
// every slot's decoded addresses are hoisted out of the search loop and spill).
__device__ __forceinline__ uint2 topaque2(uint2 m) {
  asm volatile("" : "+v"(m.x), "+v"(m.y));
  return m;
}
__device__ __forceinline__ uint32_t topaque1(uint32_t m) {
  asm volatile("" : "+v"(m));
  return m;
}

// Recompose every node with quantised values dq(s) into the buffer (slots of the finest
// group only when STORE_ALL) and return sum (rm - y)^2 over the histogram.
template <int W, int NS, bool STORE_ALL, typename DQ>
__device__ __forceinline__ double recompose_t(const TeamTabs& tb, Team<W>& T, const TeamSlots<NS>& R,
                                              const double (&rm)[NS], uint32_t keep, DQ dqf) {
  double acc = 0.0;
  {
    const uint2 m = topaque2(R.m[0]);
    const uint32_t m2 = topaque1(R.m2[0]);
    const int g0 = (int)(m2 >> 28);
    const double dq = dqf(0);
    for (int g = 0; g < tb.ncoarse; ++g) {
      if (g0 == g) {
        // the coarsest values are dq itself: +0 for a quantised zero as in the oracle
        const double v = g == 0 ? __dadd_rn(dq, 0.0) : __dadd_rn(dq, predict_t<true>(T, m, m2));
        stt(T.yb, m.x & 0xffffu, v);
        const double e = rm[0] - v;
        acc = fma(e, e, acc);
      }
      T.sync();
    }
  }
#pragma unroll
  for (int s = 1; s < NS; ++s) {
    if (s < tb.nslots) {
      const uint2 m = topaque2(R.m[s]);
      const uint32_t m2 = topaque1(R.m2[s]);
      const double dq = dqf(s);
      const double v = __dadd_rn(dq, tbit(tb.bil, s) ? predict_t<true>(T, m, m2) : predict_t<false>(T, m, m2));
      if (STORE_ALL || tbit(keep, s)) stt(T.yb, m.x & 0xffffu, v);
      const double e = rm[s] - v;
      acc = fma(e, e, acc);
      if (tbit(tb.sync, s)) T.sync();
    }
  }
  double a[1] = {acc};
  T.template sum<1>(a);
  return a[0];
}

// Column tasks: grid column i split into R row chunks of `rows` rows, task = r * n_par + i.
struct TaskSplit {
  int ntask, rows;
};
template <int W>
__device__ __forceinline__ TaskSplit task_split(const GridDev& G) {
  const int R = max(1, Team<W>::NT / G.n_par);
  const int rows = (G.n_perp + R - 1) / R;
  return TaskSplit{G.n_par * R, rows};
}
// begin(i), body(i, j, off) for the task's rows, fold(i); every thread of the team.
template <int W, typename BEGIN, typename BODY, typename FOLD>
__device__ __forceinline__ void for_tasks(const GridDev& G, const TaskSplit& S, BEGIN begin, BODY body, FOLD fold) {
  for (int task = threadIdx.x; task < S.ntask; task += Team<W>::NT) {
    const int i = task % G.n_par, j0 = (task / G.n_par) * S.rows, j1 = min(G.n_perp, j0 + S.rows);
    begin(i);
    uint32_t off = (uint32_t)(j0 * G.n_par + i) * 8u;
    for (int j = j0; j < j1; ++j) {
      body(i, j, off);
      off += (uint32_t)G.n_par * 8u;
    }
    fold(i);
  }
}
// As for_tasks, with load(i, j) issued for a chunk of rows before body(i, j, off, v) runs.
template <int W, typename BEGIN, typename LOAD, typename BODY, typename FOLD>
__device__ __forceinline__ void for_tasks_pre(const GridDev& G, const TaskSplit& S, BEGIN begin, LOAD load, BODY body,
                                              FOLD fold) {
  constexpr int CH = 24;
  using V = decltype(load(0, 0));
  for (int task = threadIdx.x; task < S.ntask; task += Team<W>::NT) {
    const int i = task % G.n_par, j0 = (task / G.n_par) * S.rows, j1 = min(G.n_perp, j0 + S.rows);
    begin(i);
    uint32_t off = (uint32_t)(j0 * G.n_par + i) * 8u;
    for (int jc = j0; jc < j1; jc += CH) {
      V v[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (jc + k < j1) v[k] = load(i, jc + k);
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (jc + k < j1) {
          body(i, jc + k, off, v[k]);
          off += (uint32_t)G.n_par * 8u;
        }
    }
    fold(i);
  }
}

// One Newton pass at lam over the team's buffer (Section III Stage 5): v[0..3] = A x, v[4] =
// sum |A_1| x, v[15] = ||x - ft||^2 when THETA, sc the stopping rule's scales and hs the
// Hessian A diag(x > 0) A^T (upper triangle as in hess order); the same per-column
// arithmetic as the wave kernels, all sums reduced in one team reduction.
template <int W, bool UVOL, bool THETA, bool POS>
__device__ __forceinline__ void newton_pass_t(const GridDev& G, Team<W>& T, const TaskSplit& S, const double (&lam)[4],
                                              double (&v)[16], double (&sc)[4], double (&hs)[9]) {
  double r[18];
#pragma unroll
  for (int k = 0; k < 18; ++k) r[k] = 0.0;
  double sx, sxc, sxa, sxca, h0, hc, hcc, s2;
  double pa = 0.0;
  for_tasks<W>(
      G, S,
      [&](int i) {
        const double a = G.apar[i];
        pa = fma(fma(lam[3], a, lam[1]), a, lam[0]);
        sx = sxc = sxa = sxca = h0 = hc = hcc = s2 = 0.0;
      },
      [&](int i, int j, uint32_t off) {
        const double c = T.s_cc[2 * j], c2 = T.s_cc[2 * j + 1];
        const double w = UVOL ? G.vol0 : G.vol[j * G.n_par + i];
        const double ft = ldt(T.yb, off);
        const double y = ft - w * fma(lam[2], c, pa);
        const double x = POS ? fmax(0.0, y) : y;
        const double wx = UVOL ? x : w * x;
        sx += wx;
        sxc = fma(c, wx, sxc);
        if (!POS) {
          const double wxa = fabs(wx);
          sxa += wxa;
          sxca = fma(c, wxa, sxca);
        }
        const double act = (!POS || x > 0.0) ? 1.0 : 0.0;
        const double w2 = UVOL ? act : act * (w * w);
        h0 += w2;
        hc = fma(w2, c, hc);
        hcc = fma(w2, c2, hcc);
        if (THETA) {
          const double dx = x - ft;
          s2 = fma(dx, dx, s2);
        }
      },
      [&](int i) {
        const double a = G.apar[i], a2 = a * a;
        r[0] += sx;
        r[1] = fma(a, sx, r[1]);
        r[2] += sxc;
        r[3] = fma(a2, sx, r[3]);
        r[4] = fma(fabs(a), POS ? sx : sxa, r[4]);
        r[5] += s2;
        if (!POS) {
          r[15] += sxa;
          r[16] += sxca;
          r[17] = fma(a2, sxa, r[17]);
        }
        r[6] += h0;
        r[7] = fma(a, h0, r[7]);
        r[8] += hc;
        r[9] = fma(a2, h0, r[9]);
        r[10] = fma(a, hc, r[10]);
        r[11] = fma(a2 * a, h0, r[11]);
        r[12] += hcc;
        r[13] = fma(a2, hc, r[13]);
        r[14] = fma(a2 * a2, h0, r[14]);
      });
  T.template sum<18>(r);
  const double s1 = UVOL ? G.vol0 : 1.0;
  v[0] = r[0] * s1;
  v[1] = r[1] * s1;
  v[2] = r[2] * s1;
  v[3] = r[3] * s1;
  v[4] = r[4] * s1;
  v[15] = THETA ? r[5] : 0.0;
  if (POS) {
    sc[0] = v[0];
    sc[1] = v[4];
    sc[2] = v[2];
    sc[3] = v[3];
  } else {
    sc[0] = r[15] * s1;
    sc[1] = v[4];
    sc[2] = r[16] * s1;
    sc[3] = r[17] * s1;
  }
  const double s2v = UVOL ? G.vol0 * G.vol0 : 1.0;
#pragma unroll
  for (int k = 0; k < 9; ++k) hs[k] = r[6 + k] * s2v;
}

template <int W, bool UVOL, bool POS>
__device__ __forceinline__ int newton_t(const GridDev& G, Team<W>& T, const TaskSplit& S, const double (&b)[4],
                                        double (&lam)[4], double s1, int max1, double s2, int max2, bool armijo2,
                                        int* upd, bool have_init, const double (&lam_init)[4], bool* rejected) {
  double hs[9];
  auto pass = [&](bool theta, const double (&cand)[4], double (&v)[16], double (&sc)[4]) {
    if (theta) newton_pass_t<W, UVOL, true, POS>(G, T, S, cand, v, sc, hs);
    else newton_pass_t<W, UVOL, false, POS>(G, T, S, cand, v, sc, hs);
  };
  auto hess = [&](double (&v)[16]) {
    constexpr int dst[9] = {5, 6, 7, 8, 10, 11, 12, 13, 14};
#pragma unroll
    for (int k = 0; k < 9; ++k) v[dst[k]] = hs[k];
    v[9] = v[8];
  };
  return newton_core(pass, hess, b, lam, s1, max1, s2, max2, armijo2, upd, have_init, lam_init, rejected);
}

template <int W>
constexpr int team_slots() { return W == 2 ? kTeamSlots2 : kTeamSlots4; }

// Histogram h (< a.H) on the first 64 W threads of the workgroup, the team's LDS set up.
template <typename TIn, bool UVOL, int W>
__device__ __forceinline__ void residual_t_hist(const GridDev& G, const ResidualArgs& a, Team<W>& T, long long h) {
  constexpr int NS = team_slots<W>();
  constexpr int NT = Team<W>::NT;
  const int N = G.N;
  const int t = threadIdx.x;
  const TeamTabs tb = team_tabs<W>(G);
  const TaskSplit S = task_split<W>(G);
  const TIn* f = (const TIn*)a.hist + h * a.hs;
  const float* fhp = a.fhat ? a.fhat + h * (long long)N : nullptr;
  uint32_t* words = (uint32_t*)T.yb;     // payload words borrow the buffer before the last recomposition

  // ---- column pass: residual into the buffer, moments, norms, range ----
  dd ff{0.0, 0.0};
  double mo[5] = {0.0, 0.0, 0.0, 0.0, 0.0};     // rr, m0..m3
  double mx2[2] = {-INFINITY, -INFINITY};        // max f, max -f
  bool bad = false;
  {
    double sf = 0.0, sfc = 0.0;
    struct FH {
      TIn f;
      float h;
    };
    for_tasks_pre<W>(
        G, S, [&](int) { sf = sfc = 0.0; },
        [&](int i, int j) { return FH{f[(long long)j * a.rs + i], fhp ? fhp[j * G.n_par + i] : 0.0f}; },
        [&](int i, int j, uint32_t off, FH ld) {
          const double fv = (double)ld.f;
          const double hv = (double)ld.h;
          const double r = fv - hv;
          stt(T.yb, off, r);
          const double p = fv * fv;
          const double hi = ff.hi + p;
          const double bb = hi - ff.hi;
          ff.lo += (ff.hi - (hi - bb)) + (p - bb);
          ff.hi = hi;
          mo[0] = fma(r, r, mo[0]);
          const double w = UVOL ? fv : G.vol[j * G.n_par + i] * fv;
          sf += w;
          sfc = fma(T.s_cc[2 * j], w, sfc);
          bad |= !isfinite(fv);
          mx2[0] = fmax(mx2[0], fv);
          mx2[1] = fmax(mx2[1], -fv);
        },
        [&](int i) {
          const double av = G.apar[i];
          mo[1] += sf;
          mo[2] = fma(av, sf, mo[2]);
          mo[3] += sfc;
          mo[4] = fma(av * av, sf, mo[4]);
        });
  }
  {
    const double hi = ff.hi + ff.lo;
    ff = dd{hi, ff.lo - (hi - ff.hi)};
  }
  ff = T.sum_dd(ff);
  T.template sum<5>(mo);
  T.template max<2>(mx2);
  bad = T.any(bad);
  const double rr = mo[0];
  double b[4] = {mo[1], mo[2], mo[3], mo[4]};
  if (UVOL) {
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] *= G.vol0;
  }
  const double tau = a.tau_hist ? a.tau_hist[h] : a.tau;
  const double tau_h = (a.tau_mode == HCZ_TAU_NRMSE) ? (tau * G.sqrtN) * (mx2[0] - (-mx2[1]))
                                                     : tau * sqrt(ff.hi + ff.lo);
  const double thr = kSelMargin * tau_h;
  const double thr2 = thr * thr;
  bool raw = bad || !(b[0] > 0.0) || !(tau >= 0.0 && tau <= DBL_MAX);
  const bool coded = rr > thr2;
  if (coded && !(tau_h > 0.0)) raw = true;

  int kst = 0xff;
  uint32_t rec_bytes = 0;
  // ft = fhat + rhat (rhat = 0 when not coded), written over the buffer in natural order
  auto load_ft = [&](bool with_r) {
    for_tasks_pre<W>(
        G, S, [](int) {}, [&](int i, int j) { return fhp ? fhp[j * G.n_par + i] : 0.0f; },
        [&](int, int, uint32_t off, float hq) {
          const double hv = (double)hq;
          stt(T.yb, off, with_r ? hv + ldt(T.yb, off) : hv);
        },
        [](int) {});
    T.sync();
  };
  bool ft_ready = false;
  if (coded && !raw) {
    // every slot: its entry words, residual and coefficient d = r - P(r) (no node is rewritten)
    TeamSlots<NS> R;
    const uint32_t* me = tb.meta;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      R.m[s] = make_uint2(0u, 0u);
      R.m2[s] = 0u;
      if (s < tb.nslots) {
        const size_t k = ((size_t)s * NT + t) * 3;
        R.m[s] = make_uint2(me[k], me[k + 1]);
        R.m2[s] = me[k + 2];
      }
    }
    const uint32_t keep = G.tslot_keep[Team<W>::K];
    double dm[NS], rm[NS];
    double mx[1] = {0.0};
    {
      const uint2 m = R.m[0];
      const uint32_t mm2 = R.m2[0];
      rm[0] = ldt(T.yb, m.x & 0xffffu);
      dm[0] = (mm2 >> 28) == 0 ? rm[0] : __dsub_rn(rm[0], predict_t<true>(T, m, mm2));
      mx[0] = fabs(dm[0]);
    }
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      dm[s] = 0.0;
      rm[s] = 0.0;
      if (s < tb.nslots) {
        const uint2 m = R.m[s];
        const uint32_t mm2 = R.m2[s];
        rm[s] = ldt(T.yb, m.x & 0xffffu);
        dm[s] = __dsub_rn(rm[s], tbit(tb.bil, s) ? predict_t<true>(T, m, mm2) : predict_t<false>(T, m, mm2));
        mx[0] = fmax(mx[0], fabs(dm[s]));
      }
    }
    T.template max<1>(mx);               // its barrier also ends every read of the residuals
    const double d0 = (kLadderMargin * tau_h) / G.den;
    if (mx[0] * (1.0 / d0) >= kQMax) raw = true;
    if (!raw) {
      // the bound search over the ladder, or the user's step (an empty search)
      LadderSearch LS;
      LS.init(a.ub_k, a.k_start);
      for (int k = LS.next(); k >= 0; k = LS.next()) {
        const double Dk = ladder(d0, k);
        const double inv = 1.0 / Dk;
        const double e2 = recompose_t<W, NS, false>(tb, T, R, rm, keep,
                                                    [&](int s) { return __dmul_rn(Dk, rint(__dmul_rn(dm[s], inv))); });
        LS.result(k, e2 <= thr2);
      }
      kst = LS.lo;
      const double Dk = ladder(d0, kst);
      const double inv = 1.0 / Dk;
      auto zz = [&](double d) -> uint32_t {
        const int q = (int)rint(__dmul_rn(d, inv));
        return ((uint32_t)q << 1) ^ (uint32_t)(q >> 31);
      };
      const uint32_t zero_off = (uint32_t)N * 8u;
      // per-group maxima of the zigzag integers (wave-uniform, then over the team)
      uint32_t gmx[kMaxLev];
#pragma unroll
      for (int g = 0; g < kMaxLev; ++g) gmx[g] = 0u;
      const int g0 = (int)(R.m2[0] >> 28);
      {
        const uint32_t u0 = zz(dm[0]);
#pragma unroll
        for (int g = 0; g < kMaxLev; ++g)
          if (g < tb.ncoarse) gmx[g] = T.umax(g0 == g ? u0 : 0u);
      }
      uint32_t cur = 0u;
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        if (s < tb.nslots) {
          cur = max(cur, zz(dm[s]));          // padding lanes hold d = 0
          if (tbit(tb.sync, s)) {
            const uint32_t v = T.umax(cur);
            const int g = tgroup_of_slot(tb, s);
#pragma unroll
            for (int q = 0; q < kMaxLev; ++q)
              if (q == g) gmx[q] = max(gmx[q], v);
            cur = 0u;
          }
        }
      }
      uint32_t wd[kMaxLev], bs[kMaxLev];
      uint32_t nbits = 0;
#pragma unroll
      for (int g = 0; g < kMaxLev; ++g) {
        wd[g] = (g < G.nlev && gmx[g]) ? 32u - (uint32_t)__clz(gmx[g]) : 0u;
        bs[g] = nbits;
        if (g < G.nlev) nbits += (uint32_t)(G.gstart[g + 1] - G.gstart[g]) * wd[g];
      }
      const uint32_t nwords = (nbits + 31u) >> 5;
      for (uint32_t k = t; k < nwords; k += NT) words[k] = 0u;
      T.sync();
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s < tb.nslots) {
          const uint32_t eo = R.m[s].x & 0xffffu;
          const int g = s == 0 ? g0 : tgroup_of_slot(tb, s);
          uint32_t wdt = 0u, base = 0u;
#pragma unroll
          for (int q = 0; q < kMaxLev; ++q)
            if (q == g) { wdt = wd[q]; base = bs[q]; }
          if (eo != zero_off && wdt != 0) {
            const uint32_t pos = base + (uint32_t)tb.rank[(size_t)s * NT + t] * wdt;
            const uint64_t v = (uint64_t)zz(dm[s]) << (pos & 31u);
            atomicOr(&words[pos >> 5], (uint32_t)v);
            if ((pos & 31u) + wdt > 32u) atomicOr(&words[(pos >> 5) + 1], (uint32_t)(v >> 32));
          }
        }
      }
      T.sync();
      uint8_t* slot = a.slots + h * a.slot_stride;
      if (t == 0) {
        uint64_t* hp = (uint64_t*)slot;
        hp[0] = (uint64_t)__double_as_longlong(Dk);
        uint64_t w1 = (uint64_t)(uint32_t)kst | ((uint64_t)(uint32_t)G.nlev << 8);
        uint64_t w2 = 0;
#pragma unroll
        for (int g = 0; g < kMaxLev; ++g) {
          const int byte = 10 + g;
          if (g < G.nlev) {
            if (byte < 16) w1 |= (uint64_t)wd[g] << (8 * (byte - 8));
            else w2 |= (uint64_t)wd[g] << (8 * (byte - 16));
          }
        }
        hp[1] = w1;
        if (G.hdr_bytes > 16) hp[2] = w2;
      }
      uint32_t* pw = (uint32_t*)(slot + G.hdr_bytes);
      for (uint32_t k = t; k < nwords; k += NT) pw[k] = words[k];
      rec_bytes = (uint32_t)G.hdr_bytes + 4u * nwords;
      T.sync();
      if (t == 0) stt(T.yb, zero_off, 0.0);     // the words may have reached the zero cell
      T.sync();
      recompose_t<W, NS, true>(tb, T, R, rm, keep, [&](int s) { return __dmul_rn(Dk, rint(__dmul_rn(dm[s], inv))); });
      load_ft(true);                                        // ft = fhat + rhat
      ft_ready = true;
    }
  }

  // ---- Newton projection ----
  double lam[4] = {0.0, 0.0, 0.0, 0.0};
  int flags = 0, total_upd = 0;
  if (!raw) {
    if (!ft_ready) load_ft(false);
    const bool paper = a.fallback == HCZ_FALLBACK_PAPER;
    double l0[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.lam0) {
#pragma unroll
      for (int k = 0; k < 4; ++k) l0[k] = a.lam0[h * 4 + k];
    } else if (a.analytic) {
      // the analytic start (A A^T)^-1 (A ft - b): one Newton step at lam = 0 with every cell
      // active; a failed factorisation leaves a non-finite start, which is rejected
      double v[16], sc[4], hs[9], g[4];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = 0.0;
      newton_pass_t<W, UVOL, false, false>(G, T, S, l0, v, sc, hs);
      constexpr int dst[9] = {5, 6, 7, 8, 10, 11, 12, 13, 14};
#pragma unroll
      for (int k = 0; k < 9; ++k) v[dst[k]] = hs[k];
      v[9] = v[8];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = v[k] - b[k];
      if (!chol4(v, g, l0)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) l0[k] = NAN;
      }
    }
    const bool have_l0 = a.lam0 != nullptr || a.analytic;
    bool rejected = false;
    const int st = a.no_positivity
                       ? newton_t<W, UVOL, false>(G, T, S, b, lam, a.newton_s, a.max_iter, paper ? 0.01 : 1.0,
                                                  a.max_iter2, !paper, &total_upd, have_l0, l0, &rejected)
                       : newton_t<W, UVOL, true>(G, T, S, b, lam, a.newton_s, a.max_iter, paper ? 0.01 : 1.0,
                                                 a.max_iter2, !paper, &total_upd, have_l0, l0, &rejected);
    if (rejected) flags |= HCZ_FLAG_WARM_REJECTED;
    if (st >= 1) flags |= HCZ_FLAG_ROUND2;
    if (st == 2) raw = true;
    if (!raw && a.no_positivity) flags |= HCZ_FLAG_NOCLIP;
  }

  uint64_t size = 0;
  if (raw) {
    flags = (flags & (HCZ_FLAG_ROUND2 | HCZ_FLAG_WARM_REJECTED)) | HCZ_FLAG_RAW;
    TIn* dst = (TIn*)(a.slots + h * a.slot_stride);
    for_tasks<W>(
        G, S, [](int) {}, [&](int i, int j, uint32_t) { dst[j * G.n_par + i] = f[(long long)j * a.rs + i]; },
        [](int) {});
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
  }
  if (a.t_done) {
    __syncthreads();            // the histogram is done when every wave of its team is
    if (t == 0) a.t_done[h] = wall_clock64();
  }
}

template <typename TIn, bool UVOL, int W>
__global__ __launch_bounds__(64 * W, 2) void k_residual_t(GridDev G, ResidualArgs a) {
  extern __shared__ double smem[];
  Team<W> T = setup_team<W>(G, smem);
  T.sync();
  residual_t_hist<TIn, UVOL, W>(G, a, T, (long long)blockIdx.x);
}

// ---- launcher ---------------------------------------------------------------------------

bool team_path(const GridDev& G, int W) {
  const int k = W == 2 ? 0 : 1;
  return (W == 2 || W == 4) && G.tnslots[k] > 0 && G.tnslots[k] <= (W == 2 ? team_slots<2>() : team_slots<4>());
}

template <int W>
static hipError_t launch_t(const GridDev& G, const ResidualArgs& a, hipStream_t st) {
  dim3 grid((unsigned)a.H), block(64 * W);
  const size_t lds = lds_bytes_t<W>(G);
#define HCZ_RT(T, U) hipLaunchKernelGGL((k_residual_t<T, U, W>), grid, block, lds, st, G, a)
  if (a.dtype == HCZ_F32) {
    if (G.uniform_vol) HCZ_RT(float, true);
    else HCZ_RT(float, false);
  } else {
    if (G.uniform_vol) HCZ_RT(double, true);
    else HCZ_RT(double, false);
  }
#undef HCZ_RT
  return hipGetLastError();
}

hipError_t launch_residual_t(const GridDev& G, const ResidualArgs& a, int W, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  if (!team_path(G, W)) return hipErrorInvalidValue;
  return W == 2 ? launch_t<2>(G, a, st) : launch_t<4>(G, a, st);
}

}  // namespace hcz
