// Wave-per-histogram residual coding, Newton projection and decompression (Section III
// Stages 4-5 and decompression), for grids whose nodes fit in kWaveSlots slots of 64.
//
// One 64-lane wave owns one histogram; a workgroup of four waves shares the per-grid
// tables in LDS, so after the first barrier no block-wide synchronisation is needed.
// Each wave keeps its histogram in an FP64 LDS buffer in natural order
// (e = j * n_par + i) followed by one zero cell.  Two lane layouts use it:
//  - node slots (decomposition, recomposition, packing): per slot, lane l holds one
//    node of the multilevel decomposition, its residual and coefficient in registers
//    and its interpolation corners as byte offsets into the buffer; padding lanes read
//    and write the zero cell, so no lane ever branches on its own node;
//  - columns (loading, moments, Newton, output): lane l walks grid column i = l (and
//    l + 64) down the rows, so a_i stays in a register, c_j is one broadcast read per
//    row, and the sums over a column are combined with powers of a_i only once.
// A wave's LDS operations complete in order, so a compiler fence between coefficient
// groups is all the ordering needed.  Reductions are DPP butterflies with the result
// read from lane 63, so every lane sees the same bits and runs repeat bitwise.
#include "wave_ops.h"

namespace hcz {

constexpr int kWPB = 4;   // waves (histograms) per workgroup

// ---- tables and layout -----------------------------------------------------------------

// Dynamic LDS, in doubles: s_w [64] interpolation weights, s_cc [2 kMaxDim] (c_j, c_j^2)
// pairs, then the slot entries as nslots * 64 uint2 (words 0-1), nslots * 64 uint32
// (word 2) and nslots * 64 uint16 packing ranks, then one (N + 1)-double buffer per wave.
constexpr int kLdsTables = 64 + 2 * kMaxDim;
__host__ __device__ __forceinline__ size_t lds_meta_doubles(int nslots) { return (size_t)nslots * 112; }
__host__ __device__ __forceinline__ size_t lds_bytes_w(const GridDev& G) {
  return (kLdsTables + lds_meta_doubles(G.nslots) + (size_t)(G.N + 1) * kWPB) * sizeof(double);
}

struct WaveLds {
  double* s_w;
  double* s_cc;
  const uint2* m01;
  const uint32_t* m2;
  const uint16_t* rk;
  char* yb;          // this wave's buffer (byte addressed)
};

__device__ __forceinline__ WaveLds setup_lds(const GridDev& G, double* smem, int wv) {
  WaveLds L;
  L.s_w = smem;
  L.s_cc = smem + 64;
  uint2* m01 = (uint2*)(smem + kLdsTables);
  uint32_t* m2 = (uint32_t*)(m01 + (size_t)G.nslots * 64);
  uint16_t* rk = (uint16_t*)(m2 + (size_t)G.nslots * 64);
  const int t = threadIdx.x;
  for (int k = t; k < G.nw; k += 256) L.s_w[k] = G.wtab[k];
  for (int k = t; k < G.n_perp; k += 256) {
    const double c = G.cperp[k];
    L.s_cc[2 * k] = c;
    L.s_cc[2 * k + 1] = c * c;
  }
  for (int k = t; k < G.nslots * 64; k += 256) {
    m01[k] = make_uint2(G.slot_meta[3 * k], G.slot_meta[3 * k + 1]);
    m2[k] = G.slot_meta[3 * k + 2];
    rk[k] = G.slot_rank[k];
  }
  L.m01 = m01;
  L.m2 = m2;
  L.rk = rk;
  double* y = smem + kLdsTables + lds_meta_doubles(G.nslots) + (size_t)(G.N + 1) * wv;
  if (t < 256) y[G.N] = 0.0;      // every wave's zero cell (lane 0 of each wave)
  L.yb = (char*)y;
  return L;
}

// A wave's copy of the slot entries in registers (read once from LDS).
template <int NS>
struct SlotRegs {
  uint2 m[NS];
  uint32_t m2[NS];
};
// Entry words hidden from loop-invariant code motion: otherwise every slot's decoded
// addresses are hoisted out of the bisection loop and the registers spill.
__device__ __forceinline__ uint2 opaque2(uint2& m) {
  asm volatile("" : "+v"(m.x), "+v"(m.y));     // in place: no copy of the register
  return m;
}
__device__ __forceinline__ uint32_t opaque1(uint32_t& m) {
  asm volatile("" : "+v"(m));
  return m;
}
template <class SH>
__device__ __forceinline__ void load_slot_regs(const GridDev& G, const WaveLds& L, SlotRegs<SH::NS>& R) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s = 0; s < SH::NS; ++s) {
    R.m[s] = make_uint2(0u, 0u);
    R.m2[s] = 0u;
    if (SH::fixed || s < G.nslots) {
      R.m[s] = L.m01[s * 64 + lane];
      R.m2[s] = L.m2[s * 64 + lane];
    }
  }
}

__device__ __forceinline__ double ldy(const char* yb, uint32_t off) { return *(const double*)(yb + off); }
__device__ __forceinline__ void sty(char* yb, uint32_t off, double v) { *(double*)(yb + off) = v; }

// Interpolated value of a node from its corners, in the fixed unfused order of the coder
// (two-corner form unless FOUR).
template <bool FOUR, bool HALF = false>
__device__ __forceinline__ double predict_w(const WaveLds& L, uint2 m, uint32_t m2) {
  const double y00 = ldy(L.yb, m.x >> 16), y10 = ldy(L.yb, m.y & 0xffffu);
  const double s = HALF ? 0.5 : L.s_w[(m2 >> 16) & 63u];
  const double p0 = __dadd_rn(y00, __dmul_rn(s, __dsub_rn(y10, y00)));
  if (!FOUR) return p0;
  const double y01 = ldy(L.yb, m.y >> 16), y11 = ldy(L.yb, m2 & 0xffffu);
  const double t = HALF ? 0.5 : L.s_w[(m2 >> 22) & 63u];
  const double p1 = __dadd_rn(y01, __dmul_rn(s, __dsub_rn(y11, y01)));
  return __dadd_rn(p0, __dmul_rn(t, __dsub_rn(p1, p0)));
}

__device__ __forceinline__ bool bit(uint32_t mask, int s) { return (mask >> s) & 1u; }

// The per-slot masks, kept as plain scalars: without the opaque copy the compiler hoists
// every slot's test out of the bisection loop as a lane mask and spills them.
struct SlotMasks {
  uint32_t bil, keep, sync;
};
__device__ __forceinline__ SlotMasks slot_masks(const GridDev& G) {
  SlotMasks m{G.slot_bil, G.slot_keep, G.slot_sync};
  asm volatile("" : "+s"(m.bil), "+s"(m.keep), "+s"(m.sync));
  return m;
}

// Slot structure of a grid: read from the plan at run time (any grid), or fixed at
// compile time for a grid whose tables match, which lets every per-slot choice fold away
// and batches of slots issue their LDS reads together.
struct ShapeDyn {
  static constexpr bool fixed = false;
  static constexpr int NS = kWaveSlots, NCO = 0, NP = 0, NQ = 0;
  static constexpr uint32_t BIL = 0, SYNC = 0, KEEP = 0, HALF = 0;
};
// 39 x 39 (the velocity grid of the paper's data): slot 0 holds groups 0-3, slots 1-2
// group 4, slots 3-7 group 5 and slots 8-25 the finest group.
struct Shape39 {
  static constexpr bool fixed = true;
  static constexpr int NS = 26, NCO = 4, NP = 39, NQ = 39;
  static constexpr uint32_t BIL = 0x3f800c7u, SYNC = 0x2000085u, KEEP = 0xffu, HALF = 0x3f7ffb8u;
};
template <class SH>
__host__ __device__ constexpr bool shape_matches(const GridDev& G) {
  return !SH::fixed || (G.nslots == SH::NS && G.ncoarse == SH::NCO && G.n_par == SH::NP && G.n_perp == SH::NQ &&
                        G.slot_bil == SH::BIL && G.slot_sync == SH::SYNC && G.slot_keep == SH::KEEP &&
                        G.slot_half == SH::HALF);
}
template <class SH> __device__ __forceinline__ int nslots_of(const GridDev& G) { return SH::fixed ? SH::NS : G.nslots; }
template <class SH> __device__ __forceinline__ int ncoarse_of(const GridDev& G) { return SH::fixed ? SH::NCO : G.ncoarse; }
template <class SH> __device__ __forceinline__ bool bil_of(const GridDev& G, int s) {
  return SH::fixed ? bit(SH::BIL, s) : bit(G.slot_bil, s);
}
template <class SH> __device__ __forceinline__ bool sync_of(const GridDev& G, int s) {
  return SH::fixed ? bit(SH::SYNC, s) : bit(G.slot_sync, s);
}
// Coefficient group of slot s >= 1: the coarse groups of slot 0, then one more per group
// end before s.
template <class SH> __device__ __forceinline__ int group_of_slot(const GridDev& G, int s) {
  const uint32_t sync = SH::fixed ? SH::SYNC : G.slot_sync;
  return ncoarse_of<SH>(G) + __popc(sync & ((1u << s) - 1u) & ~1u);
}
// x[g] for a group index known to be below kMaxLev (unrolled select, no indexed registers)
__device__ __forceinline__ uint32_t pick(const uint32_t (&x)[kMaxLev], int g) {
  uint32_t r = 0u;
#pragma unroll
  for (int q = 0; q < kMaxLev; ++q) r = g == q ? x[q] : r;
  return r;
}

// Prediction for slot s of a fixed shape: the slot's form and (when every weight is 1/2)
// its weights are compile-time constants after unrolling.
template <class SH>
__device__ __forceinline__ double predict_s(const WaveLds& L, int s, uint2 m, uint32_t m2) {
  if (bit(SH::BIL, s)) return bit(SH::HALF, s) ? predict_w<true, true>(L, m, m2) : predict_w<true>(L, m, m2);
  return bit(SH::HALF, s) ? predict_w<false, true>(L, m, m2) : predict_w<false>(L, m, m2);
}

constexpr int kBatch = 4;   // slots whose LDS reads issue together (fixed shapes)

// End of the batch that starts at slot s: at most kBatch slots, closed by a group end.
template <class SH>
constexpr int batch_end(int s) {
  int e = s;
  while (e < SH::NS && e - s < kBatch) {
    ++e;
    if ((SH::SYNC >> (e - 1)) & 1u) break;
  }
  return e;
}

// Slots [S, E) of one group: every entry and corner read first, then values, stores
// and errors.  Nothing in the batch reads what the batch writes.
template <class SH, int S, int E, bool STORE_ALL, typename DQ>
__device__ __forceinline__ void batch_fixed(const WaveLds& L, SlotRegs<SH::NS>& R, const double (&rm)[SH::NS],
                                            DQ& dqf, double& acc) {
  constexpr int B = E - S;
  double v[B], r[B];
  uint2 m[B];
#pragma unroll
  for (int k = 0; k < B; ++k) {
    m[k] = opaque2(R.m[S + k]);
    const uint32_t m2 = opaque1(R.m2[S + k]);
    v[k] = __dadd_rn(dqf(S + k), predict_s<SH>(L, S + k, m[k], m2));
    // a slot no later group reads keeps its residual in the buffer while the bisection
    // runs, which saves its register copy
    r[k] = bit(SH::KEEP, S + k) ? rm[S + k] : ldy(L.yb, m[k].x & 0xffffu);
  }
#pragma unroll
  for (int k = 0; k < B; ++k) {
    if (STORE_ALL || bit(SH::KEEP, S + k)) sty(L.yb, m[k].x & 0xffffu, v[k]);
    const double e = r[k] - v[k];
    acc = fma(e, e, acc);
  }
}

template <class SH, int S, bool STORE_ALL, typename DQ>
__device__ __forceinline__ void slots_fixed(const WaveLds& L, SlotRegs<SH::NS>& R, const double (&rm)[SH::NS],
                                            DQ& dqf, double& acc) {
  if constexpr (S < SH::NS) {
    constexpr int E = batch_end<SH>(S);
    batch_fixed<SH, S, E, STORE_ALL>(L, R, rm, dqf, acc);
    if constexpr (((SH::SYNC >> (E - 1)) & 1u) != 0) wave_sync();
    slots_fixed<SH, E, STORE_ALL>(L, R, rm, dqf, acc);
  }
}

// Recompose every node with quantised values dq(s) into the buffer (slots of the finest
// group only when STORE_ALL) and return sum (rm - y)^2 over the histogram.  DQ(s) gives
// the lane's quantised coefficient of slot s.
template <class SH, bool STORE_ALL, typename DQ>
__device__ __forceinline__ double recompose_w(const GridDev& G, const WaveLds& L, SlotRegs<SH::NS>& R,
                                              const double (&rm)[SH::NS], DQ dqf) {
  constexpr int NS = SH::NS;
  const SlotMasks sm = slot_masks(G);
  double acc = 0.0;
  {
    const uint2 m = opaque2(R.m[0]);
    const uint32_t m2 = opaque1(R.m2[0]);
    const int g0 = (int)(m2 >> 28);
    const double dq = dqf(0);
    for (int g = 0; g < ncoarse_of<SH>(G); ++g) {
      if (g0 == g) {
        // the coarsest values are dq itself: +0 for a quantised zero as in the oracle
        // (elsewhere dq + P already has the bits of +0 + P: P is never -0)
        const double v = g == 0 ? __dadd_rn(dq, 0.0) : __dadd_rn(dq, predict_w<true>(L, m, m2));
        sty(L.yb, m.x & 0xffffu, v);
        const double e = rm[0] - v;
        acc = fma(e, e, acc);
      }
      wave_sync();
    }
  }
  if constexpr (SH::fixed) {
    slots_fixed<SH, 1, STORE_ALL>(L, R, rm, dqf, acc);
  } else {
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      if (s < G.nslots) {
        const uint2 m = opaque2(R.m[s]);
        const uint32_t m2 = opaque1(R.m2[s]);
        const double dq = dqf(s);
        const double v = __dadd_rn(dq, bit(sm.bil, s) ? predict_w<true>(L, m, m2) : predict_w<false>(L, m, m2));
        if (STORE_ALL || bit(sm.keep, s)) sty(L.yb, m.x & 0xffffu, v);
        const double e = rm[s] - v;
        acc = fma(e, e, acc);
        if (bit(sm.sync, s)) wave_sync();
      }
    }
  }
  return wsum(acc);
}

// ---- column walks ---------------------------------------------------------------------

constexpr int kRowChunk = 40;   // rows whose global loads a lane issues together

// As for_columns, with load(i, j) issued for a chunk of rows before body(i, j, off, v)
// runs on them, so a column costs one memory round trip per chunk.
template <typename BEGIN, typename LOAD, typename BODY, typename FOLD>
__device__ __forceinline__ void for_columns_pre(const GridDev& G, BEGIN begin, LOAD load, BODY body, FOLD fold) {
  const int lane = threadIdx.x & 63;
  const uint32_t rowb = (uint32_t)G.n_par * 8u;
  using V = decltype(load(0, 0));
  for (int i = lane; i < G.n_par; i += 64) {
    begin(i);
    uint32_t off = (uint32_t)i * 8u;
    for (int j0 = 0; j0 < G.n_perp; j0 += kRowChunk) {
      V v[kRowChunk];
#pragma unroll
      for (int k = 0; k < kRowChunk; ++k)
        if (j0 + k < G.n_perp) v[k] = load(i, j0 + k);
#pragma unroll
      for (int k = 0; k < kRowChunk; ++k)
        if (j0 + k < G.n_perp) {
          body(i, j0 + k, off, v[k]);
          off += rowb;
        }
    }
    fold(i);
  }
}

// Lane l visits columns i = l, l + 64 (< n_par): begin(i), then body(i, j, off) for every
// row j, off the byte offset of (j, i) in the wave buffer, then fold(i).
template <typename BEGIN, typename BODY, typename FOLD>
__device__ __forceinline__ void for_columns(const GridDev& G, BEGIN begin, BODY body, FOLD fold) {
  const int lane = threadIdx.x & 63;
  const uint32_t rowb = (uint32_t)G.n_par * 8u;
  for (int i = lane; i < G.n_par; i += 64) {
    begin(i);
    uint32_t off = (uint32_t)i * 8u;
#pragma unroll 4
    for (int j = 0; j < G.n_perp; ++j) {
      body(i, j, off);
      off += rowb;
    }
    fold(i);
  }
}

// One Newton pass at lam (Section III Stage 5): v[0..3] = A x, v[4] = sum |A_1| x and,
// when THETA, v[15] = ||x - ft||^2, with x = max(0, ft - A^T lam) and ft in the wave
// buffer; hs the Hessian A diag(x > 0) A^T (upper triangle, row-major, without the
// duplicate (1,1) = (0,3) entry), all reduced together by one transposed butterfly.  Per
// column the row sums of w x, c w x and, on active
// cells, w^2, w^2 c, w^2 c^2 come first and are then weighted by the column's powers of
// a.  The correction per cell is vol * ((lam3 a + lam1) a + lam0 + lam2 c), one fixed
// order for compression and decompression.  KL: the KL reading, x = max(ft, 0) exp(-corr)
// with Hessian weights x (A diag(x) A^T) and v[15] = sum_j x_j for its dual.
template <class SH, bool UVOL, bool THETA, bool POS, bool KL = false>
__device__ __forceinline__ void newton_pass_w(const GridDev& G, const WaveLds& L, const double (&lam)[4],
                                              double (&v)[16], double (&sc)[4], double (&hs)[9]) {
  static_assert(!KL || POS, "the KL reading's x is never negative");
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0, v4 = 0.0, v15 = 0.0, c0 = 0.0, c2 = 0.0, c3 = 0.0;
  double hh[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) hh[k] = 0.0;
  double sx, sxc, sxa, sxca, h0, hc, hcc, s2;
  double pa = 0.0;
  auto begin = [&](int i) {
    const double a = G.apar[i];
    pa = fma(fma(lam[3], a, lam[1]), a, lam[0]);
    sx = sxc = sxa = sxca = h0 = hc = hcc = s2 = 0.0;
  };
  auto body = [&](int i, int j, uint32_t off) {
    const double c = L.s_cc[2 * j], c2 = L.s_cc[2 * j + 1];
    const double w = UVOL ? G.vol0 : G.vol[j * G.n_par + i];
    const double ft = ldy(L.yb, off);
    const double corr = w * fma(lam[2], c, pa);
    const double y = ft - corr;
    const double x = KL ? (ft > 0.0 ? ft * exp(-corr) : 0.0) : (POS ? fmax(0.0, y) : y);
    const double wx = UVOL ? x : w * x;
    sx += wx;
    sxc = fma(c, wx, sxc);
    if (!POS) {                      // the stopping rule's scales use |x| when x may be negative
      const double wxa = fabs(wx);
      sxa += wxa;
      sxca = fma(c, wxa, sxca);
    }
    // Hessian terms on active cells, as a 0/1 weight (exact: products with 0 or 1); in
    // the KL reading the weight is x itself
    const double act = KL ? x : ((!POS || x > 0.0) ? 1.0 : 0.0);
    const double w2 = UVOL ? act : act * (w * w);
    h0 += w2;
    hc = fma(w2, c, hc);
    hcc = fma(w2, c2, hcc);
    if (THETA) {
      if (KL) {
        s2 += x;
      } else {
        const double dx = x - ft;
        s2 = fma(dx, dx, s2);
      }
    }
  };
  auto fold = [&](int i) {
    const double a = G.apar[i], a2 = a * a;
    v0 += sx;
    v1 = fma(a, sx, v1);
    v2 += sxc;
    v3 = fma(a2, sx, v3);
    v4 = fma(fabs(a), POS ? sx : sxa, v4);
    v15 += s2;
    if (!POS) {
      c0 += sxa;
      c2 += sxca;
      c3 = fma(a2, sxa, c3);
    }
    hh[0] += h0;
    hh[1] = fma(a, h0, hh[1]);
    hh[2] += hc;
    hh[3] = fma(a2, h0, hh[3]);
    hh[4] = fma(a, hc, hh[4]);
    hh[5] = fma(a2 * a, h0, hh[5]);
    hh[6] += hcc;
    hh[7] = fma(a2, hc, hh[7]);
    hh[8] = fma(a2 * a2, h0, hh[8]);
  };
  if constexpr (SH::fixed && SH::NP <= 64 && SH::NQ <= 64) {
    // an 8 x 8 grid of lane blocks: lane (bx, by) = (l % 8, l / 8) takes columns
    // BX bx .. BX bx + BX - 1 and rows BY by .. BY by + BY - 1 (39 x 39: 5 x 5 cells, 25
    // per lane instead of a 39-row column on 39 of the 64 lanes), folding per column
    constexpr int BX = (SH::NP + 7) / 8, BY = (SH::NQ + 7) / 8;
    const int lane = threadIdx.x & 63;
    const int i0 = (lane & 7) * BX, j0 = (lane >> 3) * BY;
#pragma unroll
    for (int ci = 0; ci < BX; ++ci) {
      const int i = i0 + ci;
      if (i < SH::NP) {
        begin(i);
#pragma unroll
        for (int cj = 0; cj < BY; ++cj) {
          const int j = j0 + cj;
          if (j < SH::NQ) body(i, j, (uint32_t)(j * SH::NP + i) * 8u);
        }
        fold(i);
      }
    }
  } else {
    for_columns(G, begin, body, fold);
  }
  const double s2v = UVOL ? G.vol0 * G.vol0 : 1.0;
  if constexpr (POS) {
    const double r[16] = {v0, v1, v2, v3, v4, v15, hh[0], hh[1], hh[2], hh[3], hh[4], hh[5], hh[6], hh[7], hh[8], 0.0};
    double o[16];
    wsum16(r, o);
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] = o[k];
    v[15] = THETA ? o[5] : 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) hs[k] = o[6 + k] * s2v;
  } else {
    v[0] = wsum(v0);
    v[1] = wsum(v1);
    v[2] = wsum(v2);
    v[3] = wsum(v3);
    v[4] = wsum(v4);
    v[15] = THETA ? wsum(v15) : 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) hs[k] = wsum(hh[k]) * s2v;
  }
  if (UVOL) {
#pragma unroll
    for (int k = 0; k < 5; ++k) v[k] *= G.vol0;
  }
  // scales sum_j |A_kj| x_j of the stopping rule (every A entry but k = 1 is >= 0)
  if (POS) {
    sc[0] = v[0];
    sc[1] = v[4];
    sc[2] = v[2];
    sc[3] = v[3];
  } else {
    const double s1 = UVOL ? G.vol0 : 1.0;
    sc[0] = wsum(c0) * s1;
    sc[1] = v[4];
    sc[2] = wsum(c2) * s1;
    sc[3] = wsum(c3) * s1;
  }
}

// The pass's reduced Hessian into v[5..14].
__device__ __forceinline__ void hess_fill(const double (&hs)[9], double (&v)[16]) {
  constexpr int dst[9] = {5, 6, 7, 8, 10, 11, 12, 13, 14};
#pragma unroll
  for (int k = 0; k < 9; ++k) v[dst[k]] = hs[k];
  v[9] = v[8];
}

// Both Newton rounds (newton_core) on the wave's buffer.
template <class SH, bool UVOL, bool POS, bool KL = false>
__device__ __forceinline__ int newton_w(const GridDev& G, const WaveLds& L, const double (&b)[4], double (&lam)[4],
                                        double s1, int max1, double s2, int max2, bool armijo2, int* upd,
                                        bool have_init, const double (&lam_init)[4], bool* rejected) {
  double hh[9];
  auto pass = [&](bool theta, const double (&cand)[4], double (&v)[16], double (&sc)[4]) {
    if (theta) newton_pass_w<SH, UVOL, true, POS, KL>(G, L, cand, v, sc, hh);
    else newton_pass_w<SH, UVOL, false, POS, KL>(G, L, cand, v, sc, hh);
  };
  auto hess = [&](double (&v)[16]) { hess_fill(hh, v); };
  return newton_core<decltype(pass), decltype(hess), KL>(pass, hess, b, lam, s1, max1, s2, max2, armijo2, upd,
                                                        have_init, lam_init, rejected);
}

// ---- compression ------------------------------------------------------------------------

// This lane's cells of one histogram, loaded ahead of their use (fixed shapes): an 8 x 8
// grid of lane blocks, lane (bx, by) = (l % 8, l / 8) holding columns BX bx .. + BX - 1
// and rows BY by .. + BY - 1 (39 x 39: 5 x 5 cells), cell (ci, cj) at index cj BX + ci.
template <class SH>
struct LaneBlock {
  static constexpr int BX = SH::fixed ? (SH::NP + 7) / 8 : 1, BY = SH::fixed ? (SH::NQ + 7) / 8 : 1;
};
template <typename TIn, class SH>
struct PreRows {
  TIn f[LaneBlock<SH>::BX * LaneBlock<SH>::BY];
  float h[LaneBlock<SH>::BX * LaneBlock<SH>::BY];
};
// Every lane loads every cell of its block, clamped to a valid histogram, column and row
// (the extra values are unused).
template <typename TIn, class SH>
__device__ __forceinline__ void pre_load(PreRows<TIn, SH>& P, const GridDev& G, const ResidualArgs& a, long long h) {
  constexpr int BX = LaneBlock<SH>::BX, BY = LaneBlock<SH>::BY;
  const int lane = threadIdx.x & 63;
  const int i0 = (lane & 7) * BX, j0 = (lane >> 3) * BY;
  const long long hc = min(h, a.H - 1);
  const TIn* f = (const TIn*)a.hist + hc * a.hs;
#pragma unroll
  for (int cj = 0; cj < BY; ++cj)
#pragma unroll
    for (int ci = 0; ci < BX; ++ci)
      P.f[cj * BX + ci] = f[(long long)min(j0 + cj, SH::NQ - 1) * a.rs + min(i0 + ci, SH::NP - 1)];
  if (a.fhat) {
    const float* fhp = a.fhat + hc * (long long)G.N;
#pragma unroll
    for (int cj = 0; cj < BY; ++cj)
#pragma unroll
      for (int ci = 0; ci < BX; ++ci)
        P.h[cj * BX + ci] = fhp[min(j0 + cj, SH::NQ - 1) * SH::NP + min(i0 + ci, SH::NP - 1)];
  } else {
#pragma unroll
    for (int c = 0; c < BX * BY; ++c) P.h[c] = 0.0f;
  }
}

// Histogram h (< a.H) on this wave, with the grid's tables staged in LDS and, for a fixed
// shape, the lane's block of cells already loaded into P.  KL: the KL reading of Stage 5
// first, kept where it keeps the bound, the L2 projection elsewhere.
template <typename TIn, bool UVOL, class SH, bool KL = false>
__device__ __forceinline__ void residual_w_hist(const GridDev& G, const ResidualArgs& a, const WaveLds& L,
                                                long long h, const PreRows<TIn, SH>& P) {
  constexpr int NS = SH::NS;
  const int N = G.N;
  const int lane = threadIdx.x & 63;
  const TIn* f = (const TIn*)a.hist + h * a.hs;
  const float* fhp = a.fhat ? a.fhat + h * (long long)N : nullptr;
  uint32_t* words = (uint32_t*)L.yb;     // payload words borrow the buffer before the last recomposition

  // ---- column pass: residual into the buffer, moments, norms, range ----
  dd ff{0.0, 0.0};
  double rr = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0, m3 = 0.0, fmx = -INFINITY, fmnn = -INFINITY;
  bool bad = false;
  {
    double sf = 0.0, sfc = 0.0;
    struct FH {
      TIn f;
      float h;
    };
    auto load = [&](int i, int j) {
      return FH{f[(long long)j * a.rs + i], fhp ? fhp[j * G.n_par + i] : 0.0f};
    };
    auto body = [&](int i, int j, uint32_t off, FH ld) {
      const double fv = (double)ld.f;
      const double hv = (double)ld.h;
      const double r = fv - hv;
      sty(L.yb, off, r);
      // ||f||^2 in double-double: the products are rounded as in a plain FP64 sum of
      // squares, the sum is carried with TwoSum error terms
      const double p = fv * fv;
      const double hi = ff.hi + p;
      const double bb = hi - ff.hi;
      ff.lo += (ff.hi - (hi - bb)) + (p - bb);
      ff.hi = hi;
      rr = fma(r, r, rr);
      const double w = UVOL ? fv : G.vol[j * G.n_par + i] * fv;
      sf += w;
      sfc = fma(L.s_cc[2 * j], w, sfc);
      bad |= !isfinite(fv);
      fmx = fmax(fmx, fv);
      fmnn = fmax(fmnn, -fv);
    };
    auto fold = [&](int i) {
      const double av = G.apar[i];
      m0 += sf;
      m1 = fma(av, sf, m1);
      m2 += sfc;
      m3 = fma(av * av, sf, m3);
    };
    if constexpr (SH::fixed) {
      // the lane's block, folding per column
      constexpr int BX = LaneBlock<SH>::BX, BY = LaneBlock<SH>::BY;
      static_assert(8 * BX >= SH::NP && 8 * BY >= SH::NQ, "the lane blocks cover the grid");
      // the block origin from a lane index the compiler cannot see through, so that it is
      // not kept live until the Newton pass forms the same one
      int lb = lane;
      asm volatile("" : "+v"(lb));
      const int i0 = (lb & 7) * BX, j0 = (lb >> 3) * BY;
#pragma unroll
      for (int ci = 0; ci < BX; ++ci) {
        const int i = i0 + ci;
        if (i < SH::NP) {
          sf = sfc = 0.0;
#pragma unroll
          for (int cj = 0; cj < BY; ++cj) {
            const int j = j0 + cj;
            if (j < SH::NQ) body(i, j, (uint32_t)(j * SH::NP + i) * 8u, FH{P.f[cj * BX + ci], P.h[cj * BX + ci]});
          }
          fold(i);
        }
      }
    } else {
      for_columns_pre(G, [&](int) { sf = sfc = 0.0; }, load, body, fold);
    }
  }
  {
    const double hi = ff.hi + ff.lo;
    ff = dd{hi, ff.lo - (hi - ff.hi)};
  }
  ff = wdd(ff);
  rr = wsum(rr);
  double b[4] = {wsum(m0), wsum(m1), wsum(m2), wsum(m3)};
  if (UVOL) {
#pragma unroll
    for (int k = 0; k < 4; ++k) b[k] *= G.vol0;
  }
  fmx = wmax(fmx);
  fmnn = wmax(fmnn);
  bad = __ballot(bad) != 0;
  const double tau = a.tau_hist ? a.tau_hist[h] : a.tau;
  const double tau_h = (a.tau_mode == HCZ_TAU_NRMSE) ? (tau * G.sqrtN) * (fmx - (-fmnn))
                                                     : tau * sqrt(ff.hi + ff.lo);
  const double thr = kSelMargin * tau_h;
  const double thr2 = thr * thr;
  bool raw = bad || !(b[0] > 0.0) || !(tau >= 0.0 && tau <= DBL_MAX);
  const bool coded = rr > thr2;
  if (coded && !(tau_h > 0.0)) raw = true;
  wave_sync();

  int kst = 0xff;
  uint32_t rec_bytes = 0;
  // ft = fhat + rhat (rhat = 0 when not coded), written over the buffer in natural order
  auto load_ft = [&](bool with_r) {
    for_columns_pre(
        G, [](int) {}, [&](int i, int j) { return fhp ? fhp[j * G.n_par + i] : 0.0f; },
        [&](int, int, uint32_t off, float h) {
          const double hv = (double)h;
          sty(L.yb, off, with_r ? hv + ldy(L.yb, off) : hv);
        },
        [](int) {});
    wave_sync();
  };
  bool ft_ready = false;
  if (coded && !raw) {
    // coefficients: d = r - P(r) over the residual itself (no node is rewritten here)
    SlotRegs<NS> R;
    load_slot_regs<SH>(G, L, R);
    double dm[NS], rm[NS];
    double mx = 0.0;
    {
      const uint2 m = R.m[0];
      const uint32_t mm2 = R.m2[0];
      rm[0] = ldy(L.yb, m.x & 0xffffu);
      dm[0] = (mm2 >> 28) == 0 ? rm[0] : __dsub_rn(rm[0], predict_w<true>(L, m, mm2));
      mx = fabs(dm[0]);
    }
#pragma unroll
    for (int s = 1; s < NS; ++s) {
      dm[s] = 0.0;
      rm[s] = 0.0;
      if (s < nslots_of<SH>(G)) {
        const uint2 m = R.m[s];
        const uint32_t mm2 = R.m2[s];
        rm[s] = ldy(L.yb, m.x & 0xffffu);
        if constexpr (SH::fixed) dm[s] = __dsub_rn(rm[s], predict_s<SH>(L, s, m, mm2));
        else dm[s] = __dsub_rn(rm[s], bil_of<SH>(G, s) ? predict_w<true>(L, m, mm2) : predict_w<false>(L, m, mm2));
        mx = fmax(mx, fabs(dm[s]));
      }
    }
    mx = wmax(mx);
    wave_sync();
    const double d0 = (kLadderMargin * tau_h) / G.den;
    if (mx * (1.0 / d0) >= kQMax) raw = true;
    if (!raw) {
      // the bound search over the ladder, or the user's step (an empty search)
      LadderSearch S;
      S.init(a.ub_k, a.k_start);
      for (int t = S.next(); t >= 0; t = S.next()) {
        const double Dk = ladder(d0, t);
        const double inv = 1.0 / Dk;
        const double e2 = recompose_w<SH, false>(G, L, R, rm, [&](int s) { return __dmul_rn(Dk, rint(__dmul_rn(dm[s], inv))); });
        S.result(t, e2 <= thr2);
      }
      kst = S.lo;
      const double Dk = ladder(d0, kst);
      const double inv = 1.0 / Dk;
      // zigzag integers and per-group widths (wave-uniform, in registers); the payload
      // words borrow the buffer, which the final recomposition then fills with rhat
      auto zz = [&](double d) -> uint32_t {
        const int q = (int)rint(__dmul_rn(d, inv));
        return ((uint32_t)q << 1) ^ (uint32_t)(q >> 31);
      };
      const uint32_t zero_off = (uint32_t)N * 8u;
      uint32_t gmx[kMaxLev];
#pragma unroll
      for (int g = 0; g < kMaxLev; ++g) gmx[g] = 0u;
      const int g0 = (int)(R.m2[0] >> 28);     // slot 0 may mix groups: one maximum each
      {
        const uint32_t u0 = zz(dm[0]);
#pragma unroll
        for (int g = 0; g < kMaxLev; ++g)
          if (g < ncoarse_of<SH>(G)) gmx[g] = wumax(g0 == g ? u0 : 0u);
      }
      uint32_t cur = 0u;
#pragma unroll
      for (int s = 1; s < NS; ++s) {
        if (s < nslots_of<SH>(G)) {
          cur = max(cur, zz(dm[s]));          // padding lanes hold d = 0
          if (sync_of<SH>(G, s)) {
            const uint32_t v = wumax(cur);
            const int g = group_of_slot<SH>(G, s);
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
      uint32_t rk[NS];
#pragma unroll
      for (int s = 0; s < NS; ++s) rk[s] = s < nslots_of<SH>(G) ? (uint32_t)L.rk[s * 64 + lane] : 0u;
      for (uint32_t k = lane; k < nwords; k += 64) words[k] = 0u;
      wave_sync();
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        if (s < nslots_of<SH>(G)) {
          const uint32_t eo = R.m[s].x & 0xffffu;
          const int g = s == 0 ? g0 : group_of_slot<SH>(G, s);
          const uint32_t wdt = pick(wd, g), base = pick(bs, g);
          if (eo != zero_off && wdt != 0) {
            const uint32_t pos = base + rk[s] * wdt;
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
      for (uint32_t k = lane; k < nwords; k += 64) pw[k] = words[k];
      rec_bytes = (uint32_t)G.hdr_bytes + 4u * nwords;
      wave_sync();
      if (lane == 0) sty(L.yb, zero_off, 0.0);     // the words may have reached the zero cell
      wave_sync();
      // fhat for ft = fhat + rhat: issued before the last recomposition so that its
      // latency hides behind it (one column per lane when the grid allows)
      const bool pre = G.n_par <= 64 && G.n_perp <= kRowChunk;
      float fh[kRowChunk];
      if (pre && fhp) {
        // clamped indices keep every load in bounds and unconditional, so all issue at once
        const int ic = min(lane, G.n_par - 1);
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) fh[k] = fhp[min(k, G.n_perp - 1) * G.n_par + ic];
      } else {
#pragma unroll
        for (int k = 0; k < kRowChunk; ++k) fh[k] = 0.0f;
      }
      recompose_w<SH, true>(G, L, R, rm, [&](int s) { return __dmul_rn(Dk, rint(__dmul_rn(dm[s], inv))); });   // rhat at k*
      wave_sync();
      bool done_ft = false;
      if constexpr (SH::fixed) {
        static_assert(SH::NP <= 64 && SH::NQ <= kRowChunk, "the fixed shape's column fits one lane and one chunk");
        // the fixed shape's column: every rhat read first, then the sums stored
        if (lane < SH::NP) {
          double rh[SH::NQ];
#pragma unroll
          for (int k = 0; k < SH::NQ; ++k) rh[k] = ldy(L.yb, (uint32_t)(k * SH::NP + lane) * 8u);
#pragma unroll
          for (int k = 0; k < SH::NQ; ++k) sty(L.yb, (uint32_t)(k * SH::NP + lane) * 8u, (double)fh[k] + rh[k]);
        }
        wave_sync();
        done_ft = true;
      }
      if (done_ft) {
      } else if (pre) {
        if (lane < G.n_par) {
#pragma unroll
          for (int k = 0; k < kRowChunk; ++k) {
            if (k < G.n_perp) {
              const uint32_t off = (uint32_t)(k * G.n_par + lane) * 8u;
              sty(L.yb, off, (double)fh[k] + ldy(L.yb, off));
            }
          }
        }
        wave_sync();
      } else {
        load_ft(true);                                        // ft = fhat + rhat
      }
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
      // the analytic start (A A^T)^-1 (A ft - b): one Newton step at lam = 0 with every
      // cell active; a failed factorisation leaves a non-finite start, which is rejected
      double v[16], sc[4], hh[9], g[4];
      newton_pass_w<SH, UVOL, false, false>(G, L, l0, v, sc, hh);
      hess_fill(hh, v);
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = v[k] - b[k];
      if (!chol4(v, g, l0)) {
#pragma unroll
        for (int k = 0; k < 4; ++k) l0[k] = NAN;
      }
    }
    const bool have_l0 = a.lam0 != nullptr || a.analytic;
    bool rejected = false;
    bool kl_kept = false;
    if constexpr (KL) {
      // the KL reading first (cold, both rounds); kept only where ||f - x|| stays within
      // the selection threshold (the KL correction is not non-expansive)
      double lk[4] = {0.0, 0.0, 0.0, 0.0};
      int ku = 0;
      bool krej = false;
      const int kst = newton_w<SH, UVOL, true, true>(G, L, b, lk, a.newton_s, a.max_iter, paper ? 0.01 : 1.0,
                                                     a.max_iter2, !paper, &ku, false, lk, &krej);
      if (kst < 2) {
        double pa = 0.0, e2 = 0.0;
        for_columns(
            G,
            [&](int i) {
              const double av = G.apar[i];
              pa = fma(fma(lk[3], av, lk[1]), av, lk[0]);
            },
            [&](int i, int j, uint32_t off) {
              const double ft = ldy(L.yb, off);
              const double w = UVOL ? G.vol0 : G.vol[j * G.n_par + i];
              const double x = ft > 0.0 ? ft * exp(-(w * fma(lk[2], L.s_cc[2 * j], pa))) : 0.0;
              const double d = (double)f[(long long)j * a.rs + i] - x;
              e2 = fma(d, d, e2);
            },
            [](int) {});
        if (wsum(e2) <= thr2) {
          kl_kept = true;
          total_upd = ku;
          if (kst >= 1) flags |= HCZ_FLAG_ROUND2;
#pragma unroll
          for (int k = 0; k < 4; ++k) lam[k] = lk[k];
        }
      }
    }
    if (!kl_kept) {
      const int st = a.no_positivity
                         ? newton_w<SH, UVOL, false>(G, L, b, lam, a.newton_s, a.max_iter, paper ? 0.01 : 1.0,
                                                     a.max_iter2, !paper, &total_upd, have_l0, l0, &rejected)
                         : newton_w<SH, UVOL, true>(G, L, b, lam, a.newton_s, a.max_iter, paper ? 0.01 : 1.0,
                                                    a.max_iter2, !paper, &total_upd, have_l0, l0, &rejected);
      if (rejected) flags |= HCZ_FLAG_WARM_REJECTED;
      if (st >= 1) flags |= HCZ_FLAG_ROUND2;
      if (st == 2) raw = true;
      if (!raw && a.no_positivity) flags |= HCZ_FLAG_NOCLIP;
    }
    if (!raw && kl_kept) flags |= HCZ_FLAG_KL;
  }

  uint64_t size = 0;
  if (raw) {
    flags = (flags & (HCZ_FLAG_ROUND2 | HCZ_FLAG_WARM_REJECTED)) | HCZ_FLAG_RAW;
    TIn* dst = (TIn*)(a.slots + h * a.slot_stride);
    for_columns(
        G, [](int) {}, [&](int i, int j, uint32_t) { dst[j * G.n_par + i] = f[(long long)j * a.rs + i]; },
        [](int) {});
    size = (uint64_t)N * sizeof(TIn);
    kst = 0xff;
  } else if (coded) {
    flags |= HCZ_FLAG_CODED;
    size = rec_bytes;
  }
  if (lane == 0) {
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

// One wave per histogram.  With a fixed shape the wave's cells of the histogram are
// loaded before the workgroup stages its tables, so both latencies overlap.
template <typename TIn, bool UVOL, class SH, bool KL = false>
__global__ __launch_bounds__(256, 2) void k_residual_w(GridDev G, ResidualArgs a) {
  extern __shared__ double smem[];
  const int wv = threadIdx.x >> 6;
  const long long h = (long long)blockIdx.x * kWPB + wv;
  PreRows<TIn, SH> P;
  if constexpr (SH::fixed) pre_load(P, G, a, h);
  const WaveLds L = setup_lds(G, smem, wv);
  __syncthreads();
  if (h >= a.H) return;
  residual_w_hist<TIn, UVOL, SH, KL>(G, a, L, h, P);
}

// ---- decompression ----------------------------------------------------------------------

__device__ __forceinline__ uint32_t ld32w(const uint8_t* p) { return *(const uint32_t*)p; }

template <typename TIn, typename TOut, bool UVOL, class SH>
__global__ __launch_bounds__(256, 2) void k_decompress_w(GridDev G, DecompressArgs a) {
  constexpr int NS = SH::NS;
  extern __shared__ double smem[];
  const int N = G.N;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const WaveLds L = setup_lds(G, smem, wv);
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
    // a verbatim record holds exactly the N input values; any other size (a damaged
    // stream, or records of the other input type) decodes to NaN instead of being read
    if (a.offsets[h + 1] - a.offsets[h] != (uint64_t)N * sizeof(TIn)) {
      for (int e = lane; e < N; e += 64) out[e] = (TOut)NAN;
      return;
    }
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
    // per-group widths from the header and their bit offsets (wave-uniform)
    uint32_t wd[kMaxLev], bs[kMaxLev];
    uint32_t nb = 0;
#pragma unroll
    for (int g = 0; g < kMaxLev; ++g) {
      wd[g] = g < G.nlev ? (uint32_t)rec[10 + g] : 0u;
      bs[g] = nb;
      if (g < G.nlev) nb += (uint32_t)(G.gstart[g + 1] - G.gstart[g]) * wd[g];
    }
    // a header that does not fit its record (widths above 32 bits, or more payload than
    // the record holds) decodes to NaN rather than reading past the record
    bool corrupt = (uint64_t)G.hdr_bytes + 4ull * (((uint64_t)nb + 31u) >> 5) > a.offsets[h + 1] - a.offsets[h];
#pragma unroll
    for (int g = 0; g < kMaxLev; ++g) corrupt = corrupt || wd[g] > 32u;
    if (corrupt) {
      for (int e = lane; e < N; e += 64) out[e] = (TOut)NAN;
      return;
    }
    // the payload words, staged through the wave's buffer with whole-wave loads (at most
    // 4N bytes, below the zero cell at 8N), then read per node from LDS
    const uint8_t* payload = rec + G.hdr_bytes;
    const uint32_t nwords = (nb + 31u) >> 5;
    uint32_t* pw = (uint32_t*)L.yb;
    for (uint32_t k = lane; k < nwords; k += 64) pw[k] = ld32w(payload + 4 * k);
    wave_sync();
    const uint32_t zero_off = (uint32_t)N * 8u;
    SlotRegs<NS> R;
    load_slot_regs<SH>(G, L, R);
    double dq[NS], rm[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      dq[s] = 0.0;
      rm[s] = 0.0;
      if (s < nslots_of<SH>(G)) {
        const uint32_t eo = R.m[s].x & 0xffffu;
        const int g = s == 0 ? (int)(R.m2[0] >> 28) : group_of_slot<SH>(G, s);
        const uint32_t wdt = pick(wd, g), base = pick(bs, g);
        if (eo != zero_off) {
          uint32_t u = 0;
          if (wdt) {
            const uint32_t pos = base + (uint32_t)L.rk[s * 64 + lane] * wdt;
            const uint32_t wi = pos >> 5, sh = pos & 31u;
            uint64_t v = pw[wi];
            if (sh + wdt > 32u) v |= (uint64_t)pw[wi + 1] << 32;
            u = (uint32_t)((v >> sh) & ((wdt == 32u) ? 0xffffffffull : ((1ull << wdt) - 1ull)));
          }
          const int q = (int)((u >> 1) ^ (0u - (u & 1u)));
          dq[s] = __dmul_rn(Delta, (double)q);
        }
      }
    }
    wave_sync();      // every lane has read its words before the recomposition writes the buffer
    recompose_w<SH, true>(G, L, R, rm, [&](int s) { return dq[s]; });
  }
  double lam[4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    lam[k] = a.lambda_fp32 ? (double)((const float*)a.lambda)[h * 4 + k] : ((const double*)a.lambda)[h * 4 + k];
  const bool clip = (fl & HCZ_FLAG_NOCLIP) == 0;
  const bool kl = (fl & HCZ_FLAG_KL) != 0;
  double pa = 0.0;
  for_columns_pre(
      G,
      [&](int i) {
        const double av = G.apar[i];
        pa = fma(fma(lam[3], av, lam[1]), av, lam[0]);
      },
      [&](int i, int j) { return fhp ? fhp[j * G.n_par + i] : 0.0f; },
      [&](int i, int j, uint32_t off, float h) {
        const double hv = (double)h;
        const double ft = coded ? hv + ldy(L.yb, off) : hv;
        const double w = UVOL ? G.vol0 : G.vol[j * G.n_par + i];
        const double corr = w * fma(lam[2], L.s_cc[2 * j], pa);
        const double y = ft - corr;
        out[j * G.n_par + i] = (TOut)(kl ? (ft > 0.0 ? ft * exp(-corr) : 0.0) : (clip ? fmax(0.0, y) : y));
      },
      [](int) {});
}

// ---- launchers ----------------------------------------------------------------------------

bool wave_path(const GridDev& G) { return G.nslots > 0 && G.nslots <= kWaveSlots; }
bool wave_fixed_path(const GridDev& G) { return wave_path(G) && G.uniform_vol && shape_matches<Shape39>(G); }

hipError_t launch_residual_w(const GridDev& G, const ResidualArgs& a, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  const bool s39 = wave_fixed_path(G) && a.variant != HCZ_VARIANT_WAVE;
  dim3 grid((unsigned)((a.H + kWPB - 1) / kWPB)), block(64 * kWPB);
  const size_t lds = lds_bytes_w(G);
#define HCZ_RW(T, U, SH, K) hipLaunchKernelGGL((k_residual_w<T, U, SH, K>), grid, block, lds, st, G, a)
#define HCZ_RW2(T, K)                                     \
  do {                                                     \
    if (s39) HCZ_RW(T, true, Shape39, K);                  \
    else if (G.uniform_vol) HCZ_RW(T, true, ShapeDyn, K);  \
    else HCZ_RW(T, false, ShapeDyn, K);                    \
  } while (0)
  if (a.kl) {
    if (a.dtype == HCZ_F32) HCZ_RW2(float, true);
    else HCZ_RW2(double, true);
  } else {
    if (a.dtype == HCZ_F32) HCZ_RW2(float, false);
    else HCZ_RW2(double, false);
  }
#undef HCZ_RW2
#undef HCZ_RW
  return hipGetLastError();
}

hipError_t launch_decompress_w(const GridDev& G, const DecompressArgs& a, hipStream_t st) {
  if (a.H <= 0) return hipSuccess;
  dim3 grid((unsigned)((a.H + kWPB - 1) / kWPB)), block(64 * kWPB);
  const size_t lds = lds_bytes_w(G);
  const bool s39 = wave_fixed_path(G);
#define HCZ_DW(TI, TO, U, SH) hipLaunchKernelGGL((k_decompress_w<TI, TO, U, SH>), grid, block, lds, st, G, a)
#define HCZ_DW2(TI, TO)                                       \
  do {                                                         \
    if (s39) HCZ_DW(TI, TO, true, Shape39);                    \
    else if (G.uniform_vol) HCZ_DW(TI, TO, true, ShapeDyn);    \
    else HCZ_DW(TI, TO, false, ShapeDyn);                      \
  } while (0)
  if (a.in_dtype == HCZ_F32) {
    if (a.out_dtype == HCZ_F64) HCZ_DW2(float, double); else HCZ_DW2(float, float);
  } else {
    if (a.out_dtype == HCZ_F64) HCZ_DW2(double, double); else HCZ_DW2(double, float);
  }
#undef HCZ_DW2
#undef HCZ_DW
  return hipGetLastError();
}

}  // namespace hcz
