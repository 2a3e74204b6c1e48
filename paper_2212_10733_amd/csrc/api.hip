// Host side of libhcz: argument validation, device tables of a grid (plan) and of a
// model, workspace layout and the launch sequence of each C-ABI entry point.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hcz_internal.h"

using namespace hcz;

namespace {

thread_local std::string g_err;

hcz_status fail(hcz_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

hcz_status hip_fail(hipError_t e, const char* what) {
  return fail(HCZ_EHIP, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

namespace hcz {
hcz_status set_error(hcz_status s, const char* msg) { return fail(s, "%s", msg); }
}  // namespace hcz

namespace {

#define HCZ_TRY(expr, what)                       \
  do {                                            \
    hipError_t e_ = (expr);                       \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int nlevels_1d(int n) {
  int m = n - 2, b = 0;
  while (m > 0) { ++b; m >>= 1; }
  return b;
}

}  // namespace

// Stage timing: a ring of event sets; a set is folded into the totals when it is reused
// or when the totals are read.
struct ProfSet {
  hipEvent_t ev[2 * HCZ_NSTAGES];
  bool used[HCZ_NSTAGES];
  bool live;
};

// Workspace of hcz_compress_static: a file-scope device array, one copy per device, held
// until the process ends.  Host code never passes the array's name to a kernel (on the host
// it only stands for the symbol); it uses the device address hipGetSymbolAddress gives for
// the context's device, kept in hcz_ctx::scratch.
static __device__ __align__(256) uint8_t scratch[HCZ_STATIC_SCRATCH_BYTES];

struct hcz_ctx {
  int device;
  uint8_t* scratch = nullptr;   // this device's address of `scratch`
  bool prof = false;
  std::vector<ProfSet> ring;
  int head = 0;
  ProfSet* cur = nullptr;
  double acc_ms[HCZ_NSTAGES] = {};
  int64_t acc_calls[HCZ_NSTAGES] = {};
};

namespace {

void prof_fold(hcz_ctx* c, ProfSet& s) {
  if (!s.live) return;
  for (int k = 0; k < HCZ_NSTAGES; ++k) {
    if (!s.used[k]) continue;
    (void)hipEventSynchronize(s.ev[2 * k + 1]);
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, s.ev[2 * k], s.ev[2 * k + 1]) == hipSuccess) {
      c->acc_ms[k] += ms;
      c->acc_calls[k] += 1;
    }
    s.used[k] = false;
  }
  s.live = false;
}

// Start a new event set for one entry-point call (no-op when profiling is off).
void prof_begin(hcz_ctx* c) {
  c->cur = nullptr;
  if (!c->prof || c->ring.empty()) return;
  ProfSet& s = c->ring[c->head];
  prof_fold(c, s);
  c->head = (c->head + 1) % (int)c->ring.size();
  s.live = true;
  c->cur = &s;
}

struct StageTimer {
  hcz_ctx* c;
  int k;
  hipStream_t st;
  StageTimer(hcz_ctx* c_, int k_, hipStream_t st_) : c(c_), k(k_), st(st_) {
    if (c->cur) (void)hipEventRecord(c->cur->ev[2 * k], st);
  }
  ~StageTimer() {
    if (c->cur) {
      (void)hipEventRecord(c->cur->ev[2 * k + 1], st);
      c->cur->used[k] = true;
    }
  }
};

}  // namespace

struct hcz_plan {
  hcz_ctx* ctx;
  GridDev G;
  std::vector<void*> allocs;
  int variant = HCZ_VARIANT_AUTO;
};

struct hcz_model {
  hcz_plan* plan;
  ModelDev M;
  std::vector<void*> allocs;
};

struct hcz_mlp {
  hcz_ctx* ctx;
  const float* params;
  const double* scale;
  std::vector<void*> allocs;
};

namespace {

template <typename T>
hcz_status upload(std::vector<void*>& allocs, const std::vector<T>& v, const T** out) {
  void* p = nullptr;
  const size_t bytes = std::max<size_t>(v.size() * sizeof(T), 16);
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return fail(HCZ_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
  allocs.push_back(p);
  if (!v.empty()) {
    e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  }
  *out = (const T*)p;
  return HCZ_OK;
}

void free_all(std::vector<void*>& allocs) {
  for (void* p : allocs) (void)hipFree(p);
  allocs.clear();
}

// Per-dimension level tables: lev(i) = the finest level whose node set
// G_l = {multiples of 2^l} U {n-1} contains i (L at both ends), and the bracket of i in
// G_{lev(i)+1} with its interpolation weight.
struct DimTables {
  std::vector<uint8_t> lev, a, b;
  std::vector<double> s;
};

DimTables dim_tables(int n, int L) {
  DimTables d;
  d.lev.resize(n);
  d.a.resize(n);
  d.b.resize(n);
  d.s.resize(n);
  for (int i = 0; i < n; ++i) {
    int lev;
    if (i == 0 || i == n - 1) {
      lev = L;
    } else {
      lev = 0;
      while (((i >> (lev + 1)) << (lev + 1)) == i) ++lev;
    }
    d.lev[i] = (uint8_t)lev;
    if (lev >= L) {
      d.a[i] = d.b[i] = (uint8_t)i;
      d.s[i] = 0.0;
    } else {
      const int l = lev + 1;
      const int a = (i >> l) << l;
      const int b = std::min(a + (1 << l), n - 1);
      d.a[i] = (uint8_t)a;
      d.b[i] = (uint8_t)b;
      d.s[i] = (double)(i - a) / (double)(b - a);
    }
  }
  return d;
}

bool in_set(int n, int l, int i) { return i == n - 1 || (i % (1 << l)) == 0; }

// Slot layout of the wave-per-histogram kernels.  An entry is three words; offsets are
// bytes into a wave's FP64 buffer, which holds the histogram in natural order
// (e = j * n_par + i) followed by one zero cell at N:
//   w0 = off(e) | off(c00) << 16
//   w1 = off(c10) | off(c01) << 16
//   w2 = off(c11) | widx << 16 | tidx << 22 | group << 28
// A linear slot predicts y(c00) + s (y(c10) - y(c00)) with s = wtab[widx], the two
// corners lying on the node's coarse row or column.  A four-corner slot interpolates the
// rows (c00, c10) and (c01, c11) with s, then between the two with t = wtab[tidx]; its
// linear nodes take a degenerate form with the same bits as the linear one (a row node
// repeats its two corners with t = 0, a column node doubles each of its two corners with
// s = 0).  Padding lanes point every offset at the zero cell, with wtab[0] = 0 and
// group 15.  The packing position of each entry is kept apart (its rank within the
// group goes to the device as slot_rank).
struct SlotTables {
  int nslots = 0, ncoarse = 0;
  std::vector<uint32_t> meta;
  std::vector<uint16_t> pos;
  std::vector<double> wtab;
  std::vector<int8_t> group;
  uint32_t bil = 0, sync = 0, keep = 0, half = 0;
};

constexpr uint32_t kPadGroup = 15;

// lanes: nodes per slot, 64 for one wave per histogram, 64 W for a team of W waves; a
// layout needing more than max_slots slots is not built (nslots = 0).
SlotTables make_slots(int np, int nq, int L, const std::vector<uint32_t>& node, const std::vector<int>& gstart,
                      const DimTables& dp, const DimTables& dq, int lanes = 64, int max_slots = kWaveSlots) {
  SlotTables T;
  const int nlev = L + 1;
  const uint32_t zero = (uint32_t)(np * nq) * 8u;
  T.wtab.push_back(0.0);
  auto widx = [&](double w) {
    for (size_t k = 0; k < T.wtab.size(); ++k)
      if (T.wtab[k] == w) return (uint32_t)k;
    T.wtab.push_back(w);
    return (uint32_t)(T.wtab.size() - 1);
  };
  auto off = [&](int i, int j) { return (uint32_t)(j * np + i) * 8u; };
  auto pad = [&](uint32_t* w) {
    w[0] = zero | zero << 16;
    w[1] = zero | zero << 16;
    w[2] = zero | kPadGroup << 28;
  };
  // kind of the node at packing position p in group g: 0 coarsest, 1 row, 2 column, 3 bilinear
  auto kind = [&](int p, int g) {
    if (g == 0) return 0;
    const int i = node[p] & 0xffff, j = node[p] >> 16;
    const int l = L - g + 1;                       // group g holds G_{l-1}^2 minus G_l^2
    if (in_set(nq, l, j)) return 1;
    if (in_set(np, l, i)) return 2;
    return 3;
  };
  auto entry = [&](int p, int g, bool four, uint32_t* w) {
    const int i = node[p] & 0xffff, j = node[p] >> 16;
    uint32_t c00 = zero, c10 = zero, c01 = zero, c11 = zero, wi = 0, ti = 0;
    switch (kind(p, g)) {
      case 1:                                      // along v_par on row j
        c00 = off(dp.a[i], j); c10 = off(dp.b[i], j); wi = widx(dp.s[i]);
        if (four) { c01 = c00; c11 = c10; }
        break;
      case 2:                                      // along v_perp on column i
        if (four) {
          c00 = c10 = off(i, dq.a[j]); c01 = c11 = off(i, dq.b[j]); ti = widx(dq.s[j]);
        } else {
          c00 = off(i, dq.a[j]); c10 = off(i, dq.b[j]); wi = widx(dq.s[j]);
        }
        break;
      case 3:
        c00 = off(dp.a[i], dq.a[j]); c10 = off(dp.b[i], dq.a[j]);
        c01 = off(dp.a[i], dq.b[j]); c11 = off(dp.b[i], dq.b[j]);
        wi = widx(dp.s[i]); ti = widx(dq.s[j]);
        break;
      default:
        break;
    }
    w[0] = off(i, j) | c00 << 16;
    w[1] = c10 | c01 << 16;
    w[2] = c11 | wi << 16 | ti << 22 | (uint32_t)g << 28;
  };
  // slot 0: the coarsest groups while they fit in one slot
  int g = 0, cnt = 0;
  while (g < nlev && cnt + (gstart[g + 1] - gstart[g]) <= lanes) { cnt += gstart[g + 1] - gstart[g]; ++g; }
  if (g == 0) return T;                           // coarsest group alone exceeds a slot
  T.ncoarse = g;
  std::vector<uint32_t> slot((size_t)lanes * 3);
  std::vector<uint16_t> spos(lanes);
  for (int l = 0; l < lanes; ++l) pad(&slot[3 * l]);
  std::fill(spos.begin(), spos.end(), (uint16_t)0);
  for (int p = 0; p < cnt; ++p) {
    int gg = 0;
    while (p >= gstart[gg + 1]) ++gg;
    entry(p, gg, true, &slot[3 * p]);
    spos[p] = (uint16_t)p;
  }
  T.meta.insert(T.meta.end(), slot.begin(), slot.end());
  T.pos.insert(T.pos.end(), spos.begin(), spos.end());
  T.group.push_back(-1);
  std::vector<bool> four;
  four.push_back(true);
  for (; g < nlev; ++g) {
    std::vector<int> lin, bil;
    for (int p = gstart[g]; p < gstart[g + 1]; ++p) (kind(p, g) == 3 ? bil : lin).push_back(p);
    const size_t nlin = lin.size();
    lin.insert(lin.end(), bil.begin(), bil.end());
    for (size_t k = 0; k < lin.size(); k += lanes) {
      const size_t kend = std::min(lin.size(), k + lanes);
      const bool f4 = kend > nlin;                // the slot holds a bilinear node
      for (int l = 0; l < lanes; ++l) pad(&slot[3 * l]);
      std::fill(spos.begin(), spos.end(), (uint16_t)0);
      for (size_t q = k; q < kend; ++q) {
        entry(lin[q], g, f4, &slot[3 * (q - k)]);
        spos[q - k] = (uint16_t)lin[q];
      }
      T.meta.insert(T.meta.end(), slot.begin(), slot.end());
      T.pos.insert(T.pos.end(), spos.begin(), spos.end());
      T.group.push_back((int8_t)g);
      four.push_back(f4);
    }
  }
  T.nslots = (int)T.group.size();
  if (T.nslots > max_slots || T.wtab.size() > 64 || np * nq * 8 + 8 > 65535) {
    T.nslots = 0;
    return T;
  }
  for (int k = 0; k < T.nslots; ++k) {
    // every node of the slot interpolates with weight(s) exactly 1/2 (padding lanes read
    // the zero cell, where any weight gives 0)
    bool half = true;
    for (int l = 0; l < lanes; ++l) {
      const uint32_t* w = &T.meta[((size_t)k * lanes + l) * 3];
      if ((w[0] & 0xffffu) == zero || (w[2] >> 28) == 0) continue;
      half = half && T.wtab[(w[2] >> 16) & 63] == 0.5 && (!four[k] || T.wtab[(w[2] >> 22) & 63] == 0.5);
    }
    if (half && k > 0) T.half |= 1u << k;
    if (four[k]) T.bil |= 1u << k;
    if (k == 0 || k + 1 == T.nslots || T.group[k + 1] != T.group[k]) T.sync |= 1u << k;
    if (k == 0 || T.group[k] < nlev - 1) T.keep |= 1u << k;
  }
  return T;
}

// Every offset the wave kernels take from the slot tables must stay inside the wave's
// buffer: the node's own cell below N and each node once, corners inside the grid (or
// the zero cell) and in strictly coarser groups, weight indices inside wtab, packing
// positions inside the node's group.
bool slots_valid(const SlotTables& T, int np, int nq, int N, int nlev, const std::vector<uint32_t>& node,
                 const std::vector<int>& gstart, int lanes = 64) {
  if (T.nslots == 0) return true;
  if (T.meta.size() != (size_t)T.nslots * lanes * 3 || T.pos.size() != (size_t)T.nslots * lanes) return false;
  const uint32_t zero = (uint32_t)N * 8u;
  std::vector<int> grp(N + 1, -1);
  for (int g = 0; g < nlev; ++g)
    for (int p = gstart[g]; p < gstart[g + 1]; ++p) grp[(node[p] >> 16) * np + (node[p] & 0xffff)] = g;
  std::vector<uint8_t> seen(N, 0);
  for (int s = 0; s < T.nslots; ++s)
    for (int l = 0; l < lanes; ++l) {
      const uint32_t* w = &T.meta[((size_t)s * lanes + l) * 3];
      const uint32_t oe = w[0] & 0xffff, o[4] = {w[0] >> 16, w[1] & 0xffff, w[1] >> 16, w[2] & 0xffff};
      const uint32_t wi = (w[2] >> 16) & 63, ti = (w[2] >> 22) & 63, g = w[2] >> 28;
      for (uint32_t v : {oe, o[0], o[1], o[2], o[3]})
        if (v % 8 || v > zero) return false;
      if (wi >= T.wtab.size() || ti >= T.wtab.size()) return false;
      if (oe == zero) {                            // padding lane
        if (g != kPadGroup || o[0] != zero || o[1] != zero || o[2] != zero || o[3] != zero) return false;
        continue;
      }
      const int e = (int)(oe / 8);
      if (seen[e] || (int)g >= nlev || grp[e] != (int)g) return false;
      if (s == 0 ? (int)g >= T.ncoarse : (int)g != T.group[s]) return false;
      seen[e] = 1;
      const int p = T.pos[(size_t)s * lanes + l];
      if (p < gstart[g] || p >= gstart[g + 1] || (int)((node[p] >> 16) * np + (node[p] & 0xffff)) != e) return false;
      for (uint32_t v : o)
        if (v != zero && grp[v / 8] >= (int)g) return false;
      if (g == 0 && (o[0] != zero || o[1] != zero || o[2] != zero || o[3] != zero)) return false;
    }
  for (int e = 0; e < N; ++e)
    if (!seen[e]) return false;
  return true;
}

hcz_status check_hist(const void* hist, int32_t dtype, int64_t H, int64_t hs, int64_t rs,
                      const GridDev& G) {
  if (H < 0) return fail(HCZ_EINVAL, "H = %lld < 0", (long long)H);
  if (H > 0 && !hist) return fail(HCZ_EINVAL, "hist is NULL");
  if (dtype != HCZ_F32 && dtype != HCZ_F64) return fail(HCZ_EINVAL, "dtype %d", dtype);
  if (rs < G.n_par) return fail(HCZ_EINVAL, "row_stride %lld < n_par %d", (long long)rs, G.n_par);
  if (H > 1 && hs < (int64_t)(G.n_perp - 1) * rs + G.n_par)
    return fail(HCZ_EINVAL, "hist_stride %lld overlaps histograms", (long long)hs);
  if (H > 0x7fffffffLL) return fail(HCZ_EINVAL, "H too large");
  return HCZ_OK;
}

hcz_status check_params(const hcz_params* p) {
  if (!p) return fail(HCZ_EINVAL, "params is NULL");
  if (!p->tau_hist && (!(p->tau >= 0.0) || !std::isfinite(p->tau)))
    return fail(HCZ_EINVAL, "tau must be finite and >= 0");
  if (p->tau_mode != HCZ_TAU_REL_L2 && p->tau_mode != HCZ_TAU_NRMSE) return fail(HCZ_EINVAL, "tau_mode");
  if (!(p->newton_s > 0.0) || !std::isfinite(p->newton_s)) return fail(HCZ_EINVAL, "newton_s must be > 0");
  if (p->newton_max_iter < 0 || p->newton_max_iter2 < 0) return fail(HCZ_EINVAL, "newton iteration caps must be >= 0");
  if (p->fallback != HCZ_FALLBACK_BACKTRACK && p->fallback != HCZ_FALLBACK_PAPER) return fail(HCZ_EINVAL, "fallback");
  if (p->fit_codebook && p->sample_every < 1) return fail(HCZ_EINVAL, "sample_every must be >= 1");
  if (p->warm_start != HCZ_WARM_COLD && p->warm_start != HCZ_WARM_MLP && p->warm_start != HCZ_WARM_ANALYTIC)
    return fail(HCZ_EINVAL, "warm_start");
  if (p->warm_start == HCZ_WARM_ANALYTIC && p->no_positivity)
    return fail(HCZ_EINVAL, "the analytic start belongs to the projection with positivity");
  if (p->warm_start == HCZ_WARM_MLP && !p->mlp) return fail(HCZ_EINVAL, "warm_start needs an mlp");
  if (p->lambda_fp32 != 0 && p->lambda_fp32 != 1) return fail(HCZ_EINVAL, "lambda_fp32 must be 0 or 1");
  if (p->no_positivity != 0 && p->no_positivity != 1) return fail(HCZ_EINVAL, "no_positivity must be 0 or 1");
  if (p->kl != 0 && p->kl != 1) return fail(HCZ_EINVAL, "kl must be 0 or 1");
  if (p->lambda_bits < 0 || p->lambda_bits > 52 || (p->lambda_fp32 && p->lambda_bits > 23))
    return fail(HCZ_EINVAL, "lambda_bits must be in [0, 52] ([0, 23] with FP32 multipliers)");
  if (p->kl && (p->no_positivity || p->warm_start != HCZ_WARM_COLD))
    return fail(HCZ_EINVAL, "kl is not combined with no_positivity or a warm start");
  if (p->bound_mode != HCZ_BOUND_AB && p->bound_mode != HCZ_BOUND_UB) return fail(HCZ_EINVAL, "bound_mode");
  if (p->bound_mode == HCZ_BOUND_UB && (p->ub_level < 0 || p->ub_level > 40))
    return fail(HCZ_EINVAL, "ub_level must be in [0, 40]");
  if (p->search != HCZ_SEARCH_GUIDED && p->search != HCZ_SEARCH_BISECT) return fail(HCZ_EINVAL, "search");
  return HCZ_OK;
}

size_t slot_stride(const GridDev& G, int32_t dtype) {
  const size_t coded = (size_t)G.hdr_bytes + 4 * (size_t)G.N;
  const size_t raw = (size_t)G.N * (dtype == HCZ_F64 ? 8 : 4);
  return (std::max(coded, raw) + 15) / 16 * 16;
}

struct WsLayout {
  size_t z, fhat, lam0, sizes, kstar, iters, partial, slots, cbws, total;
};

WsLayout ws_layout(const GridDev& G, bool model, int64_t H, int32_t dtype, bool fit, int64_t every) {
  WsLayout w{};
  size_t o = 0;
  w.z = o;      o += model ? align256((size_t)H * kLatent * 4) : 0;
  w.lam0 = o;   o += model ? align256((size_t)H * 4 * 8) : 0;
  w.fhat = o;   o += model ? align256((size_t)H * G.N * 4) : 0;
  w.sizes = o;  o += align256((size_t)H * 8);
  w.kstar = o;  o += align256((size_t)H);
  w.iters = o;  o += align256((size_t)H * 2);
  w.partial = o; o += align256(scan_partial_elems(H) * 8);
  w.cbws = o;   o += (model && fit) ? align256(codebook_ws_bytes(H, kLatent, std::max<int64_t>(every, 1))) : 0;
  w.slots = o;  o += align256((size_t)H * slot_stride(G, dtype));
  w.total = o;
  return w;
}

hcz_status set_device(const hcz_ctx* ctx) {
  HCZ_TRY(hipSetDevice(ctx->device), "hipSetDevice");
  return HCZ_OK;
}

hcz_status check_cb(const hcz_codebook* cb) {
  if (!cb || !cb->centroids) return fail(HCZ_EINVAL, "codebook or its centroids is NULL");
  if (cb->bits < 1 || cb->bits > 8) return fail(HCZ_EINVAL, "codebook bits %d not in [1, 8]", cb->bits);
  return HCZ_OK;
}

}  // namespace

extern "C" {

const char* hcz_last_error(void) { return g_err.c_str(); }
const char* hcz_version(void) { return "hcz 0.1 gfx950"; }

hcz_status hcz_create(int device, hcz_ctx** out) {
  if (!out) return fail(HCZ_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  HCZ_TRY(hipGetDeviceCount(&n), "hipGetDeviceCount");
  if (device < 0 || device >= n) return fail(HCZ_EINVAL, "device %d of %d", device, n);
  HCZ_TRY(hipSetDevice(device), "hipSetDevice");
  void* sp = nullptr;
  HCZ_TRY(hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
  hcz_ctx* c = new hcz_ctx{device};
  c->scratch = (uint8_t*)sp;
  *out = c;
  return HCZ_OK;
}

void hcz_destroy(hcz_ctx* ctx) {
  if (!ctx) return;
  for (auto& set : ctx->ring)
    for (auto& e : set.ev) (void)hipEventDestroy(e);
  delete ctx;
}

hcz_status hcz_plan_create(hcz_ctx* ctx, const hcz_grid* g, hcz_plan** out) {
  if (!ctx || !g || !out) return fail(HCZ_EINVAL, "NULL argument");
  *out = nullptr;
  const int np = g->n_par, nq = g->n_perp;
  if (np < 3 || nq < 3 || np > kMaxDim || nq > kMaxDim || np * nq > kMaxN)
    return fail(HCZ_EINVAL, "grid %d x %d outside 3..%d per side, %d cells", np, nq, kMaxDim, kMaxN);
  if (!(g->vpar_hi > g->vpar_lo) || !(g->vperp_hi > g->vperp_lo) || !std::isfinite(g->vpar_lo) ||
      !std::isfinite(g->vpar_hi) || !std::isfinite(g->vperp_lo) || !std::isfinite(g->vperp_hi))
    return fail(HCZ_EINVAL, "velocity ranges must be finite with hi > lo");
  if (!(g->mass > 0.0) || !std::isfinite(g->mass)) return fail(HCZ_EINVAL, "mass must be > 0");
  hcz_status s = set_device(ctx);
  if (s) return s;
  const int N = np * nq;
  const double dpar = (g->vpar_hi - g->vpar_lo) / (np - 1);
  const double dperp = (g->vperp_hi - g->vperp_lo) / (nq - 1);
  const double Vpar = std::max(std::fabs(g->vpar_lo), std::fabs(g->vpar_hi));
  const double Vperp = std::max(std::fabs(g->vperp_lo), std::fabs(g->vperp_hi));
  std::vector<double> apar(np), cperp(nq), vol(N);
  for (int i = 0; i < np; ++i) apar[i] = (g->vpar_lo + i * dpar) / Vpar;
  for (int j = 0; j < nq; ++j) {
    const double c = (g->vperp_lo + j * dperp) / Vperp;
    cperp[j] = c * c;
  }
  bool uniform = g->vol == nullptr;
  for (int e = 0; e < N; ++e) {
    vol[e] = g->vol ? g->vol[e] : dpar * dperp;
    if (!(vol[e] > 0.0) || !std::isfinite(vol[e])) return fail(HCZ_EINVAL, "vol[%d] must be finite and > 0", e);
  }
  const int L = std::max(nlevels_1d(np), nlevels_1d(nq));
  const int nlev = L + 1;
  if (nlev > kMaxLev) return fail(HCZ_EUNSUPPORTED, "%d levels", nlev);
  // packing order: coarsest node set first, then levels L..1, row-major within a group
  std::vector<uint32_t> node;
  node.reserve(N);
  std::vector<int> gstart;
  gstart.push_back(0);
  for (int j = 0; j < nq; ++j)
    for (int i = 0; i < np; ++i)
      if (in_set(nq, L, j) && in_set(np, L, i)) node.push_back((uint32_t)i | ((uint32_t)j << 16));
  gstart.push_back((int)node.size());
  for (int l = L; l >= 1; --l) {
    for (int j = 0; j < nq; ++j)
      for (int i = 0; i < np; ++i) {
        if (!in_set(nq, l - 1, j) || !in_set(np, l - 1, i)) continue;
        if (in_set(nq, l, j) && in_set(np, l, i)) continue;
        node.push_back((uint32_t)i | ((uint32_t)j << 16));
      }
    gstart.push_back((int)node.size());
  }
  if ((int)node.size() != N) return fail(HCZ_EINVAL, "internal: node layout has %zu of %d nodes", node.size(), N);
  DimTables dp = dim_tables(np, L), dq = dim_tables(nq, L);
  SlotTables slots = make_slots(np, nq, L, node, gstart, dp, dq);
  if (!slots_valid(slots, np, nq, N, nlev, node, gstart))
    return fail(HCZ_EINVAL, "internal: slot tables for %dx%d failed their check", np, nq);
  // the wave-team layouts: slots of 128 (two waves) and 256 nodes (four waves)
  SlotTables team[2] = {make_slots(np, nq, L, node, gstart, dp, dq, 128, kTeamSlots2),
                        make_slots(np, nq, L, node, gstart, dp, dq, 256, kTeamSlots4)};
  for (int k = 0; k < 2; ++k)
    if (!slots_valid(team[k], np, nq, N, nlev, node, gstart, k == 0 ? 128 : 256))
      return fail(HCZ_EINVAL, "internal: team slot tables for %dx%d failed their check", np, nq);
  hcz_plan* P = new hcz_plan();
  P->ctx = ctx;
  GridDev& G = P->G;
  G.n_par = np;
  G.n_perp = nq;
  G.N = N;
  G.L = L;
  G.nlev = nlev;
  G.hdr_bytes = 8 * ((10 + nlev + 7) / 8);
  G.uniform_vol = uniform ? 1 : 0;
  for (int q = 0; q <= kMaxLev; ++q) G.gstart[q] = q < (int)gstart.size() ? gstart[q] : N;
  G.vol0 = dpar * dperp;
  G.sqrtN = std::sqrt((double)N);
  G.den = std::sqrt((double)N) * (double)(L + 1);
  G.Vpar = Vpar;
  G.Vperp = Vperp;
  G.mass = g->mass;
  G.nslots = slots.nslots;
  G.ncoarse = slots.ncoarse;
  G.nw = (int)slots.wtab.size();
  // packing rank of each entry within its group (0 for padding lanes)
  std::vector<uint16_t> rank(slots.pos.size(), 0);
  for (size_t k = 0; k < rank.size(); ++k) {
    const uint32_t w0 = slots.meta[3 * k], w2 = slots.meta[3 * k + 2];
    if ((w0 & 0xffffu) != (uint32_t)N * 8u) rank[k] = (uint16_t)(slots.pos[k] - gstart[w2 >> 28]);
  }
  for (int k = 0; k < kWaveSlots; ++k) G.slot_group[k] = k < slots.nslots ? slots.group[k] : 0;
  G.slot_bil = slots.bil;
  G.slot_sync = slots.sync;
  G.slot_keep = slots.keep;
  G.slot_half = slots.half;
  std::vector<uint16_t> trank[2];
  for (int k = 0; k < 2; ++k) {
    const SlotTables& T = team[k];
    G.tnslots[k] = T.nslots;
    G.tncoarse[k] = T.ncoarse;
    G.tnw[k] = (int)T.wtab.size();
    G.tslot_bil[k] = T.bil;
    G.tslot_sync[k] = T.sync;
    G.tslot_keep[k] = T.keep;
    G.tslot_meta[k] = nullptr;
    G.tslot_rank[k] = nullptr;
    G.twtab[k] = nullptr;
    trank[k].assign(T.pos.size(), 0);
    for (size_t q = 0; q < trank[k].size(); ++q) {
      const uint32_t w0 = T.meta[3 * q], w2 = T.meta[3 * q + 2];
      if ((w0 & 0xffffu) != (uint32_t)N * 8u) trank[k][q] = (uint16_t)(T.pos[q] - gstart[w2 >> 28]);
    }
  }
  if ((s = upload(P->allocs, vol, &G.vol)) || (s = upload(P->allocs, apar, &G.apar)) ||
      (s = upload(P->allocs, cperp, &G.cperp)) || (s = upload(P->allocs, node, &G.node_ij)) ||
      (s = upload(P->allocs, dp.lev, &G.lev_par)) || (s = upload(P->allocs, dp.a, &G.a_par)) ||
      (s = upload(P->allocs, dp.b, &G.b_par)) || (s = upload(P->allocs, dp.s, &G.s_par)) ||
      (s = upload(P->allocs, dq.lev, &G.lev_perp)) || (s = upload(P->allocs, dq.a, &G.a_perp)) ||
      (s = upload(P->allocs, dq.b, &G.b_perp)) || (s = upload(P->allocs, dq.s, &G.s_perp)) ||
      (s = upload(P->allocs, slots.meta, &G.slot_meta)) || (s = upload(P->allocs, rank, &G.slot_rank)) ||
      (s = upload(P->allocs, slots.wtab, &G.wtab)) ||
      (team[0].nslots > 0 && ((s = upload(P->allocs, team[0].meta, &G.tslot_meta[0])) ||
                              (s = upload(P->allocs, trank[0], &G.tslot_rank[0])) ||
                              (s = upload(P->allocs, team[0].wtab, &G.twtab[0])))) ||
      (team[1].nslots > 0 && ((s = upload(P->allocs, team[1].meta, &G.tslot_meta[1])) ||
                              (s = upload(P->allocs, trank[1], &G.tslot_rank[1])) ||
                              (s = upload(P->allocs, team[1].wtab, &G.twtab[1]))))) {
    free_all(P->allocs);
    delete P;
    return s;
  }
  *out = P;
  return HCZ_OK;
}

hcz_status hcz_plan_variants(const hcz_plan* plan, int32_t* list, int32_t* n) {
  if (!plan || !list || !n) return fail(HCZ_EINVAL, "NULL argument");
  const GridDev& G = plan->G;
  int k = 0;
  list[k++] = HCZ_VARIANT_AUTO;
  if (wave_fixed_path(G)) list[k++] = HCZ_VARIANT_WAVE_FIXED;
  if (wave_path(G)) list[k++] = HCZ_VARIANT_WAVE;
  if (G.N <= 256 * 6) list[k++] = HCZ_VARIANT_BLOCK_256x6;
  if (G.N <= 512 * 5) list[k++] = HCZ_VARIANT_BLOCK_512x5;
  if (G.N <= 512 * 9) list[k++] = HCZ_VARIANT_BLOCK_512x9;
  if (team_path(G, 2)) list[k++] = HCZ_VARIANT_TEAM2;
  if (team_path(G, 4)) list[k++] = HCZ_VARIANT_TEAM4;
  *n = k;
  return HCZ_OK;
}

hcz_status hcz_plan_set_variant(hcz_plan* plan, int32_t variant) {
  if (!plan) return fail(HCZ_EINVAL, "NULL argument");
  int32_t list[8], n = 0;
  hcz_plan_variants(plan, list, &n);
  for (int i = 0; i < n; ++i)
    if (list[i] == variant) {
      plan->variant = variant;
      return HCZ_OK;
    }
  return fail(HCZ_EUNSUPPORTED, "variant %d is not valid for this grid", variant);
}

hcz_status hcz_plan_path(const hcz_plan* plan, int32_t* path) {
  if (!plan || !path) return fail(HCZ_EINVAL, "NULL argument");
  const GridDev& G = plan->G;
  *path = wave_fixed_path(G) ? HCZ_PATH_WAVE_FIXED
          : wave_path(G)     ? HCZ_PATH_WAVE
          : team_path(G, 2)  ? HCZ_PATH_TEAM2
          : team_path(G, 4)  ? HCZ_PATH_TEAM4
                             : HCZ_PATH_BLOCK;
  return HCZ_OK;
}

void hcz_plan_destroy(hcz_plan* plan) {
  if (!plan) return;
  free_all(plan->allocs);
  delete plan;
}

// nearest-even bfloat16 of a finite or infinite FP32 value (NaN keeps a quiet NaN)
static uint16_t bf16_rne(float x) {
  uint32_t u;
  std::memcpy(&u, &x, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

static hcz_status conv_model_load(hcz_plan* plan, const hcz_model_desc* d, hcz_model** out) {
  if (plan->G.n_par != 39 || plan->G.n_perp != 39)
    return fail(HCZ_EUNSUPPORTED, "the convolutional model needs a 39 x 39 grid");
  if (d->latent != kLatent) return fail(HCZ_EUNSUPPORTED, "convolutional model must have latent %d", kLatent);
  if (d->compute != HCZ_COMPUTE_BF16) return fail(HCZ_EUNSUPPORTED, "the convolutional model runs in the BF16 form");
  if (!d->weights || !d->norm_mean || !d->norm_std) return fail(HCZ_EINVAL, "weights or norm stats NULL");
  hcz_status s = set_device(plan->ctx);
  if (s) return s;
  const int N = 1521;
  std::vector<float> mu(d->norm_mean, d->norm_mean + N), sd(d->norm_std, d->norm_std + N), rsd(N);
  for (int k = 0; k < N; ++k) {
    if (!(sd[k] > 0.0f) || !std::isfinite(sd[k]) || !std::isfinite(mu[k]))
      return fail(HCZ_EINVAL, "norm_std[%d] must be finite and > 0", k);
    rsd[k] = 1.0f / sd[k];
  }
  const float* w = d->weights;
  const float *c1w = w, *c1b = c1w + 288, *c2w = c1b + 32, *c2b = c2w + 18432, *fw = c2b + 64,
              *fb = fw + 102400, *dw = fb + 16, *db = dw + 102400, *t1w = db + 6400, *t1b = t1w + 18432,
              *t2w = t1b + 32, *t2b = t2w + 288;
  // matrix-core operands: bfloat16, [tap][out][in]
  std::vector<uint16_t> c2(9 * 64 * 32), t1(9 * 32 * 64);
  for (int co = 0; co < 64; ++co)
    for (int ci = 0; ci < 32; ++ci)
      for (int tap = 0; tap < 9; ++tap) c2[(tap * 64 + co) * 32 + ci] = bf16_rne(c2w[(co * 32 + ci) * 9 + tap]);
  for (int ci = 0; ci < 64; ++ci)
    for (int co = 0; co < 32; ++co)
      for (int tap = 0; tap < 9; ++tap) t1[(tap * 32 + co) * 64 + ci] = bf16_rne(t1w[(ci * 32 + co) * 9 + tap]);
  hcz_model* m = new hcz_model();
  m->plan = plan;
  ModelDev& M = m->M;
  M.N = N;
  M.hidden = 0;
  M.latent = kLatent;
  M.arch = HCZ_ARCH_CONV;
  M.bf16 = 1;
  auto vec = [](const float* p, size_t n) { return std::vector<float>(p, p + n); };
  if ((s = upload(m->allocs, vec(c1w, 288), &M.c1w)) || (s = upload(m->allocs, vec(c1b, 32), &M.c1b)) ||
      (s = upload(m->allocs, c2, &M.c2w)) || (s = upload(m->allocs, vec(c2b, 64), &M.c2b)) ||
      (s = upload(m->allocs, vec(fw, 102400), &M.fw)) || (s = upload(m->allocs, vec(fb, 16), &M.fb)) ||
      (s = upload(m->allocs, vec(dw, 102400), &M.dw)) || (s = upload(m->allocs, vec(db, 6400), &M.db)) ||
      (s = upload(m->allocs, t1, &M.t1w)) || (s = upload(m->allocs, vec(t1b, 32), &M.t1b)) ||
      (s = upload(m->allocs, vec(t2w, 288), &M.t2w)) || (s = upload(m->allocs, vec(t2b, 1), &M.t2b)) ||
      (s = upload(m->allocs, mu, &M.mu)) || (s = upload(m->allocs, rsd, &M.rsd)) ||
      (s = upload(m->allocs, sd, &M.sd))) {
    free_all(m->allocs);
    delete m;
    return s;
  }
  {
    void* p = nullptr;
    const size_t bytes = (size_t)kConvChunk * 6400 * sizeof(float);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      free_all(m->allocs);
      delete m;
      return fail(HCZ_ENOMEM, "hipMalloc(%zu): %s", bytes, hipGetErrorString(e));
    }
    m->allocs.push_back(p);
    M.scratch = (float*)p;
  }
  *out = m;
  return HCZ_OK;
}

hcz_status hcz_model_load(hcz_plan* plan, const hcz_model_desc* d, hcz_model** out) {
  if (!plan || !d || !out) return fail(HCZ_EINVAL, "NULL argument");
  *out = nullptr;
  if (d->arch == HCZ_ARCH_CONV) return conv_model_load(plan, d, out);
  if (d->arch != HCZ_ARCH_DENSE) return fail(HCZ_EUNSUPPORTED, "arch %d", d->arch);
  if (d->hidden != kHidden || d->latent != kLatent)
    return fail(HCZ_EUNSUPPORTED, "dense model must be hidden %d, latent %d", kHidden, kLatent);
  if (!d->weights || !d->norm_mean || !d->norm_std) return fail(HCZ_EINVAL, "weights or norm stats NULL");
  if (d->compute != HCZ_COMPUTE_FP32 && d->compute != HCZ_COMPUTE_BF16 && d->compute != HCZ_COMPUTE_FP64)
    return fail(HCZ_EINVAL, "compute %d", d->compute);
  hcz_status s = set_device(plan->ctx);
  if (s) return s;
  const int N = plan->G.N, Hd = kHidden, Ld = kLatent;
  const int kpad = (N + 31) / 32 * 32, npad = (N + 127) / 128 * 128;
  const float* w = d->weights;
  const float *W1 = w, *b1 = W1 + (size_t)Hd * N, *W2 = b1 + Hd, *b2 = W2 + Ld * Hd, *W3 = b2 + Ld,
              *b3 = W3 + Hd * Ld, *W4 = b3 + Hd, *b4 = W4 + (size_t)N * Hd;
  std::vector<float> W1p((size_t)Hd * kpad, 0.0f), W4p((size_t)npad * Hd, 0.0f);
  for (int r = 0; r < Hd; ++r)
    for (int k = 0; k < N; ++k) W1p[(size_t)r * kpad + k] = W1[(size_t)r * N + k];
  for (int c = 0; c < N; ++c)
    for (int k = 0; k < Hd; ++k) W4p[(size_t)c * Hd + (k & 1) * 64 + (k >> 1)] = W4[(size_t)c * Hd + k];
  std::vector<float> mu(d->norm_mean, d->norm_mean + N), sd(d->norm_std, d->norm_std + N), rsd(N);
  for (int k = 0; k < N; ++k) {
    if (!(sd[k] > 0.0f) || !std::isfinite(sd[k]) || !std::isfinite(mu[k]))
      return fail(HCZ_EINVAL, "norm_std[%d] must be finite and > 0", k);
    rsd[k] = 1.0f / sd[k];
  }
  hcz_model* m = new hcz_model();
  m->plan = plan;
  ModelDev& M = m->M;
  M.N = N;
  M.hidden = Hd;
  M.latent = Ld;
  M.kpad = kpad;
  M.npad = npad;
  M.bf16 = d->compute == HCZ_COMPUTE_BF16;
  M.arch = HCZ_ARCH_DENSE;
  std::vector<float> vb1(b1, b1 + Hd), vW2(W2, W2 + Ld * Hd), vb2(b2, b2 + Ld), vW3(W3, W3 + Hd * Ld),
      vb3(b3, b3 + Hd), vb4(b4, b4 + N);
  if (M.bf16) {
    // BF16 form: W1 rounded to nearest-even bfloat16 in natural k order (the strided
    // encoder), and W1 and W4 in matrix-core operand order
    std::vector<uint16_t> W1b((size_t)Hd * kpad, 0);
    for (int r = 0; r < Hd; ++r)
      for (int k = 0; k < N; ++k) W1b[(size_t)r * kpad + k] = bf16_rne(W1[(size_t)r * N + k]);
    // operand order of the encoder: [k-step t][column tile n][lane l][8]: column 32 n + l % 32,
    // k = 16 t + 8 (l / 32) + e; zero beyond N
    std::vector<uint16_t> W1m((size_t)(kpad / 16) * 4 * 64 * 8, 0);
    for (int tt = 0; tt < kpad / 16; ++tt)
      for (int n = 0; n < 4; ++n)
        for (int l = 0; l < 64; ++l)
          for (int e = 0; e < 8; ++e) {
            const int col = 32 * n + (l & 31), k = 16 * tt + 8 * (l >> 5) + e;
            W1m[(((size_t)tt * 4 + n) * 64 + l) * 8 + e] = k < N ? bf16_rne(W1[(size_t)col * N + k]) : 0;
          }
    // decoder operand order: [64-column block][tile n][k-step t][lane l][8]: column
    // 64 b + 32 n + l % 32, k = 16 t + 8 (l / 32) + e; zero for columns >= N
    std::vector<uint16_t> W4m((size_t)(npad / 64) * 2 * 8 * 64 * 8, 0);
    for (int b = 0; b < npad / 64; ++b)
      for (int n = 0; n < 2; ++n)
        for (int tt = 0; tt < 8; ++tt)
          for (int l = 0; l < 64; ++l)
            for (int e = 0; e < 8; ++e) {
              const int col = 64 * b + 32 * n + (l & 31), k = 16 * tt + 8 * (l >> 5) + e;
              W4m[((((size_t)b * 2 + n) * 8 + tt) * 64 + l) * 8 + e] =
                  col < N ? bf16_rne(W4[(size_t)col * Hd + k]) : 0;
            }
    if ((s = upload(m->allocs, W1b, &M.W1b)) || (s = upload(m->allocs, W1m, &M.W1m)) ||
        (s = upload(m->allocs, W4m, &M.W4m))) {
      free_all(m->allocs);
      delete m;
      return s;
    }
  }
  M.fp64 = d->compute == HCZ_COMPUTE_FP64;
  if (M.fp64) {
    // FP64 form: exact widenings, W1 and W4 transposed so that a thread's reads coalesce
    std::vector<double> W1t((size_t)N * Hd), W4t((size_t)Hd * N), db1(b1, b1 + Hd), dW2(W2, W2 + Ld * Hd),
        db2(b2, b2 + Ld), dW3(W3, W3 + Hd * Ld), db3(b3, b3 + Hd), db4(b4, b4 + N), dmu(mu.begin(), mu.end()),
        dsd(sd.begin(), sd.end());
    for (int r = 0; r < Hd; ++r)
      for (int k = 0; k < N; ++k) W1t[(size_t)k * Hd + r] = W1[(size_t)r * N + k];
    for (int n = 0; n < N; ++n)
      for (int c = 0; c < Hd; ++c) W4t[(size_t)c * N + n] = W4[(size_t)n * Hd + c];
    if ((s = upload(m->allocs, W1t, &M.W1t)) || (s = upload(m->allocs, db1, &M.b1d)) ||
        (s = upload(m->allocs, dW2, &M.W2d)) || (s = upload(m->allocs, db2, &M.b2d)) ||
        (s = upload(m->allocs, dW3, &M.W3d)) || (s = upload(m->allocs, db3, &M.b3d)) ||
        (s = upload(m->allocs, W4t, &M.W4t)) || (s = upload(m->allocs, db4, &M.b4d)) ||
        (s = upload(m->allocs, dmu, &M.mud)) || (s = upload(m->allocs, dsd, &M.sdd))) {
      free_all(m->allocs);
      delete m;
      return s;
    }
  }
  if ((s = upload(m->allocs, W1p, &M.W1p)) || (s = upload(m->allocs, vb1, &M.b1)) ||
      (s = upload(m->allocs, vW2, &M.W2)) || (s = upload(m->allocs, vb2, &M.b2)) ||
      (s = upload(m->allocs, vW3, &M.W3)) || (s = upload(m->allocs, vb3, &M.b3)) ||
      (s = upload(m->allocs, W4p, &M.W4p)) || (s = upload(m->allocs, vb4, &M.b4)) ||
      (s = upload(m->allocs, mu, &M.mu)) || (s = upload(m->allocs, rsd, &M.rsd)) ||
      (s = upload(m->allocs, sd, &M.sd))) {
    free_all(m->allocs);
    delete m;
    return s;
  }
  *out = m;
  return HCZ_OK;
}

void hcz_model_free(hcz_model* m) {
  if (!m) return;
  free_all(m->allocs);
  delete m;
}

hcz_status hcz_qoi(const hcz_plan* plan, const void* hist, int32_t dtype, int64_t H,
                   int64_t hist_stride, int64_t row_stride, double* b, double* qoi, double* norm,
                   hcz_stream_t stream) {
  if (!plan) return fail(HCZ_EINVAL, "plan is NULL");
  hcz_status s = check_hist(hist, dtype, H, hist_stride, row_stride, plan->G);
  if (s) return s;
  if ((s = set_device(plan->ctx))) return s;
  HCZ_TRY(launch_qoi(plan->G, hist, dtype, H, hist_stride, row_stride, b, qoi, norm, (hipStream_t)stream), "qoi launch");
  return HCZ_OK;
}

hcz_status hcz_encode(const hcz_model* model, const void* hist, int32_t dtype, int64_t H,
                      int64_t hist_stride, int64_t row_stride, float* z, hcz_stream_t stream) {
  if (!model) return fail(HCZ_EINVAL, "model is NULL");
  hcz_status s = check_hist(hist, dtype, H, hist_stride, row_stride, model->plan->G);
  if (s) return s;
  if (H > 0 && !z) return fail(HCZ_EINVAL, "z is NULL");
  if ((s = set_device(model->plan->ctx))) return s;
  HCZ_TRY(launch_encode(model->M, hist, dtype, H, hist_stride, row_stride, model->plan->G.n_par, z,
                        (hipStream_t)stream), "encode launch");
  return HCZ_OK;
}

hcz_status hcz_codebook_fit_workspace(int64_t n, int32_t latent, int64_t sample_every, size_t* bytes) {
  if (!bytes || n < 1 || latent < 1 || sample_every < 1) return fail(HCZ_EINVAL, "bad argument");
  *bytes = codebook_ws_bytes(n, latent, sample_every);
  return HCZ_OK;
}

hcz_status hcz_codebook_fit(const float* z, int64_t n, int32_t latent, int64_t sample_every,
                            hcz_codebook* cb, void* ws, size_t ws_bytes, hcz_stream_t stream) {
  if (!z || n < 1 || latent < 1 || latent > 65535 || sample_every < 1) return fail(HCZ_EINVAL, "bad argument");
  hcz_status s = check_cb(cb);
  if (s) return s;
  if (!ws || ws_bytes < codebook_ws_bytes(n, latent, sample_every))
    return fail(HCZ_EWORKSPACE, "workspace %zu < %zu", ws_bytes, codebook_ws_bytes(n, latent, sample_every));
  HCZ_TRY(launch_codebook_fit(z, n, latent, sample_every, cb->bits, cb->centroids, ws, (hipStream_t)stream),
          "codebook launch");
  return HCZ_OK;
}

hcz_status hcz_quantize(const float* z, int64_t n, int32_t latent, const hcz_codebook* cb,
                        uint8_t* codes, hcz_stream_t stream) {
  if (n < 0 || latent < 1) return fail(HCZ_EINVAL, "bad size");
  if (n > 0 && (!z || !codes)) return fail(HCZ_EINVAL, "NULL buffer");
  hcz_status s = check_cb(cb);
  if (s) return s;
  HCZ_TRY(launch_quantize(z, n, latent, cb->centroids, cb->bits, codes, (hipStream_t)stream), "quantize launch");
  return HCZ_OK;
}

hcz_status hcz_segment_tau(const int64_t* seg_start, const double* seg_tau, int32_t nseg, int64_t H,
                           double* tau_hist, hcz_stream_t stream) {
  if (nseg < 1 || H < 0) return fail(HCZ_EINVAL, "nseg must be >= 1 and H >= 0");
  if (!seg_start || !seg_tau || (H > 0 && !tau_hist)) return fail(HCZ_EINVAL, "NULL buffer");
  HCZ_TRY(launch_segment_tau(seg_start, seg_tau, nseg, H, tau_hist, (hipStream_t)stream), "segment launch");
  return HCZ_OK;
}

hcz_status hcz_segment_max(const int64_t* seg_start, int32_t nseg, int64_t H, const uint64_t* t,
                           uint64_t* seg_max, hcz_stream_t stream) {
  if (nseg < 1 || H < 0) return fail(HCZ_EINVAL, "nseg must be >= 1 and H >= 0");
  if (!seg_start || !seg_max || (H > 0 && !t)) return fail(HCZ_EINVAL, "NULL buffer");
  HCZ_TRY(launch_segment_max(seg_start, nseg, H, t, seg_max, (hipStream_t)stream), "segment launch");
  return HCZ_OK;
}

hcz_status hcz_timestamp(uint64_t* dst, hcz_stream_t stream) {
  if (!dst) return fail(HCZ_EINVAL, "NULL buffer");
  HCZ_TRY(launch_timestamp(dst, (hipStream_t)stream), "timestamp launch");
  return HCZ_OK;
}

hcz_status hcz_wall_clock_hz(int device, double* hz) {
  if (!hz) return fail(HCZ_EINVAL, "NULL argument");
  int khz = 0;
  hipError_t e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device);
  if (e != hipSuccess) return hip_fail(e, "hipDeviceGetAttribute");
  if (khz <= 0) return fail(HCZ_EUNSUPPORTED, "device reports no wall clock rate");
  *hz = 1e3 * khz;
  return HCZ_OK;
}

hcz_status hcz_decode(const hcz_model* model, const uint8_t* codes, const hcz_codebook* cb,
                      int64_t H, float* fhat, hcz_stream_t stream) {
  if (!model) return fail(HCZ_EINVAL, "model is NULL");
  if (H < 0) return fail(HCZ_EINVAL, "H < 0");
  if (H > 0 && (!codes || !fhat)) return fail(HCZ_EINVAL, "NULL buffer");
  hcz_status s = check_cb(cb);
  if (s) return s;
  if ((s = set_device(model->plan->ctx))) return s;
  HCZ_TRY(launch_decode(model->M, codes, cb->centroids, cb->bits, H, fhat, (hipStream_t)stream), "decode launch");
  return HCZ_OK;
}

hcz_status hcz_compress_workspace(const hcz_plan* plan, const hcz_model* model, int64_t H,
                                  const hcz_params* params, size_t* bytes) {
  if (!plan || !bytes || H < 0) return fail(HCZ_EINVAL, "bad argument");
  const bool fit = params && params->fit_codebook;
  const int64_t every = params ? std::max<int64_t>(params->sample_every, 1) : 1;
  // sized for FP64 input, which needs the larger verbatim records
  *bytes = ws_layout(plan->G, model != nullptr, H, HCZ_F64, fit, every).total;
  return HCZ_OK;
}

hcz_status hcz_decompress_workspace(const hcz_plan* plan, const hcz_model* model, int64_t H, size_t* bytes) {
  if (!plan || !bytes || H < 0) return fail(HCZ_EINVAL, "bad argument");
  *bytes = model ? align256((size_t)H * plan->G.N * 4) : 0;
  return HCZ_OK;
}

static ResidualArgs residual_args(const hcz_plan* plan, const hcz_params* p, const void* hist, int32_t dtype,
                                  int64_t H, int64_t hs, int64_t rs, const float* fhat, const double* lam0,
                                  hcz_compressed* out, uint8_t* ws, const WsLayout& L) {
  const GridDev& G = plan->G;
  ResidualArgs a{};
  a.hist = hist;
  a.dtype = dtype;
  a.hs = hs;
  a.rs = rs;
  a.H = H;
  a.fhat = fhat;
  a.tau = p->tau;
  a.tau_hist = p->tau_hist;
  a.tau_mode = p->tau_mode;
  a.newton_s = p->newton_s;
  a.max_iter = p->newton_max_iter;
  a.max_iter2 = p->newton_max_iter2;
  a.fallback = p->fallback;
  a.lambda = out->lambda;
  a.lambda_fp32 = p->lambda_fp32;
  a.no_positivity = p->no_positivity;
  a.kl = p->kl;
  a.lambda_bits = p->lambda_bits;
  a.ub_k = p->bound_mode == HCZ_BOUND_UB ? p->ub_level : -1;
  a.variant = plan->variant;
  a.k_start = p->search == HCZ_SEARCH_BISECT ? -1 : std::min(kLadder - 1, (int)std::floor(4.0 * std::log2(G.L + 1.0) + 0.5));
  a.flags = out->flags;
  a.sizes = (uint64_t*)(ws + L.sizes);
  a.slots = ws + L.slots;
  a.slot_stride = (long long)slot_stride(G, dtype);
  a.kstar = ws + L.kstar;
  a.iters = (uint16_t*)(ws + L.iters);
  a.lam0 = lam0;
  a.analytic = p->warm_start == HCZ_WARM_ANALYTIC;
  a.t_done = (unsigned long long*)out->t_done;
  return a;
}

// After the residual kernel: exclusive scan of the record sizes, compaction into the
// stream, statistics.
static hcz_status residual_finish(const hcz_plan* plan, const ResidualArgs& a, int64_t H, hcz_compressed* out,
                                  uint8_t* ws, const WsLayout& L, hipStream_t st) {
  hcz_ctx* c = plan->ctx;
  {
    StageTimer tm(c, HCZ_STAGE_SCAN, st);
    HCZ_TRY(launch_scan(a.sizes, out->res_offset, H, (uint64_t*)(ws + L.partial), st), "scan launch");
  }
  {
    StageTimer tm(c, HCZ_STAGE_COMPACT, st);
    HCZ_TRY(launch_compact(a.slots, a.slot_stride, out->res_offset, a.sizes, H, out->res_bytes,
                           out->res_capacity, st), "compact launch");
  }
  {
    StageTimer tm(c, HCZ_STAGE_STATS, st);
    HCZ_TRY(launch_stats(out->flags, a.kstar, a.iters, out->res_offset, H, out->res_capacity, out->stats, st),
            "stats launch");
  }
  return HCZ_OK;
}

static hcz_status residual_impl(const hcz_plan* plan, const hcz_params* p, const void* hist,
                                int32_t dtype, int64_t H, int64_t hs, int64_t rs, const float* fhat,
                                const double* lam0, hcz_compressed* out, uint8_t* ws, const WsLayout& L,
                                hipStream_t st) {
  const ResidualArgs a = residual_args(plan, p, hist, dtype, H, hs, rs, fhat, lam0, out, ws, L);
  {
    StageTimer tm(plan->ctx, HCZ_STAGE_RESIDUAL, st);
    HCZ_TRY(launch_residual(plan->G, a, st), "residual launch");
  }
  return residual_finish(plan, a, H, out, ws, L, st);
}

static hcz_status check_out(const hcz_compressed* out, int64_t H, bool codes) {
  if (!out) return fail(HCZ_EINVAL, "out is NULL");
  if (!out->res_offset || !out->stats) return fail(HCZ_EINVAL, "res_offset or stats is NULL");
  if (H > 0 && (!out->lambda || !out->flags)) return fail(HCZ_EINVAL, "lambda or flags is NULL");
  if (out->lambda_fp32 != 0 && out->lambda_fp32 != 1) return fail(HCZ_EINVAL, "lambda_fp32 must be 0 or 1");
  if (H > 0 && codes && !out->codes) return fail(HCZ_EINVAL, "codes is NULL");
  if (out->res_capacity > 0 && !out->res_bytes) return fail(HCZ_EINVAL, "res_bytes is NULL");
  return HCZ_OK;
}

hcz_status hcz_residual(const hcz_plan* plan, const hcz_params* params, const void* hist,
                        int32_t dtype, int64_t H, int64_t hist_stride, int64_t row_stride,
                        const float* fhat, const double* lam0, hcz_compressed* out, void* ws,
                        size_t ws_bytes, hcz_stream_t stream) {
  if (!plan) return fail(HCZ_EINVAL, "plan is NULL");
  hcz_status s;
  if ((s = check_params(params)) || (s = check_hist(hist, dtype, H, hist_stride, row_stride, plan->G)) ||
      (s = check_out(out, H, false)))
    return s;
  if (out->lambda_fp32 != params->lambda_fp32) return fail(HCZ_EINVAL, "out->lambda_fp32 differs from params");
  if (lam0 && params->warm_start == HCZ_WARM_ANALYTIC)
    return fail(HCZ_EINVAL, "lam0 is not given with the analytic start");
  const WsLayout L = ws_layout(plan->G, false, H, dtype, false, 1);
  if (!ws || ws_bytes < L.total) return fail(HCZ_EWORKSPACE, "workspace %zu < %zu", ws_bytes, L.total);
  if ((s = set_device(plan->ctx))) return s;
  prof_begin(plan->ctx);
  return residual_impl(plan, params, hist, dtype, H, hist_stride, row_stride, fhat, lam0, out,
                       (uint8_t*)ws, L, (hipStream_t)stream);
}

static hcz_status compress_impl(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                                const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                                int64_t hist_stride, int64_t row_stride, hcz_compressed* out, void* ws,
                                size_t ws_bytes, hcz_stream_t stream);

hcz_status hcz_compress(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                        const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                        int64_t hist_stride, int64_t row_stride, hcz_compressed* out, void* ws,
                        size_t ws_bytes, hcz_stream_t stream) {
  return compress_impl(plan, model, cb, params, hist, dtype, H, hist_stride, row_stride, out, ws, ws_bytes,
                       stream);
}

hcz_status hcz_compress_static(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                               const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                               int64_t hist_stride, int64_t row_stride, hcz_compressed* out,
                               hcz_stream_t stream) {
  if (!plan) return fail(HCZ_EINVAL, "plan is NULL");
  if (!plan->ctx->scratch) return fail(HCZ_EHIP, "no scratch address for device %d", plan->ctx->device);
  if (params && H >= 0 && (dtype == HCZ_F32 || dtype == HCZ_F64)) {
    const bool fit = model && params->fit_codebook;
    const size_t need = ws_layout(plan->G, model != nullptr, H, dtype, fit, std::max(params->sample_every, 1)).total;
    if (need > (size_t)HCZ_STATIC_SCRATCH_BYTES) {
      int64_t lo = 0, hi = H;   // largest batch whose workspace fits, for the message
      while (lo < hi) {
        const int64_t mid = lo + (hi - lo + 1) / 2;
        if (ws_layout(plan->G, model != nullptr, mid, dtype, fit, std::max(params->sample_every, 1)).total <=
            (size_t)HCZ_STATIC_SCRATCH_BYTES)
          lo = mid;
        else
          hi = mid - 1;
      }
      return fail(HCZ_EWORKSPACE,
                  "hcz_compress_static: %lld histograms need %zu bytes of workspace, more than the %u-byte "
                  "static scratch; at most %lld histograms of this grid, model and dtype fit",
                  (long long)H, need, (unsigned)HCZ_STATIC_SCRATCH_BYTES, (long long)lo);
    }
  }
  return compress_impl(plan, model, cb, params, hist, dtype, H, hist_stride, row_stride, out, plan->ctx->scratch,
                       (size_t)HCZ_STATIC_SCRATCH_BYTES, stream);
}

// The argument checks of hcz_compress; on success *L_out is the workspace layout.
static hcz_status compress_check(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                                 const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                                 int64_t hist_stride, int64_t row_stride, hcz_compressed* out, void* ws,
                                 size_t ws_bytes, WsLayout* L_out) {
  if (!plan) return fail(HCZ_EINVAL, "plan is NULL");
  if (model && model->plan->G.N != plan->G.N) return fail(HCZ_EINVAL, "model was loaded for another grid");
  hcz_status s;
  if ((s = check_params(params)) || (s = check_hist(hist, dtype, H, hist_stride, row_stride, plan->G)) ||
      (s = check_out(out, H, model != nullptr)))
    return s;
  if (out->lambda_fp32 != params->lambda_fp32) return fail(HCZ_EINVAL, "out->lambda_fp32 differs from params");
  if (model && (s = check_cb(cb))) return s;
  const bool fit = model && params->fit_codebook;
  const WsLayout L = ws_layout(plan->G, model != nullptr, H, dtype, fit, params->sample_every);
  if (!ws || ws_bytes < L.total) return fail(HCZ_EWORKSPACE, "workspace %zu < %zu", ws_bytes, L.total);
  *L_out = L;
  return HCZ_OK;
}

// The model stages of hcz_compress (encode, codebook fit, quantise, decode, warm start) on
// checked arguments, the device already current: *fhat and *lam0 are what the residual
// stage reads.
static hcz_status compress_model_stages(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                                        const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                                        int64_t hist_stride, int64_t row_stride, hcz_compressed* out,
                                        uint8_t* w, const WsLayout& L, hipStream_t st, const float** fhat_out,
                                        const double** lam0_out) {
  const bool fit = model && params->fit_codebook;
  const float* fhat = nullptr;
  hcz_ctx* c = plan->ctx;
  const double* lam0 = nullptr;
  if (model && H > 0) {
    float* z = (float*)(w + L.z);
    float* fh = (float*)(w + L.fhat);
    {
      StageTimer tm(c, HCZ_STAGE_ENCODE, st);
      HCZ_TRY(launch_encode(model->M, hist, dtype, H, hist_stride, row_stride, plan->G.n_par, z, st), "encode launch");
    }
    if (fit) {
      StageTimer tm(c, HCZ_STAGE_CODEBOOK, st);
      HCZ_TRY(launch_codebook_fit(z, H, kLatent, params->sample_every, cb->bits, cb->centroids, w + L.cbws, st),
              "codebook launch");
    }
    {
      StageTimer tm(c, HCZ_STAGE_QUANTIZE, st);
      HCZ_TRY(launch_quantize(z, H, kLatent, cb->centroids, cb->bits, out->codes, st), "quantize launch");
    }
    {
      StageTimer tm(c, HCZ_STAGE_DECODE, st);
      HCZ_TRY(launch_decode(model->M, out->codes, cb->centroids, cb->bits, H, fh, st), "decode launch");
    }
    fhat = fh;
    if (params->warm_start == HCZ_WARM_MLP) {
      StageTimer tm(c, HCZ_STAGE_WARMSTART, st);
      lam0 = (const double*)(w + L.lam0);
      HCZ_TRY(launch_mlp_infer(params->mlp->params, params->mlp->scale, out->codes, cb->centroids, cb->bits, H,
                               (double*)(w + L.lam0), st), "warm start launch");
    }
  }
  *fhat_out = fhat;
  *lam0_out = lam0;
  return HCZ_OK;
}

static hcz_status compress_impl(const hcz_plan* plan, const hcz_model* model, hcz_codebook* cb,
                                const hcz_params* params, const void* hist, int32_t dtype, int64_t H,
                                int64_t hist_stride, int64_t row_stride, hcz_compressed* out, void* ws,
                                size_t ws_bytes, hcz_stream_t stream) {
  hipStream_t st = (hipStream_t)stream;
  WsLayout L{};
  hcz_status s = compress_check(plan, model, cb, params, hist, dtype, H, hist_stride, row_stride, out, ws, ws_bytes, &L);
  if (s || (s = set_device(plan->ctx))) return s;
  prof_begin(plan->ctx);
  const float* fhat = nullptr;
  const double* lam0 = nullptr;
  if ((s = compress_model_stages(plan, model, cb, params, hist, dtype, H, hist_stride, row_stride, out, (uint8_t*)ws,
                                 L, st, &fhat, &lam0)))
    return s;
  return residual_impl(plan, params, hist, dtype, H, hist_stride, row_stride, fhat, lam0, out, (uint8_t*)ws, L, st);
}

hcz_status hcz_compress_batch(const hcz_batch_segment* seg, int32_t nseg, void* batch_ws, size_t batch_ws_bytes,
                              hcz_stream_t stream) {
  if (!seg) return fail(HCZ_EINVAL, "seg is NULL");
  if (nseg < 1 || nseg > HCZ_BATCH_MAX_SEGMENTS) return fail(HCZ_EINVAL, "nseg %d not in [1, %d]", nseg, HCZ_BATCH_MAX_SEGMENTS);
  if (!batch_ws || batch_ws_bytes < HCZ_BATCH_WORKSPACE_BYTES)
    return fail(HCZ_EWORKSPACE, "batch workspace %zu < %d", batch_ws_bytes, HCZ_BATCH_WORKSPACE_BYTES);
  static_assert(kBatchSeg == HCZ_BATCH_MAX_SEGMENTS, "segment count of the batch launch");
  WsLayout L[kBatchSeg];
  BatchArgs B{};
  hcz_status s;
  // every check before the first launch
  for (int k = 0; k < nseg; ++k) {
    const hcz_batch_segment& q = seg[k];
    if ((s = compress_check(q.plan, q.model, q.codebook, q.params, q.hist, q.dtype, q.H, q.hist_stride, q.row_stride,
                            q.out, q.ws, q.ws_bytes, &L[k])))
      return s;
    const GridDev& G = q.plan->G;
    if (q.plan->ctx != seg[0].plan->ctx) return fail(HCZ_EINVAL, "segment %d: plan of another context", k);
    if (q.dtype != seg[0].dtype) return fail(HCZ_EINVAL, "segment %d: dtype differs from segment 0", k);
    if (G.uniform_vol != seg[0].plan->G.uniform_vol)
      return fail(HCZ_EUNSUPPORTED, "segment %d: uniform and non-uniform cell volumes in one batch", k);
    if (q.params->kl) return fail(HCZ_EUNSUPPORTED, "segment %d: the KL reading is not batched", k);
    if (!wave_path(G) && !team_path(G, 4))
      return fail(HCZ_EUNSUPPORTED, "segment %d: grid %d x %d fits neither one wave nor a team of four", k, G.n_par,
                  G.n_perp);
  }
  hcz_ctx* c = seg[0].plan->ctx;
  if ((s = set_device(c))) return s;
  hipStream_t st = (hipStream_t)stream;
  prof_begin(c);
  ProfSet* prof = c->cur;
  c->cur = nullptr;            // only the batch's residual launch is timed
  for (int k = 0; k < nseg; ++k) {
    const hcz_batch_segment& q = seg[k];
    const float* fhat = nullptr;
    const double* lam0 = nullptr;
    uint8_t* w = (uint8_t*)q.ws;
    if ((s = compress_model_stages(q.plan, q.model, q.codebook, q.params, q.hist, q.dtype, q.H, q.hist_stride,
                                   q.row_stride, q.out, w, L[k], st, &fhat, &lam0)))
      return s;
    BatchSeg& S = B.s[k];
    S.G = q.plan->G;
    S.a = residual_args(q.plan, q.params, q.hist, q.dtype, q.H, q.hist_stride, q.row_stride, fhat, lam0, q.out, w, L[k]);
    S.kind = wave_path(S.G) ? kBatchWave : kBatchTeam4;
  }
  B.nseg = nseg;
  B.counter = (unsigned long long*)batch_ws;
  {
    c->cur = prof;
    StageTimer tm(c, HCZ_STAGE_RESIDUAL, st);
    HCZ_TRY(launch_residual_batch(B, seg[0].dtype, seg[0].plan->G.uniform_vol != 0, 0, st), "batch residual launch");
  }
  c->cur = nullptr;
  for (int k = 0; k < nseg; ++k)
    if ((s = residual_finish(seg[k].plan, B.s[k].a, seg[k].H, seg[k].out, (uint8_t*)seg[k].ws, L[k], st))) return s;
  return HCZ_OK;
}

hcz_status hcz_decompress(const hcz_plan* plan, const hcz_model* model, const hcz_codebook* cb,
                          const hcz_compressed* in, int32_t in_dtype, int64_t H, void* out,
                          int32_t out_dtype, void* ws, size_t ws_bytes, hcz_stream_t stream) {
  if (!plan || !in) return fail(HCZ_EINVAL, "NULL argument");
  if (H < 0) return fail(HCZ_EINVAL, "H < 0");
  if (in_dtype != HCZ_F32 && in_dtype != HCZ_F64) return fail(HCZ_EINVAL, "in_dtype");
  if (out_dtype != HCZ_F32 && out_dtype != HCZ_F64) return fail(HCZ_EINVAL, "out_dtype");
  if (H > 0 && (!out || !in->flags || !in->lambda || !in->res_offset)) return fail(HCZ_EINVAL, "NULL buffer");
  if (in->lambda_fp32 != 0 && in->lambda_fp32 != 1) return fail(HCZ_EINVAL, "lambda_fp32 must be 0 or 1");
  if (in->res_capacity > 0 && !in->res_bytes) return fail(HCZ_EINVAL, "res_bytes is NULL");
  if (model && model->plan->G.N != plan->G.N) return fail(HCZ_EINVAL, "model was loaded for another grid");
  hcz_status s;
  if (model && ((s = check_cb(cb)) || (H > 0 && !in->codes && (s = fail(HCZ_EINVAL, "codes is NULL")))))
    return s;
  const size_t need = model ? align256((size_t)H * plan->G.N * 4) : 0;
  if (need && (!ws || ws_bytes < need)) return fail(HCZ_EWORKSPACE, "workspace %zu < %zu", ws_bytes, need);
  if ((s = set_device(plan->ctx))) return s;
  hipStream_t st = (hipStream_t)stream;
  const float* fhat = nullptr;
  hcz_ctx* c = plan->ctx;
  prof_begin(c);
  if (model && H > 0) {
    StageTimer tm(c, HCZ_STAGE_DECODE, st);
    HCZ_TRY(launch_decode(model->M, in->codes, cb->centroids, cb->bits, H, (float*)ws, st), "decode launch");
    fhat = (const float*)ws;
  }
  DecompressArgs a{};
  a.flags = in->flags;
  a.lambda = in->lambda;
  a.lambda_fp32 = in->lambda_fp32;
  a.offsets = in->res_offset;
  a.stream = in->res_bytes;
  a.in_dtype = in_dtype;
  a.H = H;
  a.fhat = fhat;
  a.out = out;
  a.out_dtype = out_dtype;
  a.capacity = in->res_capacity;
  StageTimer tm(c, HCZ_STAGE_DECOMPRESS, st);
  HCZ_TRY(launch_decompress(plan->G, a, st), "decompress launch");
  return HCZ_OK;
}

// ---- training ------------------------------------------------------------------------
namespace {
struct AeOffsets {
  size_t W1, b1, W2, b2, W3, b3, W4, b4, total;
};
AeOffsets ae_offsets(int N) {
  AeOffsets o{};
  size_t p = 0;
  o.W1 = p; p += (size_t)kHidden * N;
  o.b1 = p; p += kHidden;
  o.W2 = p; p += (size_t)kLatent * kHidden;
  o.b2 = p; p += kLatent;
  o.W3 = p; p += (size_t)kHidden * kLatent;
  o.b3 = p; p += kHidden;
  o.W4 = p; p += (size_t)N * kHidden;
  o.b4 = p; p += N;
  o.total = p;
  return o;
}
size_t ae_saved_floats(long long B) { return (size_t)B * (3 * kHidden + kHidden + kLatent); }
}  // namespace

hcz_status hcz_ae_param_count(int32_t N, int64_t* count) {
  if (!count || N < 1 || N > kMaxN) return fail(HCZ_EINVAL, "bad argument");
  *count = (int64_t)ae_offsets(N).total;
  return HCZ_OK;
}

hcz_status hcz_ae_saved_bytes(int32_t N, int64_t B, size_t* bytes) {
  if (!bytes || N < 1 || N > kMaxN || B < 0) return fail(HCZ_EINVAL, "bad argument");
  *bytes = ae_saved_floats(B) * sizeof(float);
  return HCZ_OK;
}

hcz_status hcz_ae_forward(int32_t N, int32_t compute, const float* params, const float* x, int64_t B, float* z,
                          float* xhat, void* saved, size_t saved_bytes, hcz_stream_t stream) {
  if (N < 1 || N > kMaxN || B < 0) return fail(HCZ_EINVAL, "bad size");
  if (compute != HCZ_COMPUTE_FP32 && compute != HCZ_COMPUTE_BF16) return fail(HCZ_EINVAL, "compute");
  if (B == 0) return HCZ_OK;
  if (!params || !x || !z || !xhat || !saved) return fail(HCZ_EINVAL, "NULL buffer");
  if (saved_bytes < ae_saved_floats(B) * sizeof(float)) return fail(HCZ_EWORKSPACE, "saved buffer too small");
  const AeOffsets o = ae_offsets(N);
  hipStream_t st = (hipStream_t)stream;
  float* h1 = (float*)saved;
  float* h3 = h1 + (size_t)B * kHidden;
  const int Hd = kHidden, Ld = kLatent;
  const int bf = compute == HCZ_COMPUTE_BF16;
  HCZ_TRY(launch_gemm(x, N, 1, params + o.W1, 1, N, h1, Hd, B, Hd, N, 1.f, 0.f, params + o.b1, 1, st, bf), "gemm");
  HCZ_TRY(launch_gemm(h1, Hd, 1, params + o.W2, 1, Hd, z, Ld, B, Ld, Hd, 1.f, 0.f, params + o.b2, 0, st, bf), "gemm");
  HCZ_TRY(launch_gemm(z, Ld, 1, params + o.W3, 1, Ld, h3, Hd, B, Hd, Ld, 1.f, 0.f, params + o.b3, 1, st, bf), "gemm");
  HCZ_TRY(launch_gemm(h3, Hd, 1, params + o.W4, 1, Hd, xhat, N, B, N, Hd, 1.f, 0.f, params + o.b4, 0, st, bf), "gemm");
  return HCZ_OK;
}

// ---- convolutional model training ----------------------------------------------------------
namespace {
struct ConvOff {
  static constexpr size_t c1w = 0, c1b = 288, c2w = 320, c2b = 18752, fw = 18816, fb = 121216, dw = 121232,
                          db = 223632, t1w = 230032, t1b = 248464, t2w = 248496, t2b = 248784, total = 248785;
};
// saved floats per sample: a1 12800 | a2 6400 | h2 6400 | z 16 | a4 6400 | a5 12800 | T1 12800 | T2 6400 | dz 16
constexpr size_t kConvSaved = 12800 + 6400 + 6400 + 16 + 6400 + 12800 + 12800 + 6400 + 16;
struct ConvSaved {
  float *a1, *a2, *h2, *z, *a4, *a5, *T1, *T2, *dz;
  ConvSaved(void* base, int64_t B) {
    float* p = (float*)base;
    a1 = p; p += (size_t)B * 12800;
    a2 = p; p += (size_t)B * 6400;
    h2 = p; p += (size_t)B * 6400;
    z = p; p += (size_t)B * 16;
    a4 = p; p += (size_t)B * 6400;
    a5 = p; p += (size_t)B * 12800;
    T1 = p; p += (size_t)B * 12800;
    T2 = p; p += (size_t)B * 6400;
    dz = p;
  }
};
}  // namespace

hcz_status hcz_conv_ae_param_count(int64_t* count) {
  if (!count) return fail(HCZ_EINVAL, "NULL argument");
  *count = (int64_t)ConvOff::total;
  return HCZ_OK;
}

hcz_status hcz_conv_ae_saved_bytes(int64_t B, size_t* bytes) {
  if (!bytes || B < 0) return fail(HCZ_EINVAL, "bad argument");
  *bytes = std::max<size_t>((size_t)B * kConvSaved * sizeof(float), 256);
  return HCZ_OK;
}

hcz_status hcz_conv_ae_forward(int32_t compute, const float* params, const float* x, int64_t B, float* z,
                               float* xhat, void* saved, size_t saved_bytes, hcz_stream_t stream) {
  if (B < 0) return fail(HCZ_EINVAL, "bad size");
  if (compute != HCZ_COMPUTE_FP32 && compute != HCZ_COMPUTE_BF16) return fail(HCZ_EINVAL, "compute");
  const int bf = compute == HCZ_COMPUTE_BF16;
  if (B == 0) return HCZ_OK;
  if (!params || !x || !z || !xhat || !saved) return fail(HCZ_EINVAL, "NULL buffer");
  if (saved_bytes < (size_t)B * kConvSaved * sizeof(float)) return fail(HCZ_EWORKSPACE, "saved buffer too small");
  hipStream_t st = (hipStream_t)stream;
  ConvSaved S(saved, B);
  const float* P = params;
  using O = ConvOff;
  HCZ_TRY(launch_cv_fwd(x, 1, 39, 0, P + O::c1w, P + O::c1b, S.a1, 32, 20, B, st, bf), "conv1");
  HCZ_TRY(launch_cv_fwd(S.a1, 32, 20, 1, P + O::c2w, P + O::c2b, S.a2, 64, 10, B, st, bf), "conv2");
  HCZ_TRY(launch_relu_copy(S.a2, S.h2, (long long)B * 6400, st), "relu");
  HCZ_TRY(launch_gemm(S.h2, 6400, 1, P + O::fw, 1, 6400, S.z, 16, B, 16, 6400, 1.f, 0.f, P + O::fb, 0, st, bf), "fc");
  HCZ_TRY(hipMemcpyAsync(z, S.z, (size_t)B * 16 * sizeof(float), hipMemcpyDeviceToDevice, st), "copy z");
  HCZ_TRY(launch_gemm(S.z, 16, 1, P + O::dw, 1, 16, S.a4, 6400, B, 6400, 16, 1.f, 0.f, P + O::db, 0, st, bf), "dfc");
  HCZ_TRY(launch_cvt_fwd(S.a4, 64, 10, 1, P + O::t1w, P + O::t1b, S.a5, 32, 20, B, st, bf), "convT1");
  HCZ_TRY(launch_cvt_fwd(S.a5, 32, 20, 1, P + O::t2w, P + O::t2b, xhat, 1, 39, B, st, bf), "convT2");
  return HCZ_OK;
}

hcz_status hcz_conv_ae_backward(int32_t compute, const float* params, const float* x, int64_t B,
                                const float* dz_in, const float* dxh, void* saved, size_t saved_bytes, float* grad,
                                hcz_stream_t stream) {
  if (B < 0) return fail(HCZ_EINVAL, "bad size");
  if (compute != HCZ_COMPUTE_FP32 && compute != HCZ_COMPUTE_BF16) return fail(HCZ_EINVAL, "compute");
  const int bf = compute == HCZ_COMPUTE_BF16;
  if (!params || !grad) return fail(HCZ_EINVAL, "NULL buffer");
  if (B > 0 && (!x || !dxh || !saved)) return fail(HCZ_EINVAL, "NULL buffer");
  if (saved_bytes < (size_t)B * kConvSaved * sizeof(float)) return fail(HCZ_EWORKSPACE, "saved buffer too small");
  hipStream_t st = (hipStream_t)stream;
  ConvSaved S(saved, B);
  const float* P = params;
  float* G = grad;
  using O = ConvOff;
  // transposed conv2 (32 -> 1)
  HCZ_TRY(launch_cv_fwd(dxh, 1, 39, 0, P + O::t2w, nullptr, S.T1, 32, 20, B, st, bf), "dh5");
  HCZ_TRY(launch_cv_wgrad(S.a5, 32, 20, 1, dxh, 1, 39, 0, B, G + O::t2w, st, bf), "dt2w");
  HCZ_TRY(launch_chsum(dxh, 1, 1521, B, G + O::t2b, st), "dt2b");
  HCZ_TRY(launch_relu_mask(S.T1, S.a5, (long long)B * 12800, st), "relu mask");
  // transposed conv1 (64 -> 32)
  HCZ_TRY(launch_cv_wgrad(S.a4, 64, 10, 1, S.T1, 32, 20, 0, B, G + O::t1w, st, bf), "dt1w");
  HCZ_TRY(launch_chsum(S.T1, 32, 400, B, G + O::t1b, st), "dt1b");
  HCZ_TRY(launch_cv_fwd(S.T1, 32, 20, 0, P + O::t1w, nullptr, S.T2, 64, 10, B, st, bf), "dh4");
  HCZ_TRY(launch_relu_mask(S.T2, S.a4, (long long)B * 6400, st), "relu mask");
  // decoder dense layer (16 -> 6400)
  HCZ_TRY(launch_gemm(S.T2, 1, 6400, S.z, 16, 1, G + O::dw, 16, 6400, 16, B, 1.f, 0.f, nullptr, 0, st, bf), "ddw");
  HCZ_TRY(launch_colsum(S.T2, B, 6400, G + O::db, st), "ddb");
  if (dz_in) {
    HCZ_TRY(hipMemcpyAsync(S.dz, dz_in, (size_t)B * 16 * sizeof(float), hipMemcpyDeviceToDevice, st), "copy dz");
    HCZ_TRY(launch_gemm(S.T2, 6400, 1, P + O::dw, 16, 1, S.dz, 16, B, 16, 6400, 1.f, 1.f, nullptr, 0, st, bf), "dz");
  } else {
    HCZ_TRY(launch_gemm(S.T2, 6400, 1, P + O::dw, 16, 1, S.dz, 16, B, 16, 6400, 1.f, 0.f, nullptr, 0, st, bf), "dz");
  }
  // encoder dense layer (6400 -> 16)
  HCZ_TRY(launch_gemm(S.dz, 1, 16, S.h2, 6400, 1, G + O::fw, 6400, 16, 6400, B, 1.f, 0.f, nullptr, 0, st, bf), "dfw");
  HCZ_TRY(launch_colsum(S.dz, B, 16, G + O::fb, st), "dfb");
  HCZ_TRY(launch_gemm(S.dz, 16, 1, P + O::fw, 6400, 1, S.T2, 6400, B, 6400, 16, 1.f, 0.f, nullptr, 0, st, bf), "dh2");
  HCZ_TRY(launch_relu_mask(S.T2, S.a2, (long long)B * 6400, st), "relu mask");
  // conv2 (32 -> 64)
  HCZ_TRY(launch_cv_wgrad(S.T2, 64, 10, 0, S.a1, 32, 20, 1, B, G + O::c2w, st, bf), "dc2w");
  HCZ_TRY(launch_chsum(S.T2, 64, 100, B, G + O::c2b, st), "dc2b");
  HCZ_TRY(launch_cvt_fwd(S.T2, 64, 10, 0, P + O::c2w, nullptr, S.T1, 32, 20, B, st, bf), "dh1");
  HCZ_TRY(launch_relu_mask(S.T1, S.a1, (long long)B * 12800, st), "relu mask");
  // conv1 (1 -> 32)
  HCZ_TRY(launch_cv_wgrad(S.T1, 32, 20, 0, x, 1, 39, 0, B, G + O::c1w, st, bf), "dc1w");
  HCZ_TRY(launch_chsum(S.T1, 32, 400, B, G + O::c1b, st), "dc1b");
  return HCZ_OK;
}

hcz_status hcz_ae_backward(int32_t N, int32_t compute, const float* params, const float* x, int64_t B,
                           const float* dz_in, const float* dxh, void* saved, size_t saved_bytes,
                           float* grad, float* dx, hcz_stream_t stream) {
  if (N < 1 || N > kMaxN || B < 0) return fail(HCZ_EINVAL, "bad size");
  if (compute != HCZ_COMPUTE_FP32 && compute != HCZ_COMPUTE_BF16) return fail(HCZ_EINVAL, "compute");
  if (!params || !grad) return fail(HCZ_EINVAL, "NULL buffer");
  if (B > 0 && (!x || !dxh || !saved)) return fail(HCZ_EINVAL, "NULL buffer");
  if (saved_bytes < ae_saved_floats(B) * sizeof(float)) return fail(HCZ_EWORKSPACE, "saved buffer too small");
  const AeOffsets o = ae_offsets(N);
  hipStream_t st = (hipStream_t)stream;
  const int Hd = kHidden, Ld = kLatent;
  const int bf = compute == HCZ_COMPUTE_BF16;
  float* h1 = (float*)saved;
  float* h3 = h1 + (size_t)B * Hd;
  float* d3 = h3 + (size_t)B * Hd;      // dL/d(pre-activation 3), [B][Hd]
  float* d1 = d3 + (size_t)B * Hd;      // dL/d(pre-activation 1), [B][Hd]
  float* dz = d1 + (size_t)B * Hd;      // dL/dz, [B][Ld]
  // z is needed for dW3: recompute it from h1 (cheap) into dz's slot first
  HCZ_TRY(launch_gemm(h1, Hd, 1, params + o.W2, 1, Hd, dz, Ld, B, Ld, Hd, 1.f, 0.f, params + o.b2, 0, st, bf), "gemm");
  // output layer
  HCZ_TRY(launch_gemm(dxh, 1, N, h3, Hd, 1, grad + o.W4, Hd, N, Hd, B, 1.f, 0.f, nullptr, 0, st, bf), "gemm dW4");
  HCZ_TRY(launch_colsum(dxh, B, N, grad + o.b4, st), "colsum");
  HCZ_TRY(launch_gemm(dxh, N, 1, params + o.W4, Hd, 1, d3, Hd, B, Hd, N, 1.f, 0.f, nullptr, 0, st, bf), "gemm dh3");
  HCZ_TRY(launch_relu_mask(d3, h3, (long long)B * Hd, st), "relu mask");
  // decoder input layer: dW3 = d3^T z
  HCZ_TRY(launch_gemm(d3, 1, Hd, dz, Ld, 1, grad + o.W3, Ld, Hd, Ld, B, 1.f, 0.f, nullptr, 0, st, bf), "gemm dW3");
  HCZ_TRY(launch_colsum(d3, B, Hd, grad + o.b3, st), "colsum");
  // dz = d3 W3 (+ dz_in)
  if (dz_in) {
    HCZ_TRY(hipMemcpyAsync(dz, dz_in, (size_t)B * Ld * sizeof(float), hipMemcpyDeviceToDevice, st), "copy dz");
    HCZ_TRY(launch_gemm(d3, Hd, 1, params + o.W3, Ld, 1, dz, Ld, B, Ld, Hd, 1.f, 1.f, nullptr, 0, st, bf), "gemm dz");
  } else {
    HCZ_TRY(launch_gemm(d3, Hd, 1, params + o.W3, Ld, 1, dz, Ld, B, Ld, Hd, 1.f, 0.f, nullptr, 0, st, bf), "gemm dz");
  }
  // encoder output layer
  HCZ_TRY(launch_gemm(dz, 1, Ld, h1, Hd, 1, grad + o.W2, Hd, Ld, Hd, B, 1.f, 0.f, nullptr, 0, st, bf), "gemm dW2");
  HCZ_TRY(launch_colsum(dz, B, Ld, grad + o.b2, st), "colsum");
  HCZ_TRY(launch_gemm(dz, Ld, 1, params + o.W2, Hd, 1, d1, Hd, B, Hd, Ld, 1.f, 0.f, nullptr, 0, st, bf), "gemm dh1");
  HCZ_TRY(launch_relu_mask(d1, h1, (long long)B * Hd, st), "relu mask");
  // encoder input layer
  HCZ_TRY(launch_gemm(d1, 1, Hd, x, N, 1, grad + o.W1, N, Hd, N, B, 1.f, 0.f, nullptr, 0, st, bf), "gemm dW1");
  HCZ_TRY(launch_colsum(d1, B, Hd, grad + o.b1, st), "colsum");
  if (dx) HCZ_TRY(launch_gemm(d1, Hd, 1, params + o.W1, N, 1, dx, N, B, N, Hd, 1.f, 0.f, nullptr, 0, st, bf), "gemm dx");
  return HCZ_OK;
}

hcz_status hcz_mse_workspace(size_t* bytes) {
  if (!bytes) return fail(HCZ_EINVAL, "NULL argument");
  *bytes = mse_ws_bytes();
  return HCZ_OK;
}

hcz_status hcz_mse(const float* xhat, const float* x, int64_t n, float* loss, float* dxhat, void* ws,
                   size_t ws_bytes, hcz_stream_t stream) {
  if (n < 1 || !xhat || !x || !loss) return fail(HCZ_EINVAL, "bad argument");
  if (!ws || ws_bytes < mse_ws_bytes()) return fail(HCZ_EWORKSPACE, "workspace too small");
  HCZ_TRY(launch_mse(xhat, x, n, loss, dxhat, ws, (hipStream_t)stream), "mse");
  return HCZ_OK;
}

hcz_status hcz_adam_step(float* params, const float* grad, float* m, float* v, int64_t n, double lr,
                         double beta1, double beta2, double eps, int64_t step, hcz_stream_t stream) {
  if (n < 0 || step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(HCZ_EINVAL, "bad Adam argument");
  if (n > 0 && (!params || !grad || !m || !v)) return fail(HCZ_EINVAL, "NULL buffer");
  HCZ_TRY(launch_adam(params, grad, m, v, n, lr, beta1, beta2, eps, step, (hipStream_t)stream), "adam");
  return HCZ_OK;
}

hcz_status hcz_norm_stats_workspace(const hcz_plan* plan, int64_t H, size_t* bytes) {
  if (!plan || !bytes || H < 1) return fail(HCZ_EINVAL, "bad argument");
  *bytes = norm_stats_ws_bytes(H, plan->G.N);
  return HCZ_OK;
}

hcz_status hcz_norm_stats(const hcz_plan* plan, const void* hist, int32_t dtype, int64_t H,
                          int64_t hist_stride, int64_t row_stride, float* mean, float* sd, void* ws,
                          size_t ws_bytes, hcz_stream_t stream) {
  if (!plan) return fail(HCZ_EINVAL, "plan is NULL");
  if (H < 1) return fail(HCZ_EINVAL, "H must be >= 1");
  hcz_status s = check_hist(hist, dtype, H, hist_stride, row_stride, plan->G);
  if (s) return s;
  if (!mean || !sd) return fail(HCZ_EINVAL, "NULL output");
  if (!ws || ws_bytes < norm_stats_ws_bytes(H, plan->G.N)) return fail(HCZ_EWORKSPACE, "workspace too small");
  if ((s = set_device(plan->ctx))) return s;
  HCZ_TRY(launch_norm_stats(hist, dtype, H, hist_stride, row_stride, plan->G.n_par, plan->G.N, mean, sd, ws,
                            (hipStream_t)stream), "norm stats");
  return HCZ_OK;
}

hcz_status hcz_column_stats_workspace(int64_t rows, int64_t cols, size_t* bytes) {
  if (!bytes || rows < 1 || cols < 1 || cols > INT32_MAX) return fail(HCZ_EINVAL, "bad argument");
  *bytes = norm_stats_ws_bytes(rows, (int)cols);
  return HCZ_OK;
}

hcz_status hcz_column_stats(const void* x, int32_t dtype, int64_t rows, int64_t cols, int64_t ld, float* mean,
                            float* sd, void* ws, size_t ws_bytes, hcz_stream_t stream) {
  if (!x || !mean || !sd) return fail(HCZ_EINVAL, "NULL argument");
  if (dtype != HCZ_F32 && dtype != HCZ_F64) return fail(HCZ_EINVAL, "dtype");
  if (rows < 1 || cols < 1 || cols > INT32_MAX || ld < cols) return fail(HCZ_EINVAL, "bad shape");
  if (!ws || ws_bytes < norm_stats_ws_bytes(rows, (int)cols)) return fail(HCZ_EWORKSPACE, "workspace too small");
  // one row of `cols` elements per "histogram": the statistics kernel's (n_par = N = cols) case
  HCZ_TRY(launch_norm_stats(x, dtype, rows, ld, cols, (int)cols, (int)cols, mean, sd, ws, (hipStream_t)stream),
          "column stats");
  return HCZ_OK;
}

hcz_status hcz_column_normalize(const void* x, int32_t dtype, int64_t rows, int64_t cols, int64_t ld,
                                const float* mean, const float* sd, float* out, hcz_stream_t stream) {
  if (rows < 0 || cols < 0 || ld < cols) return fail(HCZ_EINVAL, "bad shape");
  if (dtype != HCZ_F32 && dtype != HCZ_F64) return fail(HCZ_EINVAL, "dtype");
  if (rows * cols > 0 && (!x || !sd || !out)) return fail(HCZ_EINVAL, "NULL argument");
  HCZ_TRY(launch_col_normalize(x, dtype, rows, cols, ld, mean, sd, out, (hipStream_t)stream), "column normalize");
  return HCZ_OK;
}

// ---- warm-start network -------------------------------------------------------------
namespace {
constexpr int kMH = 64, kMI = 16, kMO = 4;
struct MlpOffsets { size_t W1, b1, W2, b2, W3, b3; };
MlpOffsets mlp_offsets() {
  MlpOffsets o{};
  size_t p = 0;
  o.W1 = p; p += kMH * kMI;
  o.b1 = p; p += kMH;
  o.W2 = p; p += kMH * kMH;
  o.b2 = p; p += kMH;
  o.W3 = p; p += kMO * kMH;
  o.b3 = p;
  return o;
}
size_t mlp_saved_floats(long long B) { return (size_t)B * 4 * kMH; }
}  // namespace

hcz_status hcz_mlp_param_count(int64_t* count) {
  if (!count) return fail(HCZ_EINVAL, "NULL argument");
  *count = mlp_param_count();
  return HCZ_OK;
}

hcz_status hcz_mlp_saved_bytes(int64_t B, size_t* bytes) {
  if (!bytes || B < 0) return fail(HCZ_EINVAL, "bad argument");
  *bytes = mlp_saved_floats(B) * sizeof(float);
  return HCZ_OK;
}

hcz_status hcz_mlp_load(hcz_ctx* ctx, const float* params, const double* scale, hcz_mlp** out) {
  if (!ctx || !params || !scale || !out) return fail(HCZ_EINVAL, "NULL argument");
  *out = nullptr;
  for (int k = 0; k < 4; ++k)
    if (!std::isfinite(scale[k])) return fail(HCZ_EINVAL, "scale must be finite");
  hcz_status s = set_device(ctx);
  if (s) return s;
  hcz_mlp* m = new hcz_mlp();
  m->ctx = ctx;
  std::vector<float> pv(params, params + mlp_param_count());
  std::vector<double> sv(scale, scale + 4);
  if ((s = upload(m->allocs, pv, &m->params)) || (s = upload(m->allocs, sv, &m->scale))) {
    free_all(m->allocs);
    delete m;
    return s;
  }
  *out = m;
  return HCZ_OK;
}

void hcz_mlp_free(hcz_mlp* m) {
  if (!m) return;
  free_all(m->allocs);
  delete m;
}

hcz_status hcz_mlp_forward(const float* params, const float* z, int64_t B, float* out, void* saved,
                           size_t saved_bytes, hcz_stream_t stream) {
  if (B < 0) return fail(HCZ_EINVAL, "B < 0");
  if (B == 0) return HCZ_OK;
  if (!params || !z || !out || !saved) return fail(HCZ_EINVAL, "NULL buffer");
  if (saved_bytes < mlp_saved_floats(B) * sizeof(float)) return fail(HCZ_EWORKSPACE, "saved buffer too small");
  const MlpOffsets o = mlp_offsets();
  hipStream_t st = (hipStream_t)stream;
  float* h1 = (float*)saved;
  float* h2 = h1 + (size_t)B * kMH;
  HCZ_TRY(launch_gemm(z, kMI, 1, params + o.W1, 1, kMI, h1, kMH, B, kMH, kMI, 1.f, 0.f, params + o.b1, 1, st), "gemm");
  HCZ_TRY(launch_gemm(h1, kMH, 1, params + o.W2, 1, kMH, h2, kMH, B, kMH, kMH, 1.f, 0.f, params + o.b2, 1, st), "gemm");
  HCZ_TRY(launch_gemm(h2, kMH, 1, params + o.W3, 1, kMH, out, kMO, B, kMO, kMH, 1.f, 0.f, params + o.b3, 0, st), "gemm");
  return HCZ_OK;
}

hcz_status hcz_mlp_backward(const float* params, const float* z, int64_t B, const float* dout, void* saved,
                            size_t saved_bytes, float* grad, hcz_stream_t stream) {
  if (B < 0) return fail(HCZ_EINVAL, "B < 0");
  if (!params || !grad) return fail(HCZ_EINVAL, "NULL buffer");
  if (B > 0 && (!z || !dout || !saved)) return fail(HCZ_EINVAL, "NULL buffer");
  if (saved_bytes < mlp_saved_floats(B) * sizeof(float)) return fail(HCZ_EWORKSPACE, "saved buffer too small");
  const MlpOffsets o = mlp_offsets();
  hipStream_t st = (hipStream_t)stream;
  float* h1 = (float*)saved;
  float* h2 = h1 + (size_t)B * kMH;
  float* d2 = h2 + (size_t)B * kMH;
  float* d1 = d2 + (size_t)B * kMH;
  HCZ_TRY(launch_gemm(dout, 1, kMO, h2, kMH, 1, grad + o.W3, kMH, kMO, kMH, B, 1.f, 0.f, nullptr, 0, st), "gemm");
  HCZ_TRY(launch_colsum(dout, B, kMO, grad + o.b3, st), "colsum");
  HCZ_TRY(launch_gemm(dout, kMO, 1, params + o.W3, kMH, 1, d2, kMH, B, kMH, kMO, 1.f, 0.f, nullptr, 0, st), "gemm");
  HCZ_TRY(launch_relu_mask(d2, h2, (long long)B * kMH, st), "mask");
  HCZ_TRY(launch_gemm(d2, 1, kMH, h1, kMH, 1, grad + o.W2, kMH, kMH, kMH, B, 1.f, 0.f, nullptr, 0, st), "gemm");
  HCZ_TRY(launch_colsum(d2, B, kMH, grad + o.b2, st), "colsum");
  HCZ_TRY(launch_gemm(d2, kMH, 1, params + o.W2, kMH, 1, d1, kMH, B, kMH, kMH, 1.f, 0.f, nullptr, 0, st), "gemm");
  HCZ_TRY(launch_relu_mask(d1, h1, (long long)B * kMH, st), "mask");
  HCZ_TRY(launch_gemm(d1, 1, kMH, z, kMI, 1, grad + o.W1, kMI, kMH, kMI, B, 1.f, 0.f, nullptr, 0, st), "gemm");
  HCZ_TRY(launch_colsum(d1, B, kMH, grad + o.b1, st), "colsum");
  return HCZ_OK;
}

hcz_status hcz_dequantize(const uint8_t* codes, int64_t n, int32_t latent, const hcz_codebook* cb, float* z,
                          hcz_stream_t stream) {
  if (n < 0 || latent < 1) return fail(HCZ_EINVAL, "bad size");
  if (n > 0 && (!codes || !z)) return fail(HCZ_EINVAL, "NULL buffer");
  hcz_status s = check_cb(cb);
  if (s) return s;
  HCZ_TRY(launch_dequant(codes, n, latent, cb->centroids, cb->bits, z, (hipStream_t)stream), "dequant");
  return HCZ_OK;
}

hcz_status hcz_mlp_predict(const hcz_mlp* mlp, const uint8_t* codes, const hcz_codebook* cb, int64_t H,
                           double* lam0, hcz_stream_t stream) {
  if (!mlp || H < 0) return fail(HCZ_EINVAL, "bad argument");
  if (H > 0 && (!codes || !lam0)) return fail(HCZ_EINVAL, "NULL buffer");
  hcz_status s = check_cb(cb);
  if (s) return s;
  HCZ_TRY(launch_mlp_infer(mlp->params, mlp->scale, codes, cb->centroids, cb->bits, H, lam0, (hipStream_t)stream),
          "mlp");
  return HCZ_OK;
}

hcz_status hcz_profile_enable(hcz_ctx* ctx, int enable) {
  if (!ctx) return fail(HCZ_EINVAL, "ctx is NULL");
  hcz_status s = set_device(ctx);
  if (s) return s;
  if (enable && ctx->ring.empty()) {
    ctx->ring.resize(64);
    for (auto& set : ctx->ring) {
      set.live = false;
      for (int k = 0; k < HCZ_NSTAGES; ++k) set.used[k] = false;
      for (auto& e : set.ev) HCZ_TRY(hipEventCreate(&e), "hipEventCreate");
    }
  }
  ctx->prof = enable != 0;
  return HCZ_OK;
}

hcz_status hcz_profile_read(hcz_ctx* ctx, double* ms, int64_t* calls) {
  if (!ctx || !ms || !calls) return fail(HCZ_EINVAL, "NULL argument");
  hcz_status s = set_device(ctx);
  if (s) return s;
  for (auto& set : ctx->ring) prof_fold(ctx, set);
  for (int k = 0; k < HCZ_NSTAGES; ++k) {
    ms[k] = ctx->acc_ms[k];
    calls[k] = ctx->acc_calls[k];
    ctx->acc_ms[k] = 0.0;
    ctx->acc_calls[k] = 0;
  }
  return HCZ_OK;
}

hcz_status hcz_stats_read(const hcz_stats* dev, hcz_stats* host_out, hcz_stream_t stream) {
  if (!dev || !host_out) return fail(HCZ_EINVAL, "NULL argument");
  HCZ_TRY(hipMemcpyAsync(host_out, dev, sizeof(hcz_stats), hipMemcpyDeviceToHost, (hipStream_t)stream),
          "stats copy");
  HCZ_TRY(hipStreamSynchronize((hipStream_t)stream), "stream sync");
  if (host_out->overflow) return fail(HCZ_ECAPACITY, "residual stream needs %llu bytes",
                                      (unsigned long long)host_out->stream_bytes);
  return HCZ_OK;
}

}  // extern "C"
