// The output buffer of one compressed batch (Section III, end of Stage 5): a 44-byte
// header, the autoencoder weights (with the z-score statistics), the quantized codes, the
// PQ table, the residual bytes and the Lagrange multipliers, in that order; plus an
// optional order-0 rANS coding of the codes, the residual bytes and the multipliers.  Host
// code only.
//
// Header (little-endian): magic "HCZ1"; u16 scheme (bits 0-1 architecture: 0 none,
// 1 dense, 2 convolutional; bit 2 BF16 compute; bit 3 FP32 multipliers; bit 4 entropy
// coded; bit 5 residual integers coded; bit 6 FP64 compute); u8 latent; u8 bits; u64 H;
// u16 n_par; u16 n_perp; u32 weight-section bytes; u64 end of the residual section; u64 total size; u32 FNV-1a checksum of the first 40
// header bytes.  Sections start at multiples of 8: weights (FP32 weights, mean, std),
// codes [H][latent] (raw or rANS), PQ table [latent][2^bits] FP32, residual (flags [H],
// record sizes [H] u32, the records back to back, raw or rANS, or with entropy = 2 (scheme
// bit 5) split into headers and per-group integer symbols, see below), multipliers [H][4]
// (raw or rANS).
//
// rANS (Duda's asymmetric numeral systems, range variant, byte-wise renormalisation):
// 32-bit state kept in [2^23, 2^31), symbol frequencies quantised to 12 bits.  A coded
// block is u64 n, u16 freq[256], u64 m, m bytes.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hcz_internal.h"

namespace {

using hcz::set_error;

constexpr uint32_t kScale = 12, kM = 1u << kScale, kL = 1u << 23;
constexpr size_t kHeader = 44;

size_t up8(size_t x) { return (x + 7) & ~(size_t)7; }

uint32_t fnv1a(const uint8_t* p, size_t n) {
  uint32_t h = 2166136261u;
  for (size_t i = 0; i < n; ++i) h = (h ^ p[i]) * 16777619u;
  return h;
}

// counts -> frequencies summing to kM, every present symbol >= 1
void quantise(const uint64_t (&cnt)[256], uint64_t n, uint32_t (&f)[256]) {
  uint32_t sum = 0;
  int big = -1;
  for (int s = 0; s < 256; ++s) {
    f[s] = 0;
    if (!cnt[s]) continue;
    uint64_t q = (cnt[s] * kM + n / 2) / n;
    f[s] = (uint32_t)(q ? q : 1);
    sum += f[s];
    if (big < 0 || cnt[s] > cnt[big]) big = s;
  }
  // move the difference onto the most frequent symbols, keeping each >= 1
  while (sum != kM) {
    int s = big;
    if (sum > kM) {
      for (int t = 0; t < 256; ++t)
        if (f[t] > f[s]) s = t;
      const uint32_t d = std::min(sum - kM, f[s] - 1);
      f[s] -= d;
      sum -= d;
      if (d == 0) break;
    } else {
      f[s] += kM - sum;
      sum = kM;
    }
  }
}

size_t rans_bound(size_t n) { return 8 + 512 + 8 + n + n / 64 + 16; }

// Encode n bytes into out (capacity rans_bound(n)); returns the block size.
size_t rans_encode(const uint8_t* in, size_t n, uint8_t* out) {
  uint64_t cnt[256] = {};
  for (size_t i = 0; i < n; ++i) ++cnt[in[i]];
  uint32_t f[256], c[257];
  if (n) quantise(cnt, n, f);
  else std::memset(f, 0, sizeof f);
  c[0] = 0;
  for (int s = 0; s < 256; ++s) c[s + 1] = c[s] + f[s];
  uint8_t* p = out;
  std::memcpy(p, &n, 8);
  p += 8;
  for (int s = 0; s < 256; ++s) {
    const uint16_t v = (uint16_t)f[s];
    std::memcpy(p + 2 * s, &v, 2);
  }
  p += 512;
  uint8_t* lenp = p;
  p += 8;
  // symbols are coded last to first; the bytes come out in reverse and are flipped
  std::vector<uint8_t> rev;
  rev.reserve(n + 16);
  uint32_t x = kL;
  for (size_t i = n; i-- > 0;) {
    const uint32_t s = in[i], fs = f[s];
    const uint32_t xmax = ((kL >> kScale) << 8) * fs;
    while (x >= xmax) {
      rev.push_back((uint8_t)(x & 0xff));
      x >>= 8;
    }
    x = ((x / fs) << kScale) + (x % fs) + c[s];
  }
  for (int k = 0; k < 4; ++k) {
    rev.push_back((uint8_t)(x & 0xff));
    x >>= 8;
  }
  const uint64_t m = rev.size();
  std::memcpy(lenp, &m, 8);
  for (size_t k = 0; k < rev.size(); ++k) p[k] = rev[rev.size() - 1 - k];
  return (size_t)(p - out) + rev.size();
}

// Decode a block at in (avail bytes) into out (exactly n_expect bytes); false if malformed.
bool rans_decode(const uint8_t* in, size_t avail, uint8_t* out, uint64_t n_expect, size_t* used) {
  if (avail < 528) return false;
  uint64_t n, m;
  std::memcpy(&n, in, 8);
  if (n != n_expect) return false;
  uint32_t f[256], c[257];
  c[0] = 0;
  for (int s = 0; s < 256; ++s) {
    uint16_t v;
    std::memcpy(&v, in + 8 + 2 * s, 2);
    f[s] = v;
    c[s + 1] = c[s] + f[s];
  }
  std::memcpy(&m, in + 520, 8);
  if (m > avail - 528) return false;
  *used = 528 + (size_t)m;
  if (n == 0) return true;
  if (c[256] != kM || m < 4) return false;
  static thread_local std::vector<uint8_t> slot;
  slot.assign(kM, 0);
  for (int s = 0; s < 256; ++s)
    for (uint32_t k = c[s]; k < c[s + 1]; ++k) slot[k] = (uint8_t)s;
  const uint8_t* p = in + 528;
  const uint8_t* end = p + m;
  uint32_t x = 0;
  for (int k = 0; k < 4; ++k) x = (x << 8) | *p++;
  for (uint64_t i = 0; i < n; ++i) {
    const uint32_t r = x & (kM - 1);
    const uint32_t s = slot[r];
    out[i] = (uint8_t)s;
    x = f[s] * (x >> kScale) + r - c[s];
    while (x < kL) {
      if (p >= end) return false;
      x = (x << 8) | *p++;
    }
  }
  return p == end && x == kL;
}

// ---- integer model of the residual records (entropy = 2) ----------------------------
// A coded record is a header (Delta, k*, nlev, one bit width per coefficient group, zero
// padding to 8 bytes) and the zigzag integers of the groups, coarsest first, each with its
// group's width, packed LSB first.  Here the headers and the verbatim records go to one
// byte stream; every integer u becomes its magnitude class c = bit length of u (0 for
// u = 0) as a byte symbol in its group's stream, and the c - 1 bits of u below its leading
// one go to a raw bit stream (LSB first).  The byte streams are rANS coded, each with its
// own table.  Unpacking re-packs the integers with the header's widths, so the records
// come back byte for byte.  The group sizes follow from the grid: with
// G_l(n) = {i : i mod 2^l = 0} U {n - 1} and L = max over both axes of ceil(log2(n - 1)),
// group 0 is G_L x G_L and group L - l + 1 is G_(l-1)^2 minus G_l^2.

size_t set_1d(int n, int l) {
  if (n <= 1) return 1;
  const size_t m = (size_t)(n - 1);
  return (m >> l) + 1 + ((m & (((size_t)1 << l) - 1)) ? 1 : 0);
}

std::vector<size_t> group_counts(int n_par, int n_perp) {
  auto lev = [](int n) { int L = 0; while (n > 1 && (1 << L) < n - 1) ++L; return L; };
  const int L = std::max(lev(n_par), lev(n_perp));
  std::vector<size_t> g;
  g.push_back(set_1d(n_par, L) * set_1d(n_perp, L));
  for (int l = L; l >= 1; --l) g.push_back(set_1d(n_par, l - 1) * set_1d(n_perp, l - 1) - set_1d(n_par, l) * set_1d(n_perp, l));
  return g;
}

struct IntStreams {
  std::vector<uint8_t> side;                 // coded-record headers, verbatim records
  std::vector<std::vector<uint8_t>> sym;     // per group, the magnitude class of each integer
  std::vector<uint8_t> bits;                 // bits below the leading one, LSB first
  uint64_t nbits = 0;
  void put(uint32_t v, int n) {              // append the n low bits of v
    for (int k = 0; k < n; ++k, ++nbits) {
      if ((nbits & 7) == 0) bits.push_back(0);
      bits.back() |= (uint8_t)(((v >> k) & 1u) << (nbits & 7));
    }
  }
};

int bit_length(uint32_t u) { return u ? 32 - __builtin_clz(u) : 0; }

// Record sizes the residual kernels write: a verbatim record holds the N input values (4N
// or 8N bytes), a coded one at least its header, any other histogram none.
bool record_sizes_valid(int n_par, int n_perp, int64_t H, const uint8_t* flags, const uint64_t* off) {
  const size_t N = (size_t)n_par * n_perp;
  const size_t nlev = group_counts(n_par, n_perp).size(), hdr = (10 + nlev + 7) / 8 * 8;
  for (int64_t h = 0; h < H; ++h) {
    if (off[h + 1] < off[h]) return false;
    const size_t size = (size_t)(off[h + 1] - off[h]);
    if (flags[h] & HCZ_FLAG_RAW) {
      if (size != 4 * N && size != 8 * N) return false;
    } else if (flags[h] & HCZ_FLAG_CODED) {
      if (size < hdr) return false;
    } else if (size) {
      return false;
    }
  }
  return true;
}

// Split the records of a batch into the streams; false if a coded record is not in the
// coder's canonical form (nlev, widths <= 32, size, zero padding bits).
bool split_records(int n_par, int n_perp, int64_t H, const uint8_t* flags, const uint64_t* off,
                   const uint8_t* rec, IntStreams* s) {
  const std::vector<size_t> cnt = group_counts(n_par, n_perp);
  const size_t nlev = cnt.size(), hdr = (10 + nlev + 7) / 8 * 8;
  s->sym.assign(nlev, {});
  for (int64_t h = 0; h < H; ++h) {
    const size_t size = (size_t)(off[h + 1] - off[h]);
    if (!size) continue;
    const uint8_t* r = rec + off[h];
    if (flags[h] & HCZ_FLAG_RAW) {
      s->side.insert(s->side.end(), r, r + size);
      continue;
    }
    if (size < hdr || r[9] != nlev) return false;
    size_t bits = 0;
    for (size_t g = 0; g < nlev; ++g) {
      if (r[10 + g] > 32) return false;
      bits += cnt[g] * r[10 + g];
    }
    const size_t pay = 4 * ((bits + 31) / 32);
    if (size != hdr + pay) return false;
    s->side.insert(s->side.end(), r, r + hdr);
    const uint8_t* p = r + hdr;
    size_t pos = 0;
    for (size_t g = 0; g < nlev; ++g) {
      const int w = r[10 + g];
      for (size_t k = 0; k < cnt[g]; ++k) {
        uint64_t win = 0;
        if (w) {
          const size_t b0 = pos >> 3;
          for (size_t j = 0; j < 8 && b0 + j < pay; ++j) win |= (uint64_t)p[b0 + j] << (8 * j);
          win = (win >> (pos & 7)) & ((w == 32) ? 0xffffffffull : ((1ull << w) - 1));
        }
        pos += (size_t)w;
        const uint32_t u = (uint32_t)win;
        const int c = bit_length(u);
        s->sym[g].push_back((uint8_t)c);
        if (c > 1) s->put(u, c - 1);
      }
    }
    // the padding after the last integer must be zero for an exact round trip
    for (size_t q = pos; q < 8 * pay; ++q)
      if ((p[q >> 3] >> (q & 7)) & 1) return false;
  }
  return true;
}

size_t int_streams_bound(const IntStreams& s) {
  size_t b = rans_bound(s.side.size()) + 8 + s.bits.size();
  for (const auto& v : s.sym) b += rans_bound(v.size());
  return b;
}

size_t int_streams_write(const IntStreams& s, uint8_t* out) {
  size_t o = rans_encode(s.side.data(), s.side.size(), out);
  for (const auto& v : s.sym) o += rans_encode(v.data(), v.size(), out + o);
  std::memcpy(out + o, &s.nbits, 8);
  o += 8;
  if (!s.bits.empty()) std::memcpy(out + o, s.bits.data(), s.bits.size());
  return o + s.bits.size();
}

// Rebuild the records from the streams at in[0, avail); sizes and flags from the container.
bool int_streams_read(int n_par, int n_perp, int64_t H, const uint8_t* flags, const uint64_t* off,
                      const uint8_t* in, size_t avail, uint8_t* rec, size_t* used) {
  const std::vector<size_t> cnt = group_counts(n_par, n_perp);
  const size_t nlev = cnt.size(), hdr = (10 + nlev + 7) / 8 * 8;
  // stream lengths: the side bytes and the symbols of each group follow from the records
  size_t side_n = 0;
  std::vector<size_t> sym_n(nlev, 0);
  for (int64_t h = 0; h < H; ++h) {
    const size_t size = (size_t)(off[h + 1] - off[h]);
    if (!size) continue;
    if (flags[h] & HCZ_FLAG_RAW) side_n += size;
    else {
      if (size < hdr) return false;
      side_n += hdr;
      for (size_t g = 0; g < nlev; ++g) sym_n[g] += cnt[g];
    }
  }
  std::vector<uint8_t> side(side_n);
  std::vector<std::vector<uint8_t>> sym(nlev);
  size_t o = 0, u = 0;
  if (!rans_decode(in, avail, side.data(), side_n, &u)) return false;
  o += u;
  for (size_t g = 0; g < nlev; ++g) {
    sym[g].resize(sym_n[g]);
    if (!rans_decode(in + o, avail - o, sym[g].data(), sym_n[g], &u)) return false;
    o += u;
  }
  if (avail - o < 8) return false;
  uint64_t nbits;
  std::memcpy(&nbits, in + o, 8);
  o += 8;
  if (nbits / 8 > avail - o || (nbits + 7) / 8 > avail - o) return false;
  const uint8_t* bits = in + o;
  o += (size_t)((nbits + 7) / 8);
  uint64_t bp = 0;
  size_t si = 0;
  std::vector<size_t> gi(nlev, 0);
  for (int64_t h = 0; h < H; ++h) {
    const size_t size = (size_t)(off[h + 1] - off[h]);
    if (!size) continue;
    uint8_t* r = rec + off[h];
    if (flags[h] & HCZ_FLAG_RAW) {
      std::memcpy(r, side.data() + si, size);
      si += size;
      continue;
    }
    std::memcpy(r, side.data() + si, hdr);
    si += hdr;
    if (r[9] != nlev) return false;
    size_t nb = 0;
    for (size_t g = 0; g < nlev; ++g) {
      if (r[10 + g] > 32) return false;
      nb += cnt[g] * r[10 + g];
    }
    const size_t pay = 4 * ((nb + 31) / 32);
    if (size != hdr + pay) return false;
    uint8_t* p = r + hdr;
    std::memset(p, 0, pay);
    size_t pos = 0;
    for (size_t g = 0; g < nlev; ++g) {
      const int w = r[10 + g];
      for (size_t k = 0; k < cnt[g]; ++k) {
        const int c = sym[g][gi[g]++];
        if (c > w) return false;
        uint32_t v = 0;
        if (c > 0) {
          if (bp + (uint64_t)(c - 1) > nbits) return false;
          v = 1u << (c - 1);
          for (int q = 0; q < c - 1; ++q, ++bp) v |= (uint32_t)((bits[bp >> 3] >> (bp & 7)) & 1u) << q;
        }
        uint64_t win = (uint64_t)v << (pos & 7);
        for (size_t j = 0; win && j < 8; ++j, win >>= 8) p[(pos >> 3) + j] |= (uint8_t)(win & 0xff);
        pos += (size_t)w;
      }
    }
  }
  if (bp != nbits) return false;
  *used = o;
  return true;
}

struct Sizes {
  size_t N, weights, codes_raw, pq, flags, recs, lam;
};

bool sizes_of(const hcz_container_info& i, Sizes* z) {
  if (i.H < 0 || i.n_par < 1 || i.n_perp < 1 || i.n_par > 65535 || i.n_perp > 65535) return false;
  if (i.arch < 0 || i.arch > 2) return false;
  z->N = (size_t)i.n_par * i.n_perp;
  if (i.arch) {
    if (i.latent < 1 || i.latent > 255 || i.bits < 1 || i.bits > 8 || i.n_weights < 1) return false;
    z->weights = 4 * ((size_t)i.n_weights + 2 * z->N);
    if (z->weights > 0xffffffffu) return false;
    z->codes_raw = (size_t)i.H * i.latent;
    z->pq = 4 * (size_t)i.latent << i.bits;
  } else {
    z->weights = z->codes_raw = z->pq = 0;
  }
  z->flags = (size_t)i.H;
  z->recs = 4 * (size_t)i.H;
  z->lam = (size_t)i.H * 4 * (i.lambda_fp32 ? 4 : 8);
  return true;
}

}  // namespace

extern "C" {

hcz_status hcz_rans_bound(size_t n, size_t* bytes) {
  if (!bytes) return set_error(HCZ_EINVAL, "NULL argument");
  *bytes = rans_bound(n);
  return HCZ_OK;
}

hcz_status hcz_rans_encode(const void* in, size_t n, void* out, size_t capacity, size_t* written) {
  if ((n && !in) || !out || !written) return set_error(HCZ_EINVAL, "NULL argument");
  if (capacity < rans_bound(n)) return set_error(HCZ_ECAPACITY, "output smaller than hcz_rans_bound");
  *written = rans_encode((const uint8_t*)in, n, (uint8_t*)out);
  return HCZ_OK;
}

hcz_status hcz_rans_decode(const void* in, size_t avail, void* out, size_t n) {
  if (!in || (n && !out)) return set_error(HCZ_EINVAL, "NULL argument");
  size_t used = 0;
  if (!rans_decode((const uint8_t*)in, avail, (uint8_t*)out, n, &used))
    return set_error(HCZ_EINVAL, "malformed rANS block");
  return HCZ_OK;
}

hcz_status hcz_container_bound(const hcz_container_in* c, size_t* bytes) {
  if (!c || !bytes) return set_error(HCZ_EINVAL, "NULL argument");
  Sizes z;
  if (!sizes_of(c->info, &z)) return set_error(HCZ_EINVAL, "bad container description");
  if (!c->res_offset) return set_error(HCZ_EINVAL, "res_offset is NULL");
  if (c->info.entropy < 0 || c->info.entropy > 2) return set_error(HCZ_EINVAL, "entropy must be 0, 1 or 2");
  if (c->info.H && !c->flags) return set_error(HCZ_EINVAL, "flags is NULL");
  if (!record_sizes_valid(c->info.n_par, c->info.n_perp, c->info.H, c->flags, c->res_offset))
    return set_error(HCZ_EINVAL, "a residual record's size does not fit its flags");
  const size_t rb = (size_t)c->res_offset[c->info.H];
  const size_t codes = c->info.entropy ? rans_bound(z.codes_raw) : z.codes_raw;
  size_t res = c->info.entropy ? rans_bound(rb) : rb;
  if (c->info.entropy == 2) {
    if (c->info.H && (!c->flags || (rb && !c->res_bytes))) return set_error(HCZ_EINVAL, "NULL section");
    IntStreams s;
    if (!split_records(c->info.n_par, c->info.n_perp, c->info.H, c->flags, c->res_offset, c->res_bytes, &s))
      return set_error(HCZ_EINVAL, "a coded residual record is not in the coder's format");
    res = int_streams_bound(s);
  }
  const size_t lam = c->info.entropy ? rans_bound(z.lam) : z.lam;
  *bytes = up8(kHeader) + up8(z.weights) + up8(codes) + up8(z.pq) + up8(z.flags + z.recs + res) + up8(lam);
  return HCZ_OK;
}

hcz_status hcz_container_pack(const hcz_container_in* c, void* out, size_t capacity, size_t* written) {
  size_t need = 0;
  hcz_status st = hcz_container_bound(c, &need);
  if (st) return st;
  if (!out || !written) return set_error(HCZ_EINVAL, "NULL argument");
  if (capacity < need) return set_error(HCZ_ECAPACITY, "output smaller than hcz_container_bound");
  const hcz_container_info& i = c->info;
  Sizes z;
  sizes_of(i, &z);
  const int64_t H = i.H;
  if ((H && (!c->flags || !c->lambda)) || (c->res_offset[H] && !c->res_bytes))
    return set_error(HCZ_EINVAL, "NULL section");
  if (i.arch && (!c->weights || !c->norm_mean || !c->norm_std || (H && !c->codes) || !c->centroids))
    return set_error(HCZ_EINVAL, "NULL model section");
  for (int64_t h = 0; h < H; ++h)
    if (c->res_offset[h + 1] < c->res_offset[h] || c->res_offset[h + 1] - c->res_offset[h] > 0xffffffffu)
      return set_error(HCZ_EINVAL, "res_offset is not an exclusive scan of record sizes");
  uint8_t* b = (uint8_t*)out;
  std::memset(b, 0, need);
  size_t o = up8(kHeader);
  if (i.arch) {
    std::memcpy(b + o, c->weights, 4 * (size_t)i.n_weights);
    std::memcpy(b + o + 4 * (size_t)i.n_weights, c->norm_mean, 4 * z.N);
    std::memcpy(b + o + 4 * ((size_t)i.n_weights + z.N), c->norm_std, 4 * z.N);
    o += up8(z.weights);
    if (i.entropy) o += up8(rans_encode(c->codes, z.codes_raw, b + o));
    else {
      std::memcpy(b + o, c->codes, z.codes_raw);
      o += up8(z.codes_raw);
    }
    std::memcpy(b + o, c->centroids, z.pq);
    o += up8(z.pq);
  }
  const size_t res0 = o;
  std::memcpy(b + o, c->flags, z.flags);
  o += z.flags;
  for (int64_t h = 0; h < H; ++h) {
    const uint32_t r = (uint32_t)(c->res_offset[h + 1] - c->res_offset[h]);
    std::memcpy(b + o + 4 * h, &r, 4);
  }
  o += z.recs;
  const size_t rb = (size_t)c->res_offset[H];
  if (i.entropy == 2) {
    IntStreams s;
    split_records(i.n_par, i.n_perp, H, c->flags, c->res_offset, c->res_bytes, &s);
    o += int_streams_write(s, b + o);
  } else if (i.entropy) {
    o += rans_encode(c->res_bytes, rb, b + o);
  } else {
    if (rb) std::memcpy(b + o, c->res_bytes, rb);
    o += rb;
  }
  const uint64_t res_end = o;
  o = up8(o);
  (void)res0;
  if (i.entropy) o += up8(rans_encode((const uint8_t*)c->lambda, z.lam, b + o));
  else {
    std::memcpy(b + o, c->lambda, z.lam);
    o += up8(z.lam);
  }
  // header
  const uint16_t scheme = (uint16_t)(i.arch | (i.compute == HCZ_COMPUTE_BF16 ? 4 : 0) |
                                     (i.compute == HCZ_COMPUTE_FP64 ? 64 : 0) | (i.lambda_fp32 ? 8 : 0) |
                                     (i.entropy ? 16 : 0) | (i.entropy == 2 ? 32 : 0));
  const uint8_t lat = (uint8_t)(i.arch ? i.latent : 0), bits = (uint8_t)(i.arch ? i.bits : 0);
  const uint64_t HH = (uint64_t)H, tot = o;
  const uint16_t np = (uint16_t)i.n_par, nq = (uint16_t)i.n_perp;
  const uint32_t wb = (uint32_t)z.weights;
  std::memcpy(b, "HCZ1", 4);
  std::memcpy(b + 4, &scheme, 2);
  b[6] = lat;
  b[7] = bits;
  std::memcpy(b + 8, &HH, 8);
  std::memcpy(b + 16, &np, 2);
  std::memcpy(b + 18, &nq, 2);
  std::memcpy(b + 20, &wb, 4);
  std::memcpy(b + 24, &res_end, 8);
  std::memcpy(b + 32, &tot, 8);
  const uint32_t ck = fnv1a(b, 40);
  std::memcpy(b + 40, &ck, 4);
  *written = (size_t)tot;
  return HCZ_OK;
}

hcz_status hcz_container_read_info(const void* buf, size_t n, hcz_container_info* info) {
  if (!buf || !info) return set_error(HCZ_EINVAL, "NULL argument");
  const uint8_t* b = (const uint8_t*)buf;
  if (n < kHeader || std::memcmp(b, "HCZ1", 4) != 0) return set_error(HCZ_EINVAL, "not a container");
  uint32_t ck;
  std::memcpy(&ck, b + 40, 4);
  if (ck != fnv1a(b, 40)) return set_error(HCZ_EINVAL, "container header checksum mismatch");
  uint16_t scheme, np, nq;
  uint64_t HH, res_end, tot;
  uint32_t wb;
  std::memcpy(&scheme, b + 4, 2);
  std::memcpy(&HH, b + 8, 8);
  std::memcpy(&np, b + 16, 2);
  std::memcpy(&nq, b + 18, 2);
  std::memcpy(&wb, b + 20, 4);
  std::memcpy(&res_end, b + 24, 8);
  std::memcpy(&tot, b + 32, 8);
  if (tot > n || res_end > tot || HH > (uint64_t)INT64_MAX / 64) return set_error(HCZ_EINVAL, "container sizes inconsistent");
  hcz_container_info i{};
  i.H = (int64_t)HH;
  i.n_par = np;
  i.n_perp = nq;
  i.arch = scheme & 3;
  i.compute = (scheme & 64) ? HCZ_COMPUTE_FP64 : ((scheme & 4) ? HCZ_COMPUTE_BF16 : HCZ_COMPUTE_FP32);
  i.lambda_fp32 = (scheme & 8) ? 1 : 0;
  i.entropy = (scheme & 32) ? 2 : ((scheme & 16) ? 1 : 0);
  i.latent = b[6];
  i.bits = b[7];
  const size_t N = (size_t)np * nq;
  if (i.arch) {
    if (wb % 4 || wb / 4 <= 2 * N) return set_error(HCZ_EINVAL, "container weight section inconsistent");
    i.n_weights = (int64_t)(wb / 4 - 2 * N);
  }
  // residual bytes: the sum of the record sizes
  Sizes z;
  if (!sizes_of(i, &z)) return set_error(HCZ_EINVAL, "container header inconsistent");
  size_t o = up8(kHeader) + up8(z.weights);
  if (i.arch) {
    if (i.entropy) {
      if (o + 528 > res_end) return set_error(HCZ_EINVAL, "container codes section truncated");
      uint64_t m;
      std::memcpy(&m, b + o + 520, 8);
      if (m > res_end - o - 528) return set_error(HCZ_EINVAL, "container codes section truncated");
      o += up8(528 + (size_t)m);
    } else {
      o += up8(z.codes_raw);
    }
    o += up8(z.pq);
  }
  if (o + z.flags + z.recs > res_end) return set_error(HCZ_EINVAL, "container residual section truncated");
  uint64_t rb = 0;
  for (int64_t h = 0; h < i.H; ++h) {
    uint32_t r;
    std::memcpy(&r, b + o + z.flags + 4 * h, 4);
    rb += r;
  }
  i.res_bytes = rb;
  i.total_bytes = tot;
  *info = i;
  return HCZ_OK;
}

hcz_status hcz_container_unpack(const void* buf, size_t n, const hcz_container_out* out) {
  hcz_container_info i;
  hcz_status st = hcz_container_read_info(buf, n, &i);
  if (st) return st;
  if (!out) return set_error(HCZ_EINVAL, "NULL argument");
  Sizes z;
  sizes_of(i, &z);
  const uint8_t* b = (const uint8_t*)buf;
  uint64_t res_end, tot;
  std::memcpy(&res_end, b + 24, 8);
  std::memcpy(&tot, b + 32, 8);
  if ((i.H && (!out->flags || !out->res_offset || !out->lambda)) || (!i.H && !out->res_offset) ||
      (i.res_bytes && !out->res_bytes))
    return set_error(HCZ_EINVAL, "NULL output array");
  size_t o = up8(kHeader);
  if (i.arch) {
    if (!out->weights || !out->norm_mean || !out->norm_std || (i.H && !out->codes) || !out->centroids)
      return set_error(HCZ_EINVAL, "NULL model output array");
    std::memcpy(out->weights, b + o, 4 * (size_t)i.n_weights);
    std::memcpy(out->norm_mean, b + o + 4 * (size_t)i.n_weights, 4 * z.N);
    std::memcpy(out->norm_std, b + o + 4 * ((size_t)i.n_weights + z.N), 4 * z.N);
    o += up8(z.weights);
    if (i.entropy) {
      size_t used = 0;
      if (!rans_decode(b + o, res_end - o, out->codes, z.codes_raw, &used))
        return set_error(HCZ_EINVAL, "malformed codes section");
      o += up8(used);
    } else {
      std::memcpy(out->codes, b + o, z.codes_raw);
      o += up8(z.codes_raw);
    }
    std::memcpy(out->centroids, b + o, z.pq);
    o += up8(z.pq);
  }
  std::memcpy(out->flags, b + o, z.flags);
  o += z.flags;
  out->res_offset[0] = 0;
  for (int64_t h = 0; h < i.H; ++h) {
    uint32_t r;
    std::memcpy(&r, b + o + 4 * h, 4);
    out->res_offset[h + 1] = out->res_offset[h] + r;
  }
  o += z.recs;
  if (!record_sizes_valid(i.n_par, i.n_perp, i.H, out->flags, out->res_offset))
    return set_error(HCZ_EINVAL, "a residual record's size does not fit its flags");
  if (i.entropy == 2) {
    size_t used = 0;
    if (!int_streams_read(i.n_par, i.n_perp, i.H, out->flags, out->res_offset, b + o, res_end - o,
                          out->res_bytes, &used) || o + used != res_end)
      return set_error(HCZ_EINVAL, "malformed residual section");
  } else if (i.entropy) {
    size_t used = 0;
    if (!rans_decode(b + o, res_end - o, out->res_bytes, i.res_bytes, &used) || o + used != res_end)
      return set_error(HCZ_EINVAL, "malformed residual section");
  } else {
    if (o + i.res_bytes != res_end) return set_error(HCZ_EINVAL, "residual section size mismatch");
    if (i.res_bytes) std::memcpy(out->res_bytes, b + o, i.res_bytes);
  }
  o = up8(res_end);
  if (i.entropy) {
    size_t used = 0;
    if (o > tot || !rans_decode(b + o, tot - o, (uint8_t*)out->lambda, z.lam, &used))
      return set_error(HCZ_EINVAL, "malformed multiplier section");
  } else {
    if (o + z.lam > tot) return set_error(HCZ_EINVAL, "container multipliers truncated");
    std::memcpy(out->lambda, b + o, z.lam);
  }
  return HCZ_OK;
}

}  // extern "C"
