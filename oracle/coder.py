"""Error-bounded multilevel residual coder (Section III Stage 4).

The paper codes residuals with MGARD "uniform": a multilevel decomposition with uniform
quantisation bins, whose bound parameter is found by a binary search so that the
reconstruction meets the primary-data bound.  MGARD itself is not used; this module
restates the textbook multilevel (hierarchical-basis) decomposition it rests on:

Nested 1-D node sets on n points: G_l = {i : i mod 2^l = 0} U {n-1}, l = 0..L_n with
L_n = ceil(log2(n-1)); for l >= L_n the set is {0, n-1}.  In 2-D, L = max(L_par, L_perp).

Decomposition (fine to coarse, original values only): every node of
G_{l-1}^2 \\ G_l^2 gets d = y - P, where P interpolates y from the G_l neighbours:
  * on a coarse row (j in G_l): linear along i between a < i < b,
  * on a coarse column (i in G_l): linear along j,
  * otherwise bilinear from the four corners, evaluated as
        p0 = y[aj,a] + s (y[aj,b] - y[aj,a]),  p1 = y[bj,a] + s (y[bj,b] - y[bj,a]),
        P = p0 + t (p1 - p0),   s = (i-a)/(b-a), t = (j-aj)/(bj-aj)
    (separate multiplies and adds, never fused).
Nodes of G_L^2 keep their values.  Recomposition runs coarse to fine: y = d + P.

Quantisation: a ladder Delta_k = Delta_0 * 2^(k/4), k = 0..40, with
Delta_0 = 2 (1 - 2^-19) tau_h / (sqrt(N) (L+1)); q = rint(d / Delta_k) (round half to
even, via multiplication by 1/Delta_k).  Level 0 always meets the bound, since each
recomposition level adds at most Delta/2 to a convex combination of coarser errors.
feasible(k): sum (r - T^-1(Delta_k q))^2 <= thr^2, thr = (1 - 2^-20) tau_h.
The bound search (the paper's 'ab', a binary search): by default an exponential search from
the predicted index round(4 log2(L+1)) that brackets the feasibility boundary, then a
bisection of the bracket; optionally the bisection over k in [0, 41) alone: lo = 0, hi = 41,
mid = (lo+hi) >> 1.  With a user-specified step ('ub') the ladder index is given and there is
no search (Section IV-F).

Record: header = Delta_k* (f64 LE), k* (u8), nlev = L+1 (u8), one bit width per
coefficient group (u8), zero padded to a multiple of 8 bytes; payload = the zigzag
integers u = 2q (q >= 0) or -2q-1 (q < 0), group by group (coarsest first, row-major
within a group), each with its group's bit width, packed LSB first into little-endian
32-bit words.
"""
from __future__ import annotations

import math
import struct
from dataclasses import dataclass, field

import numpy as np

NLADDER = 41
# 2^(m/4), m = 0..3, as correctly rounded binary64 literals.
LADDER_C = (1.0, float.fromhex("0x1.306fe0a31b715p+0"), float.fromhex("0x1.6a09e667f3bcdp+0"),
            float.fromhex("0x1.ae89f995ad3adp+0"))
SEL_MARGIN = 1.0 - 2.0 ** -20
LADDER_MARGIN = 2.0 * (1.0 - 2.0 ** -19)
QMAX = 2 ** 30


def nlevels_1d(n: int) -> int:
    return (n - 2).bit_length() if n >= 2 else 0


def node_set(n: int, l: int) -> list:
    return sorted(set(range(0, n, 1 << l)) | {n - 1})


def neighbours(n: int, l: int, i: int):
    """(a, b, s) for index i at level l: itself with s = 0 if i is in G_l, else the G_l bracket."""
    G = node_set(n, l)
    if i in G:
        return i, i, 0.0
    a = max(g for g in G if g < i)
    b = min(g for g in G if g > i)
    return a, b, (i - a) / (b - a)


@dataclass
class Level:
    l: int
    J: np.ndarray
    I: np.ndarray
    kind: np.ndarray   # 0: along i, 1: along j, 2: bilinear
    A: np.ndarray
    B: np.ndarray
    S: np.ndarray
    AJ: np.ndarray
    BJ: np.ndarray
    T: np.ndarray


@dataclass
class Layout:
    n_par: int
    n_perp: int
    L: int
    coarse_J: np.ndarray
    coarse_I: np.ndarray
    levels: list = field(default_factory=list)   # l = L .. 1 (coarse to fine)

    @property
    def nlev(self) -> int:
        return self.L + 1

    def groups(self):
        """Coefficient groups in packing order: (J, I) arrays, coarsest first."""
        out = [(self.coarse_J, self.coarse_I)]
        out += [(lv.J, lv.I) for lv in self.levels]
        return out

    @property
    def header_bytes(self) -> int:
        return 8 * math.ceil((10 + self.nlev) / 8)


def layout(n_par: int, n_perp: int) -> Layout:
    L = max(nlevels_1d(n_par), nlevels_1d(n_perp))
    Gp, Gq = node_set(n_par, L), node_set(n_perp, L)
    cj = np.array([j for j in Gq for i in Gp], dtype=np.int64)
    ci = np.array([i for j in Gq for i in Gp], dtype=np.int64)
    lay = Layout(n_par, n_perp, L, cj, ci)
    for l in range(L, 0, -1):
        Gi_f, Gj_f = node_set(n_par, l - 1), node_set(n_perp, l - 1)
        Gi_c, Gj_c = set(node_set(n_par, l)), set(node_set(n_perp, l))
        rows = []
        for j in Gj_f:
            for i in Gi_f:
                if j in Gj_c and i in Gi_c:
                    continue
                a, b, s = neighbours(n_par, l, i)
                aj, bj, t = neighbours(n_perp, l, j)
                kind = 0 if j in Gj_c else (1 if i in Gi_c else 2)
                rows.append((j, i, kind, a, b, s, aj, bj, t))
        R = list(zip(*rows))
        lay.levels.append(Level(l, np.array(R[0]), np.array(R[1]), np.array(R[2]),
                                np.array(R[3]), np.array(R[4]), np.array(R[5], np.float64),
                                np.array(R[6]), np.array(R[7]), np.array(R[8], np.float64)))
    return lay


def _predict(y: np.ndarray, lv: Level) -> np.ndarray:
    """Interpolated values at the nodes of one level from y (H, n_perp, n_par)."""
    P = np.empty((y.shape[0], lv.J.size))
    for kind in (0, 1, 2):
        m = lv.kind == kind
        if not m.any():
            continue
        J, I, A, B, S, AJ, BJ, T = (x[m] for x in (lv.J, lv.I, lv.A, lv.B, lv.S, lv.AJ, lv.BJ, lv.T))
        if kind == 0:
            y0, y1 = y[:, J, A], y[:, J, B]
            P[:, m] = y0 + S * (y1 - y0)
        elif kind == 1:
            y0, y1 = y[:, AJ, I], y[:, BJ, I]
            P[:, m] = y0 + T * (y1 - y0)
        else:
            y00, y10, y01, y11 = y[:, AJ, A], y[:, AJ, B], y[:, BJ, A], y[:, BJ, B]
            p0 = y00 + S * (y10 - y00)
            p1 = y01 + S * (y11 - y01)
            P[:, m] = p0 + T * (p1 - p0)
    return P


def decompose(r: np.ndarray, lay: Layout) -> np.ndarray:
    """Multilevel coefficients d (H, n_perp, n_par) of residuals r (H, n_perp, n_par)."""
    r = np.asarray(r, np.float64)
    d = r.copy()
    for lv in lay.levels:
        d[:, lv.J, lv.I] = r[:, lv.J, lv.I] - _predict(r, lv)
    return d


def recompose(d: np.ndarray, lay: Layout) -> np.ndarray:
    """Inverse of `decompose`: coarse to fine, y = d + P(y)."""
    d = np.asarray(d, np.float64)
    y = np.zeros_like(d)
    y[:, lay.coarse_J, lay.coarse_I] = d[:, lay.coarse_J, lay.coarse_I]
    for lv in lay.levels:
        y[:, lv.J, lv.I] = d[:, lv.J, lv.I] + _predict(y, lv)
    return y


def delta0(tau_h: np.ndarray, lay: Layout) -> np.ndarray:
    N = lay.n_par * lay.n_perp
    return (LADDER_MARGIN * np.asarray(tau_h, np.float64)) / (math.sqrt(N) * (lay.L + 1))


def ladder(d0: np.ndarray, k: np.ndarray) -> np.ndarray:
    """Delta_k = ldexp(Delta_0, k >> 2) * c[k & 3]."""
    k = np.asarray(k, np.int64)
    c = np.asarray(LADDER_C)[k & 3]
    return np.ldexp(np.asarray(d0, np.float64), k >> 2) * c


def quantize(d: np.ndarray, Delta: np.ndarray) -> np.ndarray:
    inv = 1.0 / np.asarray(Delta, np.float64)
    return np.rint(d * inv[:, None, None]).astype(np.int64)


def sumsq(e: np.ndarray) -> np.ndarray:
    """Sum of squares per histogram with a correctly rounded sum of the rounded squares."""
    e = np.asarray(e, np.float64).reshape(e.shape[0], -1)
    return np.array([math.fsum(row * row) for row in e])


def reconstruct(q: np.ndarray, Delta: np.ndarray, lay: Layout) -> np.ndarray:
    return recompose(np.asarray(Delta, np.float64)[:, None, None] * q.astype(np.float64), lay)


def feasible(r, d, Delta, thr, lay):
    q = quantize(d, Delta)
    rh = reconstruct(q, Delta, lay)
    return sumsq(r - rh) <= thr * thr, q, rh


def bisect(r: np.ndarray, d: np.ndarray, d0: np.ndarray, thr: np.ndarray, lay: Layout):
    """Bound search over the ladder for a batch; returns (k*, q, rhat)."""
    H = r.shape[0]
    lo = np.zeros(H, np.int64)
    hi = np.full(H, NLADDER, np.int64)
    while np.any(hi - lo > 1):
        act = hi - lo > 1
        mid = (lo + hi) >> 1
        ok, _, _ = feasible(r[act], d[act], ladder(d0[act], mid[act]), thr[act], lay)
        idx = np.nonzero(act)[0]
        lo[idx[ok]] = mid[idx[ok]]
        hi[idx[~ok]] = mid[idx[~ok]]
    q = quantize(d, ladder(d0, lo))
    rh = reconstruct(q, ladder(d0, lo), lay)
    return lo, q, rh


def search_start(lay: Layout) -> int:
    """Ladder index where the guided search starts: round(4 log2(L+1)).  Independent uniform
    quantisation errors have variance Delta^2/12 per coefficient; the recomposition adds the
    coarser levels' interpolated errors, about three times that per cell, so the error
    estimate N Delta^2 / 4 meets tau_h^2 at Delta = 2 tau_h / sqrt(N) = (L+1) Delta_0,
    i.e. k = 4 log2(L+1) (margins ignored)."""
    return int(min(NLADDER - 1, math.floor(4.0 * math.log2(lay.L + 1) + 0.5)))


def search(r: np.ndarray, d: np.ndarray, d0: np.ndarray, thr: np.ndarray, lay: Layout,
           start: int | None = None, feasible_at=None):
    """Bound search over the ladder for a batch; returns (k*, q, rhat).

    start None: bisection over [0, 41) (lo = 0, hi = 41, mid = (lo+hi) >> 1).
    start k_g: exponential search from a predicted index (Bentley and Yao), then the same
    bisection: probe k_g; if it is feasible, probe k_g+1, k_g+3, k_g+7, ... (steps doubling)
    until one is infeasible or past 40; otherwise probe k_g-1, k_g-3, ... until one is
    feasible or at most 0 (index 0 is feasible by construction).  The last feasible and the
    first infeasible probe bracket the bisection.  Either way k* is feasible and k*+1 is
    infeasible or 41.  feasible_at(rows, k) replaces the feasibility test (for checking the
    search alone)."""
    H = r.shape[0] if r is not None else d.shape[0]
    if feasible_at is None:
        def feasible_at(rows, k):
            ok, _, _ = feasible(r[rows], d[rows], ladder(d0[rows], k), thr[rows], lay)
            return ok
    lo = np.zeros(H, np.int64)
    hi = np.full(H, NLADDER, np.int64)
    step = np.ones(H, np.int64)
    # phase 0: first probe, 1: climbing, 2: descending, 3: bisection
    phase = np.full(H, 3 if start is None else 0, np.int64)
    kg = 0 if start is None else int(min(max(start, 0), NLADDER - 1))
    while True:
        up = (phase == 1) & (lo + step >= NLADDER)
        phase[up] = 3
        down = (phase == 2) & (hi - step <= 0)
        lo[down] = 0
        phase[down] = 3
        act = (phase != 3) | (hi - lo > 1)
        if not act.any():
            break
        t = np.where(phase == 0, kg, np.where(phase == 1, lo + step,
                     np.where(phase == 2, hi - step, (lo + hi) >> 1)))
        rows = np.nonzero(act)[0]
        ok = np.zeros(H, bool)
        ok[rows] = feasible_at(rows, t[rows])
        p0, p1, p2, p3 = (act & (phase == i) for i in range(4))
        # first probe
        lo[p0 & ok] = kg
        hi[p0 & ~ok] = kg
        phase[p0] = np.where(ok[p0], 1, 2)
        # climbing: a feasible probe moves lo and doubles the step, an infeasible one brackets
        lo[p1 & ok] = t[p1 & ok]
        step[p1 & ok] *= 2
        hi[p1 & ~ok] = t[p1 & ~ok]
        phase[p1 & ~ok] = 3
        # descending: an infeasible probe moves hi and doubles the step, a feasible one brackets
        hi[p2 & ~ok] = t[p2 & ~ok]
        step[p2 & ~ok] *= 2
        lo[p2 & ok] = t[p2 & ok]
        phase[p2 & ok] = 3
        # bisection
        lo[p3 & ok] = t[p3 & ok]
        hi[p3 & ~ok] = t[p3 & ~ok]
    if r is None:
        return lo
    q = quantize(d, ladder(d0, lo))
    rh = reconstruct(q, ladder(d0, lo), lay)
    return lo, q, rh


def at_level(d: np.ndarray, d0: np.ndarray, k: int, lay: Layout):
    """The user-specified step ('ub', Section IV-F): every histogram quantised with ladder
    step k, without a search; returns (k*, q, rhat) like `bisect`."""
    ks = np.full(d.shape[0], int(k), np.int64)
    Delta = ladder(d0, ks)
    q = quantize(d, Delta)
    return ks, q, reconstruct(q, Delta, lay)


def zigzag(q: int) -> int:
    return 2 * q if q >= 0 else -2 * q - 1


def unzigzag(u: int) -> int:
    return (u >> 1) if (u & 1) == 0 else -((u + 1) >> 1)


def pack(q: np.ndarray, Delta: float, kstar: int, lay: Layout) -> bytes:
    """One record for one histogram's integer coefficients q (n_perp, n_par)."""
    widths, vals = [], []
    for J, I in lay.groups():
        u = [zigzag(int(v)) for v in q[J, I]]
        w = max(u).bit_length() if u else 0
        widths.append(w)
        vals.append((u, w))
    head = struct.pack("<d", float(Delta)) + bytes([kstar, lay.nlev]) + bytes(widths)
    head += b"\0" * (lay.header_bytes - len(head))
    acc, pos = 0, 0
    for u, w in vals:
        for v in u:
            acc |= v << pos
            pos += w
    nwords = (pos + 31) // 32
    return head + acc.to_bytes(4 * nwords, "little")


def unpack(rec: bytes, lay: Layout):
    """Inverse of `pack`: (q (n_perp, n_par) int64, Delta, k*)."""
    Delta = struct.unpack("<d", rec[:8])[0]
    kstar, nlev = rec[8], rec[9]
    assert nlev == lay.nlev
    widths = list(rec[10:10 + nlev])
    acc = int.from_bytes(rec[lay.header_bytes:], "little")
    q = np.zeros((lay.n_perp, lay.n_par), np.int64)
    pos = 0
    for (J, I), w in zip(lay.groups(), widths):
        mask = (1 << w) - 1
        for j, i in zip(J, I):
            q[j, i] = unzigzag((acc >> pos) & mask)
            pos += w
    return q, Delta, kstar


def record_size(widths, lay: Layout) -> int:
    bits = sum(len(J) * w for (J, _), w in zip(lay.groups(), widths))
    return lay.header_bytes + 4 * ((bits + 31) // 32)
