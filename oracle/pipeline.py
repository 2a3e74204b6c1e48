"""Compress / decompress of a batch of histograms (Section III, Fig. 1).

Compress, per histogram (FP64):
  1. widen the input; non-finite input or b0 <= 0 is stored verbatim;
  2. b = A f (true moments, Eq. 1-4);
  3. tau_h = tau ||f||_2 (relative L2) or tau sqrt(N) (max f - min f) (Eq. 7 per image);
  4. z = encoder(f), codes = PQ(z), fhat = decoder(codebook[codes]) (Stages 2-3);
     without a model fhat = 0 (the MGARD-only pipeline the paper compares against);
  5. r = f - fhat; coded iff ||r||^2 > thr^2, thr = (1 - 2^-20) tau_h (Stage 4 selection);
  6. coded: multilevel coefficients, bound search, record (Stage 4);
  7. ft = fhat + rhat; Newton projection onto A x = b, x >= 0 (Stage 5);
  8. outputs: codes, multipliers, flags, residual records.
Decompress: fhat from the codes, rhat from the record, ft = fhat + rhat,
f_c = max(0, ft - A^T lam); verbatim records are returned as stored.

Flags: bit0 coder record, bit1 round-2 Newton used, bit2 verbatim record, bit3 warm
start rejected, bit4 correction without positivity, bit5 KL correction.  Multipliers can be stored as FP32
(the paper's float multipliers, Section I and Fig. 7).  An optional warm-start network (oracle.mlp) seeds the Newton solve from
the dequantised latent; the projection keeps cold start as fallback and judge.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import ae, coder, conv, mlp as mlp_net, newton, pq
from .grid import Grid
from .moments import moments

FLAG_CODED, FLAG_ROUND2, FLAG_RAW, FLAG_WARM_REJECTED, FLAG_NOCLIP, FLAG_KL = 1, 2, 4, 8, 16, 32


@dataclass
class Params:
    tau: float = 1e-3
    tau_mode: str = "rel_l2"        # or "nrmse"
    newton_s: float = 1.0
    newton_max_iter: int = 50
    newton_max_iter2: int = 400
    fallback: str = "backtrack"     # or "paper" (s = 0.01)
    lambda_fp32: bool = False       # store the multipliers as FP32
    positivity: bool = True         # False: projection onto {A x = b} only
    kl: bool = False                # True: the KL / I-divergence correction (multiplicative)
    lambda_bits: int = 0            # > 0: multipliers rounded to this many mantissa bits
    ub_level: int | None = None     # None: searched coder step ('ab'); 0..40: the user's step ('ub')
    search: str = "guided"          # 'ab' search: "guided" (from the predicted index) or "bisect"
    analytic_start: bool = False    # Newton starts from (A A^T)^-1 (A ft - b) (not with a network)


def round_mantissa(v: np.ndarray, bits: int) -> np.ndarray:
    """Round FP64 values to `bits` explicit mantissa bits, nearest with ties to even
    (bits = 0 or >= 52 keeps them): the truncation of the multipliers (Section I)."""
    v = np.ascontiguousarray(v, np.float64)
    if bits <= 0 or bits >= 52:
        return v.copy()
    u = v.view(np.uint64)
    drop = np.uint64(52 - bits)
    half = (np.uint64(1) << (drop - np.uint64(1))) - np.uint64(1) + ((u >> drop) & np.uint64(1))
    return ((u + half) & ~((np.uint64(1) << drop) - np.uint64(1))).view(np.float64)


def tau_of(H: int, p: Params) -> np.ndarray:
    """The bound of every histogram: p.tau is one value for the batch or one per histogram
    (subdomains of a batch with their own bounds)."""
    return np.broadcast_to(np.asarray(p.tau, np.float64), (H,))


def tau_h(F64: np.ndarray, p: Params) -> np.ndarray:
    H = F64.shape[0]
    X = F64.reshape(H, -1)
    tau = tau_of(H, p)
    if p.tau_mode == "nrmse":
        return tau * math.sqrt(X.shape[1]) * (X.max(axis=1) - X.min(axis=1))
    return np.array([t * math.sqrt(math.fsum(x * x)) for t, x in zip(tau, X)])


def _bf16(model: dict) -> bool:
    """model["compute"] == "bf16" selects the BF16 form of the autoencoder (bfloat16
    operands for the two large products); the default is the FP64 model."""
    return model.get("compute", "fp64") == "bf16"


def _staged(model: dict) -> bool:
    """model["compute"] == "fp64_staged": the FP64 model whose latent z and reconstruction
    fhat are stored as FP32 (rounded to nearest) before the quantiser and the residual
    stage read them, as the library's FP64 form stores them."""
    return model.get("compute", "fp64") == "fp64_staged"


def _f32(a: np.ndarray) -> np.ndarray:
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def _conv_plain(model: dict) -> bool:
    """The convolutional model runs in its BF16 form unless model["compute"] == "fp64"
    asks for the plain FP64 model (the reference for the BF16 form's error)."""
    return model.get("arch", "dense") == "conv" and model.get("compute") == "fp64"


def encode_ae(F64: np.ndarray, model: dict) -> np.ndarray:
    if _conv_plain(model):
        return conv.encode64(F64, model["mu"], model["sd"], model["W"])
    if model.get("arch", "dense") == "conv":
        sd32 = np.asarray(model["sd"], np.float32)
        return conv.encode_bf16(F64.astype(np.float32), np.asarray(model["mu"], np.float32),
                                np.float32(1) / sd32, model["W"])
    if _bf16(model):
        sd32 = np.asarray(model["sd"], np.float32)
        return ae.dense_encode_bf16(F64.astype(np.float32), np.asarray(model["mu"], np.float32),
                                    np.float32(1) / sd32, model["W"])
    Z = ae.dense_encode(ae.normalize(F64, model["mu"], model["sd"]), model["W"])
    return _f32(Z) if _staged(model) else Z


def reconstruct_ae(codes: np.ndarray, C: np.ndarray, model: dict, shape) -> np.ndarray:
    Zh = pq.decode(codes, C)
    if _conv_plain(model):
        return conv.decode64(Zh, model["W"], model["mu"], model["sd"]).reshape(shape)
    if model.get("arch", "dense") == "conv":
        return conv.decode_bf16(Zh, model["W"], np.asarray(model["mu"], np.float32),
                                np.asarray(model["sd"], np.float32)).reshape(shape)
    if _bf16(model):
        return ae.dense_decode_bf16(Zh, model["W"], np.asarray(model["mu"], np.float32),
                                    np.asarray(model["sd"], np.float32)).reshape(shape)
    Xh = ae.dense_decode(Zh, model["W"])
    fhat = ae.denormalize(Xh, model["mu"], model["sd"])
    return (_f32(fhat) if _staged(model) else fhat).reshape(shape)


def compress(F: np.ndarray, g: Grid, model: dict | None, C: np.ndarray | None, p: Params,
             fit_codebook: bool = False, bits: int = 8, sample_every: int = 16,
             warm: tuple | None = None) -> dict:
    """warm: optional (network parameters, scale) of the warm-start network (needs a model)."""
    H = F.shape[0]
    F64 = np.asarray(F, np.float64).reshape(H, g.n_perp, g.n_par)
    lay = coder.layout(g.n_par, g.n_perp)
    finite = np.isfinite(F64).reshape(H, -1).all(axis=1)
    Fz = np.where(finite[:, None, None], F64, 0.0)
    b = moments(Fz, g)
    th = tau_h(Fz, p)
    L = (model["W"]["fw"] if model.get("arch") == "conv" else model["W"]["W2"]).shape[0] if model else 0
    codes = np.zeros((H, L), np.uint8)
    Z = None
    if model is not None:
        Z = encode_ae(Fz, model)
        if fit_codebook:
            C = pq.fit(Z, bits, sample_every)
        codes = pq.encode(Z, C)
        fhat = reconstruct_ae(codes, C, model, F64.shape)
    else:
        fhat = np.zeros_like(F64)
    r = Fz - fhat
    thr = coder.SEL_MARGIN * th
    coded = coder.sumsq(r) > thr * thr
    tau = tau_of(H, p)
    raw = ~finite | ~(b[:, 0] > 0) | (coded & ~(th > 0)) | ~(np.isfinite(tau) & (tau >= 0))
    kstar = np.zeros(H, np.int64)
    q = np.zeros(F64.shape, np.int64)
    rhat = np.zeros_like(F64)
    d0 = coder.delta0(th, lay)
    act = coded & ~raw
    if act.any():
        d = coder.decompose(r[act], lay)
        big = np.abs(d).reshape(d.shape[0], -1).max(axis=1) * (1.0 / d0[act]) >= coder.QMAX
        idx = np.nonzero(act)[0]
        raw[idx[big]] = True
        act = coded & ~raw
        keep = ~big
        if keep.any():
            if p.ub_level is None:
                start = coder.search_start(lay) if p.search == "guided" else None
                ks, qs, rh = coder.search(r[act], d[keep], d0[act], thr[act], lay, start)
            else:
                ks, qs, rh = coder.at_level(d[keep], d0[act], p.ub_level, lay)
            kstar[act], q[act], rhat[act] = ks, qs, rh
    ft = fhat + rhat
    lam = np.zeros((H, 4))
    flags = np.zeros(H, np.uint8)
    iters = np.zeros(H, np.int64)
    fc = np.zeros_like(F64)
    lam0 = None
    if warm is not None and model is not None:
        lam0 = mlp_net.predict(pq.decode(codes, C), warm[0], warm[1])
    if p.analytic_start:
        if lam0 is not None:
            raise ValueError("the analytic start and a warm-start network exclude each other")
        if not p.positivity or p.kl:
            raise ValueError("the analytic start belongs to the projection with positivity")
        lam0 = np.array([newton.analytic_start(ft[h], b[h], g) if not raw[h] else np.zeros(4)
                         for h in range(H)]).reshape(H, 4)
    for h in range(H):
        if raw[h]:
            continue
        kl = False
        if p.kl:
            # the KL correction is not non-expansive: it is kept only where it keeps the bound,
            # elsewhere the histogram gets the L2 projection
            res = newton.project_kl(ft[h], b[h], g, p.newton_s, p.newton_max_iter, p.newton_max_iter2, p.fallback)
            kl = res["status"] < 2 and coder.sumsq(Fz[h:h + 1] - res["x"][None])[0] <= thr[h] * thr[h]
        if not kl:
            res = newton.project(ft[h], b[h], g, p.newton_s, p.newton_max_iter, p.newton_max_iter2,
                                 p.fallback, lam0=None if lam0 is None else lam0[h], positivity=p.positivity)
        iters[h] = res["iters"]
        if res.get("warm_rejected"):
            flags[h] |= FLAG_WARM_REJECTED
        if res["status"] >= 1:
            flags[h] |= FLAG_ROUND2
        if res["status"] == 2:
            raw[h] = True
            continue
        lam[h] = res["lam"]
        fc[h] = res["x"]
        if not p.positivity:
            flags[h] |= FLAG_NOCLIP
        if kl:
            flags[h] |= FLAG_KL
    records = []
    for h in range(H):
        if raw[h]:
            flags[h] = (flags[h] & (FLAG_ROUND2 | FLAG_WARM_REJECTED)) | FLAG_RAW
            records.append(np.ascontiguousarray(np.asarray(F)[h]).tobytes())
            fc[h] = F64[h]
            lam[h] = 0.0
        elif act[h]:
            flags[h] |= FLAG_CODED
            records.append(coder.pack(q[h], coder.ladder(d0[h:h + 1], kstar[h:h + 1])[0],
                                      int(kstar[h]), lay))
        else:
            records.append(b"")
    sizes = np.array([len(x) for x in records], np.uint64)
    offsets = np.zeros(H + 1, np.uint64)
    offsets[1:] = np.cumsum(sizes)
    lam = round_mantissa(lam, p.lambda_bits)
    if p.lambda_fp32:
        lam = lam.astype(np.float32)
    return dict(codes=codes, lam=lam, flags=flags, stream=b"".join(records), offsets=offsets,
                codebook=C, b=b, tau_h=th, z=Z, fhat=fhat, rhat=rhat, ft=ft, fc=fc, kstar=kstar,
                iters=iters)


def decompress(comp: dict, g: Grid, model: dict | None, C: np.ndarray | None, H: int,
               in_dtype=np.float32) -> np.ndarray:
    lay = coder.layout(g.n_par, g.n_perp)
    shape = (H, g.n_perp, g.n_par)
    if model is not None:
        fhat = reconstruct_ae(comp["codes"], C, model, shape)
    else:
        fhat = np.zeros(shape)
    out = np.zeros(shape)
    stream, off = comp["stream"], comp["offsets"]
    for h in range(H):
        rec = stream[int(off[h]):int(off[h + 1])]
        fl = comp["flags"][h]
        if fl & FLAG_RAW:
            out[h] = np.frombuffer(rec, dtype=in_dtype).reshape(g.n_perp, g.n_par)
            continue
        ft = fhat[h].copy()
        if fl & FLAG_CODED:
            qh, Delta, _ = coder.unpack(rec, lay)
            ft = fhat[h] + coder.reconstruct(qh[None], np.array([Delta]), lay)[0]
        out[h] = newton.apply(ft, np.asarray(comp["lam"][h], np.float64), g,
                              positivity=not comp["flags"][h] & FLAG_NOCLIP, kl=bool(comp["flags"][h] & FLAG_KL))
    return out
