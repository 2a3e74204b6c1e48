"""Stage parity of the HIP path against the oracle on identical seeded inputs (GPU).

Each stage gets its inputs from the generator, never from another GPU stage, so the
oracle never consumes HIP output.  Integer results are compared bit for bit; floating
point within tolerances stated next to each comparison.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import coder, grid, moments, pipeline, pq
from paper_2212_10733_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    from paper_2212_10733_amd import hcz
    return hcz


@pytest.fixture(scope="module")
def ctx(H):
    return H.Context(0)


def say(*a):
    print("[case]", *a, flush=True)


def to_dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# ---- moments / QoIs -------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float64, np.float32])
@pytest.mark.parametrize("shape,vol", [((39, 39), None), ((39, 39), "jacobian"), ((33, 37), None), ((65, 65), None)])
def test_qoi_parity(H, ctx, dtype, shape, vol):
    n_perp, n_par = shape
    say("qoi", dtype.__name__, shape, vol)
    g = grid.make_grid(n_par, n_perp, vol=vol)
    plan = H.Plan(ctx, n_par, n_perp, vol=None if vol is None else g.vol)
    F = synth.histograms(300, n_par, n_perp, seed=21, dtype=dtype)
    b, q, nrm = H.qoi(plan, to_dev(F))
    torch.cuda.synchronize()
    b, q, nrm = b.cpu().numpy(), q.cpu().numpy(), nrm.cpu().numpy()
    bo = moments.moments(F, g)
    assert np.allclose(b, bo, rtol=1e-13, atol=1e-15 * np.abs(bo).max())
    assert np.allclose(q, moments.qoi_from_moments(bo, g), rtol=1e-12, atol=1e-14)
    # ||f|| is the correctly rounded sqrt of the correctly rounded sum of rounded squares
    X = F.reshape(300, -1).astype(np.float64)
    ref = np.array([math.sqrt(math.fsum(x * x)) for x in X])
    assert np.array_equal(nrm, ref)


# ---- quantizer -------------------------------------------------------------------------------

@pytest.mark.parametrize("latent,bits,n", [(16, 8, 5000), (40, 8, 3001), (7, 3, 1000)])
def test_quantize_bit_exact(H, ctx, latent, bits, n):
    """Codes equal the oracle's, exact midpoints, duplicates and non-finite latents
    included; 40 x 255 midpoints exceed what the LDS-staged kernel takes, so that case
    runs the search over the codebook in memory."""
    say("quantize", latent, bits, n)
    Z = synth.latents(n, latent, seed=22)
    C = synth.sorted_codebook(latent, bits, seed=23)
    C[3, 2] = C[3, 3]                        # duplicate centroid
    beta = (C[:, :-1].astype(np.float64) + C[:, 1:]) * 0.5
    exact = beta.astype(np.float32).astype(np.float64) == beta
    Z[:40, 5] = beta[5][exact[5]][:40].astype(np.float32) if exact[5].sum() >= 40 else Z[:40, 5]
    Z[40, :] = np.nan
    Z[41, :] = np.inf
    Z[42, :] = -np.inf
    got = H.quantize(to_dev(Z), to_dev(C)).cpu().numpy()
    assert np.array_equal(got, pq.encode(Z, C))


@pytest.mark.parametrize("n,bits,every", [(4096, 8, 1), (20000, 4, 16), (777, 6, 3), (100, 8, 1)])
def test_codebook_fit(H, ctx, n, bits, every):
    say("codebook", n, bits, every)
    Z = synth.latents(n, 16, seed=24)
    got = H.codebook_fit(to_dev(Z), bits, every).cpu().numpy()
    ref = pq.fit(Z, bits, every)
    scale = np.abs(Z).max()
    # same Lloyd path: centroids agree to FP32 rounding of means summed in different orders
    close = np.isclose(got, ref, rtol=0, atol=4 * np.finfo(np.float32).eps * scale)
    assert close.mean() > 0.999, close.mean()
    assert np.all(np.diff(got, axis=1) >= 0)


# ---- autoencoder -----------------------------------------------------------------------------

def dense_model(H, plan, F, seed=0):
    W = synth.dense_ae_weights(plan.N, seed=seed)
    rng = np.random.default_rng(seed + 100)
    for k in ("b1", "b2", "b3", "b4"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    mu, sd = oracle.ae.norm_stats(F)
    return W, mu.astype(np.float32), sd.astype(np.float32), H.Model(plan, W, mu, sd)


@pytest.mark.parametrize("Hn,dtype,shape", [(300, np.float32, (39, 39)), (129, np.float64, (39, 39)),
                                            (1000, np.float32, (33, 33)), (50, np.float32, (65, 65))])
def test_encode_parity(H, ctx, Hn, dtype, shape):
    n_perp, n_par = shape
    say("encode", Hn, dtype.__name__, shape)
    plan = H.Plan(ctx, n_par, n_perp)
    F = synth.histograms(Hn, n_par, n_perp, seed=25, dtype=dtype)
    W, mu, sd, model = dense_model(H, plan, F)
    z = H.encode(model, to_dev(F)).cpu().numpy()
    X = (F.reshape(Hn, -1).astype(np.float32).astype(np.float64) - mu) / sd
    zo = oracle.ae.dense_encode(X, W)
    # FP32 products and sums over K = N terms: error ~ sqrt(K) eps32 sum|terms|
    h1 = np.maximum(X @ W["W1"].T.astype(np.float64) + W["b1"], 0)
    mag = np.abs(h1) @ np.abs(W["W2"].T.astype(np.float64)) + (np.abs(X) @ np.abs(W["W1"].T.astype(np.float64))).max() * 0.01
    assert np.all(np.abs(z - zo) <= 5e-5 * (mag + 1e-3)), np.abs(z - zo).max()


@pytest.mark.parametrize("Hn,shape", [(300, (39, 39)), (1000, (33, 33)), (50, (65, 65))])
def test_decode_parity(H, ctx, Hn, shape):
    n_perp, n_par = shape
    say("decode", Hn, shape)
    plan = H.Plan(ctx, n_par, n_perp)
    F = synth.histograms(64, n_par, n_perp, seed=26, dtype=np.float32)
    W, mu, sd, model = dense_model(H, plan, F)
    C = synth.sorted_codebook(16, 8, seed=27)
    codes = synth.codes(Hn, 16, 8, seed=28)
    fh = H.decode(model, to_dev(codes), to_dev(C)).cpu().numpy().reshape(Hn, -1)
    Zh = pq.decode(codes, C)
    ref = oracle.ae.denormalize(oracle.ae.dense_decode(Zh, W), mu.astype(np.float64), sd.astype(np.float64))
    h3 = np.maximum(Zh @ W["W3"].T.astype(np.float64) + W["b3"], 0)
    mag = sd * (np.abs(h3) @ np.abs(W["W4"].T.astype(np.float64)) + np.abs(W["b4"])) + np.abs(mu)
    assert np.all(np.abs(fh - ref) <= 2e-5 * mag + 1e-30), np.abs(fh - ref).max()


def bf16_model(H, plan, F, seed=0):
    W, mu, sd, _ = dense_model(H, plan, F, seed)
    return W, mu, sd, H.Model(plan, W, mu, sd, compute="bf16")


@pytest.mark.parametrize("Hn,dtype,shape,pad", [(300, np.float32, (39, 39), 0), (129, np.float64, (39, 39), 0),
                                                (1000, np.float32, (33, 33), 0), (70, np.float32, (39, 39), 3),
                                                (50, np.float32, (65, 65), 0)])
def test_encode_parity_bf16(H, ctx, Hn, dtype, shape, pad):
    """BF16 form: the oracle forms the same bfloat16 operands (FP32 z-score, nearest-even
    rounding), so the two sides differ only in how the products are summed: FP32
    accumulation on the matrix cores against FP64 in the oracle.  Bound: about 100 FP32
    roundings of the running sum per output of layer 1 (K/16 accumulations plus the
    instruction's own), propagated through the FP32 layer 2."""
    n_perp, n_par = shape
    say("encode bf16", Hn, dtype.__name__, shape, "row pad", pad)
    plan = H.Plan(ctx, n_par, n_perp)
    F = synth.histograms(Hn, n_par, n_perp, seed=29, dtype=dtype)
    F[3, 2, 5] = np.nan                        # a non-finite element enters as 0
    W, mu, sd, model = bf16_model(H, plan, F[4:])
    x = to_dev(F)
    if pad:                                    # rows with a stride beyond n_par
        xp = torch.zeros((Hn, n_perp, n_par + pad), dtype=x.dtype, device=x.device)
        xp[:, :, :n_par] = x
        x = xp[:, :, :n_par]
    z = H.encode(model, x).cpu().numpy()
    rsd = np.float32(1) / sd
    zo = oracle.ae.dense_encode_bf16(F.astype(np.float32), mu, rsd, W)
    xb = oracle.ae.bf16_encode_input(F.reshape(Hn, -1).astype(np.float32), mu, rsd).astype(np.float64)
    w1 = oracle.ae.bf16(W["W1"]).astype(np.float64)
    s1 = np.abs(xb) @ np.abs(w1.T) + np.abs(W["b1"])
    h1 = np.maximum(xb @ w1.T + W["b1"], 0)
    w2 = np.abs(W["W2"].astype(np.float64)).T
    eps = 2.0 ** -24
    bound = 120 * eps * (s1 @ w2) + 140 * eps * (np.abs(h1) @ w2 + np.abs(W["b2"]))
    err = np.abs(z - zo)
    assert np.all(err <= bound), (err / bound).max()
    # against the FP32 form: the bfloat16 operands move z by about 2^-9 of the terms
    z32 = H.encode(H.Model(plan, W, mu, sd), x).cpu().numpy()
    assert np.abs(z - z32).max() > 100 * np.abs(err).max()


@pytest.mark.parametrize("Hn,shape", [(300, (39, 39)), (1000, (33, 33)), (50, (65, 65))])
def test_decode_parity_bf16(H, ctx, Hn, shape):
    """BF16 form: h3 is the same FP32 fused multiply-add chain on both sides (the oracle's
    FMA is exact), so its bfloat16 operands agree bit for bit; the output differs by FP32
    accumulation over K = 128 and the two roundings of sigma (y + b4) + mu."""
    n_perp, n_par = shape
    say("decode bf16", Hn, shape)
    plan = H.Plan(ctx, n_par, n_perp)
    F = synth.histograms(64, n_par, n_perp, seed=30, dtype=np.float32)
    W, mu, sd, model = bf16_model(H, plan, F)
    C = synth.sorted_codebook(16, 8, seed=31)
    codes = synth.codes(Hn, 16, 8, seed=32)
    fh = H.decode(model, to_dev(codes), to_dev(C)).cpu().numpy().reshape(Hn, -1)
    Zh = pq.decode(codes, C)
    ref = oracle.ae.dense_decode_bf16(Zh, W, mu, sd)
    w3 = W["W3"].astype(np.float64)
    h3 = np.maximum(Zh @ w3.T + W["b3"], 0)
    mag = np.abs(sd) * (np.abs(h3) @ np.abs(oracle.ae.bf16(W["W4"]).astype(np.float64).T) * 1.01
                        + np.abs(W["b4"])) + np.abs(mu)
    err = np.abs(fh - ref)
    assert np.all(err <= 40 * 2.0 ** -24 * mag), (err / mag).max()
    # decoding twice gives the same bits (compress and decompress share this kernel)
    fh2 = H.decode(model, to_dev(codes), to_dev(C)).cpu().numpy().reshape(Hn, -1)
    assert np.array_equal(fh, fh2)


# ---- residual coder + Newton -------------------------------------------------------------------

def oracle_residual(F, fhat, g, p, lam0=None):
    """Oracle compress with a given reconstruction (the coder-only pipeline when fhat is None);
    p.analytic_start seeds Newton with the oracle's own analytic start."""
    class _M:   # pipeline hook: a fixed reconstruction instead of the autoencoder
        pass
    Hn = F.shape[0]
    F64 = F.astype(np.float64)
    lay = coder.layout(g.n_par, g.n_perp)
    fh = np.zeros_like(F64) if fhat is None else fhat.astype(np.float64)
    finite = np.isfinite(F64).reshape(Hn, -1).all(axis=1)
    Fz = np.where(finite[:, None, None], F64, 0.0)
    b = moments.moments(Fz, g)
    th = pipeline.tau_h(Fz, p)
    r = Fz - fh
    thr = coder.SEL_MARGIN * th
    rr = coder.sumsq(r)
    coded = rr > thr * thr
    raw = ~finite | ~(b[:, 0] > 0) | (coded & ~(th > 0))
    out = dict(flags=np.zeros(Hn, np.uint8), lam=np.zeros((Hn, 4)), records=[], kstar=np.full(Hn, 255),
               margin=np.full(Hn, np.inf), iters=np.zeros(Hn, int))
    d0 = coder.delta0(th, lay)
    for h in range(Hn):
        rec = b""
        if not raw[h] and coded[h]:
            d = coder.decompose(r[h:h + 1], lay)
            if np.abs(d).max() * (1.0 / d0[h]) >= coder.QMAX:
                raw[h] = True
            else:
                # the search, recording the distance of every feasibility decision on its path
                # from the threshold
                margins = [abs(rr[h] - thr[h] ** 2) / thr[h] ** 2]

                def probe(rows, k, h=h, d=d):
                    Dk = coder.ladder(d0[h:h + 1], np.asarray(k))
                    e2 = coder.sumsq(r[h:h + 1] - coder.reconstruct(coder.quantize(d, Dk), Dk, lay))[0]
                    margins.append(abs(e2 - thr[h] ** 2) / thr[h] ** 2)
                    return np.array([e2 <= thr[h] ** 2])

                start = coder.search_start(lay) if p.search == "guided" else None
                ks = coder.search(None, d, d0[h:h + 1], thr[h:h + 1], lay, start, feasible_at=probe)
                Dk = coder.ladder(d0[h:h + 1], ks)
                q = coder.quantize(d, Dk)
                rh = coder.reconstruct(q, Dk, lay)
                out["kstar"][h] = ks[0]
                rec = coder.pack(q[0], Dk[0], int(ks[0]), lay)
                out["margin"][h] = min(margins)
                fh[h] = fh[h] + rh[0]
        elif not raw[h]:
            out["margin"][h] = abs(rr[h] - thr[h] ** 2) / max(thr[h] ** 2, 1e-300)
        flag = 0
        if not raw[h]:
            l0 = oracle.newton.analytic_start(fh[h], b[h], g) if p.analytic_start else \
                None if lam0 is None else lam0[h]
            res = oracle.newton.project(fh[h], b[h], g, p.newton_s, p.newton_max_iter, p.newton_max_iter2, p.fallback,
                                        lam0=l0, positivity=p.positivity)
            out["iters"][h] = res["iters"]
            if res.get("warm_rejected"):
                flag |= 8
            if res["status"] >= 1:
                flag |= pipeline.FLAG_ROUND2
            if res["status"] == 2:
                raw[h] = True
            else:
                out["lam"][h] = res["lam"]
                flag |= pipeline.FLAG_CODED if coded[h] else 0
                flag |= 0 if p.positivity else pipeline.FLAG_NOCLIP
        if raw[h]:
            flag = (flag & (pipeline.FLAG_ROUND2 | 8)) | pipeline.FLAG_RAW
            rec = np.ascontiguousarray(F[h]).tobytes()
            out["kstar"][h] = 255
        out["flags"][h] = flag
        out["records"].append(rec)
    out["raw"] = raw
    out["b"] = b
    out["tau_h"] = th
    return out


def compare_residual(H, plan, g, F, fhat, p, hp, near_tie=1e-9, lam0=None, flag_mask=0xff):
    Hn = F.shape[0]
    comp = H.residual(plan, hp, to_dev(F), None if fhat is None else to_dev(fhat),
                      lam0=None if lam0 is None else to_dev(lam0))
    torch.cuda.synchronize()
    flags = comp.flags.cpu().numpy()
    lam = comp.lam.cpu().numpy()
    off = comp.offsets.cpu().numpy().astype(np.uint64)
    stream = comp.stream_bytes()
    st = comp.stats()
    ref = oracle_residual(F, fhat, g, p, lam0=lam0)
    sure = ref["margin"] > near_tie          # decisions that rounding order cannot flip
    assert np.array_equal(flags[sure] & flag_mask, ref["flags"][sure] & flag_mask)
    assert (~sure).sum() <= max(1, Hn // 1000)
    nrec_equal = 0
    for h in np.nonzero(sure)[0]:
        rec = stream[int(off[h]):int(off[h + 1])]
        assert rec == ref["records"][h], (h, len(rec), len(ref["records"][h]))
        nrec_equal += 1
    assert int(off[-1]) == len(stream) == st["stream_bytes"]
    ok = sure & ~ref["raw"]
    scale = np.abs(ref["lam"][ok]).max() if ok.any() else 1.0
    assert np.allclose(lam[ok], ref["lam"][ok], rtol=1e-7, atol=1e-9 * scale)
    assert st["n_hist"] == Hn
    assert st["n_coded"] == int((flags & 1).sum()) and st["n_raw"] == int(((flags & 4) != 0).sum())
    return comp, ref, nrec_equal


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("Hn", [257, 64])
def test_residual_bit_exact_with_reconstruction(H, ctx, dtype, Hn):
    say("residual", dtype.__name__, Hn)
    g = grid.make_grid()
    plan = H.Plan(ctx)
    F = synth.histograms(Hn, seed=29, dtype=dtype)
    rel = np.geomspace(1e-5, 1e-1, Hn)
    fhat = synth.perturbed(F, rel, seed=30, dtype=np.float32)
    p = pipeline.Params(tau=1e-3)
    comp, ref, n = compare_residual(H, plan, g, F, fhat, p, H.params(tau=1e-3))
    coded = (comp.flags.cpu().numpy() & 1) != 0
    assert 0 < coded.sum() < Hn                  # both kinds present


def test_plan_paths(H, ctx):
    """Which kernel family serves a grid; every path is checked bit-exact below."""
    say("plan paths")
    cases = [((39, 39), None, "wave_fixed"), ((39, 39), "jacobian", "wave"), ((33, 37), None, "wave"),
             ((3, 3), None, "wave"), ((65, 65), None, "team4"), ((49, 49), "jacobian", "team2")]
    for (n_perp, n_par), vol, want in cases:
        g = grid.make_grid(n_par, n_perp, vol=vol)
        plan = H.Plan(ctx, n_par, n_perp, vol=None if vol is None else g.vol)
        assert plan.path == want, ((n_perp, n_par), vol, plan.path)


@pytest.mark.parametrize("shape,vol", [((39, 39), None), ((39, 39), "jacobian"), ((33, 33), None),
                                       ((49, 49), "jacobian"), ((65, 65), None), ((37, 33), None), ((3, 3), None),
                                       ((12, 5), None)])
@pytest.mark.parametrize("tau", [1e-2, 1e-4])
def test_residual_coder_only_grids(H, ctx, shape, vol, tau):
    n_perp, n_par = shape
    say("coder-only", shape, vol, tau)
    g = grid.make_grid(n_par, n_perp, vol=vol)
    plan = H.Plan(ctx, n_par, n_perp, vol=None if vol is None else g.vol)
    F = synth.histograms(67, n_par, n_perp, seed=31, dtype=np.float32)
    compare_residual(H, plan, g, F, None, pipeline.Params(tau=tau), H.params(tau=tau))


def test_residual_nrmse_mode_and_edge_cases(H, ctx):
    say("edge cases")
    g = grid.make_grid()
    plan = H.Plan(ctx)
    F = synth.histograms(40, seed=32, dtype=np.float32)
    F[0, 2, 3] = np.nan
    F[1] = 0.0
    F[2, 5, 5] = np.inf
    F[3] = 0.0
    F[3, 10, 10] = 1.0            # single cell: singular Hessian after a large perturbation
    fhat = synth.perturbed(F, 0.02, seed=33)
    fhat[3] = 0.0
    fhat[3, 12, 12] = 1.0
    p = pipeline.Params(tau=1e-3, tau_mode="nrmse")
    comp, ref, _ = compare_residual(H, plan, g, F, np.nan_to_num(fhat), p, H.params(tau=1e-3, tau_mode=H.TAU_NRMSE))
    flags = comp.flags.cpu().numpy()
    assert flags[0] & 4 and flags[1] & 4 and flags[2] & 4 and flags[3] & 4


def test_residual_tau_zero_and_forced_fallbacks(H, ctx):
    g = grid.make_grid()
    plan = H.Plan(ctx)
    F = synth.histograms(20, seed=34, dtype=np.float32)
    say("tau=0")
    compare_residual(H, plan, g, F, None, pipeline.Params(tau=0.0), H.params(tau=0.0))
    say("max_iter=0")
    p = pipeline.Params(tau=1e-2, newton_max_iter=0, newton_max_iter2=0)
    comp, _, _ = compare_residual(H, plan, g, F, None, p, H.params(tau=1e-2, newton_max_iter=0, newton_max_iter2=0))
    assert np.all(comp.flags.cpu().numpy() == 6)
    say("paper fallback")
    p = pipeline.Params(tau=1e-2, newton_max_iter=1, newton_max_iter2=400, fallback="paper")
    compare_residual(H, plan, g, F, None, p, H.params(tau=1e-2, newton_max_iter=1, fallback=H.FALLBACK_PAPER))


def test_residual_overflow_capacity(H, ctx):
    say("capacity")
    plan = H.Plan(ctx)
    F = synth.histograms(16, seed=35, dtype=np.float32)
    comp = H.residual(plan, H.params(tau=1e-3), to_dev(F), None, capacity=1000)
    with pytest.raises(H.HczError) as e:
        import ctypes
        s = H.Stats()
        st = H.LIB.hcz_stats_read(ctypes.c_void_p(comp.stats_dev.data_ptr()), ctypes.byref(s), None)
        H._check(st)
    assert e.value.status == -5
    assert s.overflow == 1 and s.stream_bytes > 1000


# ---- decompression ------------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_decompress_reads_oracle_stream(H, ctx, dtype):
    """The GPU decompressor rebuilds the oracle's own compressed stream (coder-only pipeline)."""
    say("decompress oracle stream", dtype.__name__)
    g = grid.make_grid()
    plan = H.Plan(ctx)
    F = synth.histograms(50, seed=36, dtype=dtype)
    F[7, 1, 1] = np.nan
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    ref = pipeline.decompress(comp, g, None, None, 50, dtype)
    cmp_ = H.alloc_compressed(50, plan.N, "cuda", capacity=len(comp["stream"]) + 16)
    cmp_.flags.copy_(torch.from_numpy(comp["flags"]))
    cmp_.lam.copy_(torch.from_numpy(comp["lam"]))
    cmp_.offsets.copy_(torch.from_numpy(comp["offsets"].astype(np.int64)))
    cmp_.stream[:len(comp["stream"])].copy_(torch.frombuffer(bytearray(comp["stream"]), dtype=torch.uint8))
    cz = H.Compressor(plan, None, 50, H.params(), in_dtype=torch.float32 if dtype == np.float32 else torch.float64)
    out = cz.decompress(cmp_, 50, in_dtype=torch.float32 if dtype == np.float32 else torch.float64).cpu().numpy()
    both_nan = np.isnan(out) & np.isnan(ref)
    assert np.all(both_nan | np.isclose(out, ref, rtol=1e-13, atol=1e-15 * np.nanmax(np.abs(ref))))


@pytest.mark.parametrize("shape", [(39, 39), (33, 37), (65, 65)])
def test_residual_stage5_variants(H, ctx, shape):
    """Correction without positivity: flags (bit 4), records and multipliers equal the
    oracle's closed form.  FP32 multipliers: the FP64 solution rounded (one FP32 ulp)."""
    n_perp, n_par = shape
    say("stage-5 variants", shape)
    g = grid.make_grid(n_par, n_perp)
    plan = H.Plan(ctx, n_par, n_perp)
    F = synth.histograms(96, n_par, n_perp, seed=43, dtype=np.float32)
    fhat = synth.perturbed(F, np.geomspace(1e-4, 5e-2, 96), seed=44)
    p = pipeline.Params(tau=1e-3, positivity=False)
    comp, ref, _ = compare_residual(H, plan, g, F, fhat, p, H.params(tau=1e-3, no_positivity=True))
    flags = comp.flags.cpu().numpy()
    raw = (flags & 4) != 0
    assert np.all((flags[~raw] & 16) != 0) and not np.any(flags[raw] & 16)
    p32 = pipeline.Params(tau=1e-3)
    c32 = H.residual(plan, H.params(tau=1e-3, lambda_fp32=True), to_dev(F), to_dev(fhat))
    assert c32.lam.dtype == torch.float32
    ref = oracle_residual(F, fhat, g, p32)
    lam32 = c32.lam.cpu().numpy()
    ok = ~ref["raw"]
    want = ref["lam"][ok].astype(np.float32)
    ulp = np.spacing(np.abs(want)).astype(np.float64)
    assert np.all(np.abs(lam32[ok].astype(np.float64) - want.astype(np.float64)) <= ulp)


@pytest.mark.parametrize("shape", [(39, 39), (65, 65)])
def test_decompress_rejects_corrupt_headers(H, ctx, shape):
    """A record whose header claims more payload than the record holds (or a width above 32
    bits) decodes to NaN; the records around it decode as before."""
    n = shape[0]
    say("corrupt headers", shape)
    g = grid.make_grid(n, n)
    plan = H.Plan(ctx, n, n)
    F = synth.histograms(6, n, n, seed=40, dtype=np.float32)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    assert np.all(comp["flags"] & 1)
    lay = oracle.coder.layout(n, n)
    stream = bytearray(comp["stream"])
    off = comp["offsets"].astype(np.int64)
    stream[off[1] + 10] = 40                                  # width above 32 bits
    stream[off[3] + 10 + lay.nlev - 1] += 8                   # finest group: payload past the record
    ref = pipeline.decompress(comp, g, None, None, 6)
    cmp_ = H.alloc_compressed(6, plan.N, "cuda", capacity=len(stream))
    cmp_.flags.copy_(torch.from_numpy(comp["flags"]))
    cmp_.lam.copy_(torch.from_numpy(comp["lam"]))
    cmp_.offsets.copy_(torch.from_numpy(off))
    cmp_.stream.copy_(torch.frombuffer(stream, dtype=torch.uint8))
    cz = H.Compressor(plan, None, 6, H.params())
    out = cz.decompress(cmp_, 6).cpu().numpy()
    assert np.all(np.isnan(out[[1, 3]]))
    ok = [0, 2, 4, 5]
    assert np.allclose(out[ok], ref[ok], rtol=1e-13, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("shape", [(39, 39), (49, 49)])
def test_decompress_rejects_raw_records_of_wrong_size(H, ctx, shape):
    """A verbatim record must hold exactly the N input values: the last histogram's record
    cut 4 bytes short (ending at the stream's capacity) decodes to NaN instead of being read
    past its end, and FP32 records decoded as FP64 input decode to NaN; coded records around
    them decode as before (wave and workgroup kernels)."""
    n = shape[0]
    say("raw record sizes", shape)
    g = grid.make_grid(n, n)
    plan = H.Plan(ctx, n, n)
    F = synth.histograms(6, n, n, seed=41, dtype=np.float32)
    F[2, 1, 1] = np.nan
    F[5, 2, 3] = np.nan
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    assert comp["flags"][2] & 4 and comp["flags"][5] & 4
    ref = pipeline.decompress(comp, g, None, None, 6)
    off = comp["offsets"].astype(np.int64).copy()
    off[6] -= 4
    stream = bytearray(comp["stream"][:off[6]])

    def run(offsets, data, in_dtype):
        c = H.alloc_compressed(6, plan.N, "cuda", capacity=len(data))
        c.flags.copy_(torch.from_numpy(comp["flags"]))
        c.lam.copy_(torch.from_numpy(comp["lam"]))
        c.offsets.copy_(torch.from_numpy(offsets))
        c.stream[:len(data)].copy_(torch.frombuffer(data, dtype=torch.uint8))
        return H.Compressor(plan, None, 6, H.params()).decompress(c, 6, in_dtype=in_dtype).cpu().numpy()

    out = run(off, stream, torch.float32)
    assert np.all(np.isnan(out[5]))
    ok = [0, 1, 3, 4]
    assert np.allclose(out[ok], ref[ok], rtol=1e-13, atol=1e-15 * np.nanmax(np.abs(ref)))
    assert np.array_equal(np.isnan(out[2]), np.isnan(ref[2]))
    assert np.array_equal(out[2][~np.isnan(out[2])], ref[2][~np.isnan(ref[2])])
    full = bytearray(comp["stream"])
    out = run(comp["offsets"].astype(np.int64), full, torch.float64)
    assert np.all(np.isnan(out[[2, 5]]))
    assert np.allclose(out[ok], ref[ok], rtol=1e-13, atol=1e-15 * np.nanmax(np.abs(ref)))


def test_fp64_round_trip_with_default_arguments(H, ctx):
    """A compressor built for FP64 input decompresses with its own element type by default:
    verbatim FP64 records come back bit for bit, the rest within the bound; asking for the
    other type than the batch was compressed from is refused."""
    say("fp64 default in_dtype")
    plan = H.Plan(ctx)
    F = synth.histograms(64, seed=42, dtype=np.float64)
    F[9, 4, 4] = np.nan
    cz = H.Compressor(plan, None, 64, H.params(tau=1e-3), in_dtype=torch.float64)
    comp = cz.compress(to_dev(F))
    out = cz.decompress(comp, 64).cpu().numpy()
    flags = comp.flags.cpu().numpy()
    assert flags[9] & 4
    assert np.array_equal(np.isnan(out[9]), np.isnan(F[9]))
    assert np.array_equal(out[9][~np.isnan(F[9])].view(np.uint64), F[9][~np.isnan(F[9])].view(np.uint64))
    ok = (flags & 4) == 0
    th = pipeline.tau_h(F[ok], pipeline.Params(tau=1e-3))
    dist = np.sqrt(((out[ok] - F[ok]) ** 2).sum(axis=(1, 2)))
    assert np.all(dist <= th)
    with pytest.raises(ValueError):
        cz.decompress(comp, 64, in_dtype=torch.float32)
    with pytest.raises(ValueError):
        H.Compressor(plan, None, 64, H.params(tau=1e-3)).compress(to_dev(F))


@pytest.mark.parametrize("shape", [(39, 39), (49, 49)])
def test_residual_warm_start(H, ctx, shape):
    """Warm starts near the solution, garbage and NaN: flags (incl. rejection), records and
    multipliers match the oracle given the same warm starts."""
    n = shape[0]
    say("warm start", shape)
    g = grid.make_grid(n, n)
    plan = H.Plan(ctx, n, n)
    F = synth.histograms(96, n, n, seed=37, dtype=np.float32)
    fhat = synth.perturbed(F, np.geomspace(1e-4, 3e-2, 96), seed=38)
    p = pipeline.Params(tau=1e-3)
    cold = oracle_residual(F, fhat, g, p)
    rng = np.random.default_rng(39)
    lam0 = cold["lam"] * (1 + 1e-3 * rng.normal(size=(96, 4)))
    lam0[::7] = [1e6, 0.0, 0.0, 0.0]          # every cell clipped: no usable step, rejected
    lam0[3::11] = np.nan
    comp, ref, _ = compare_residual(H, plan, g, F, fhat, p, H.params(tau=1e-3), lam0=lam0)
    flags = comp.flags.cpu().numpy()
    assert (flags[::7] & 8).all() and (flags[3::11] & 8).all()
    acc = (flags & 8) == 0
    assert acc.sum() > 50
    st = comp.stats()
    assert st["newton_iters_total"] < cold["iters"].sum()


@pytest.mark.parametrize("shape", [(39, 39), (33, 33), (65, 65)])
def test_residual_analytic_start(H, ctx, shape):
    """The analytic-linear start (A A^T)^-1 (A f~ - b), formed in the kernel from its own f~:
    records and flags equal to the oracle seeded with its own analytic start, multipliers
    to the Newton tolerance, the acceptance decision (flag bit 3) on all but near-ties, and
    the same projection as the cold start; on the compiled 39x39, run-time-table and
    workgroup kernels."""
    n = shape[0]
    say("analytic start", shape)
    g = grid.make_grid(n, n)
    plan = H.Plan(ctx, n, n)
    F = synth.histograms(128, n, n, seed=41, dtype=np.float32)
    fhat = synth.perturbed(F, np.geomspace(1e-4, 3e-2, 128), seed=42)
    p = pipeline.Params(tau=1e-3, analytic_start=True)
    comp, ref, _ = compare_residual(H, plan, g, F, fhat, p, H.params(tau=1e-3, analytic_start=True),
                                    flag_mask=0xff & ~8)
    flags = comp.flags.cpu().numpy()
    agree = ((flags & 8) == (ref["flags"] & 8)).mean()
    assert agree >= 0.98, agree
    cold = H.residual(plan, H.params(tau=1e-3), to_dev(F), to_dev(fhat))
    lam_c, lam_a = cold.lam.cpu().numpy(), comp.lam.cpu().numpy()
    ok = (flags & 4) == 0
    assert np.allclose(lam_a[ok], lam_c[ok], rtol=1e-7, atol=1e-9 * np.abs(lam_c[ok]).max())
    assert cold.stream_bytes() == comp.stream_bytes()
    with pytest.raises(Exception):
        H.residual(plan, H.params(tau=1e-3, analytic_start=True, no_positivity=True), to_dev(F), to_dev(fhat))


@pytest.mark.parametrize("shape,vol,team", [((49, 49), None, "team2"), ((49, 49), "jacobian", "team2"),
                                            ((65, 65), None, "team4"), ((49, 49), None, "team4"),
                                            ((39, 39), None, "team2"), ((37, 33), None, "team4")])
def test_team_variants_bit_exact(H, ctx, shape, vol, team):
    """The wave-team kernels (two or four waves per histogram): with a reconstruction and
    coder-only, at a tight and a loose bound, with NaN, empty and single-cell histograms
    and a forced fallback: flags, offsets and every record byte-exact against the oracle,
    multipliers to the Newton tolerance."""
    n_perp, n_par = shape
    say("team variant", shape, vol, team)
    g = grid.make_grid(n_par, n_perp, vol=vol)
    plan = H.Plan(ctx, n_par, n_perp, vol=None if vol is None else g.vol)
    assert team in plan.variants()
    plan.set_variant(team)
    Hn = 96
    F = synth.histograms(Hn, n_par, n_perp, seed=43, dtype=np.float32)
    F[5, 3, 4] = np.nan                          # verbatim
    F[9] = 0.0                                   # empty: b0 = 0, verbatim
    F[13] = 0.0
    F[13, n_perp // 2, n_par // 2] = 1.0         # a single cell
    fhat = synth.perturbed(F, np.geomspace(1e-5, 3e-2, Hn), seed=44, dtype=np.float32)
    fhat = np.where(np.isfinite(fhat), fhat, 0.0).astype(np.float32)
    # the single-cell histogram reconstructed exactly: with noise around one cell the
    # projection is ill-conditioned and whether Newton converges depends on summation order
    fhat[13] = F[13]
    for tau in (1e-4, 1e-2):
        compare_residual(H, plan, g, F, fhat, pipeline.Params(tau=tau), H.params(tau=tau))
        compare_residual(H, plan, g, F, None, pipeline.Params(tau=tau), H.params(tau=tau))
    # the paper's literal fallback schedule with a one-update first round: round 2 on most
    p = pipeline.Params(tau=1e-3, newton_max_iter=1, fallback="paper")
    compare_residual(H, plan, g, F, fhat, p, H.params(tau=1e-3, newton_max_iter=1, fallback=H.FALLBACK_PAPER))
