"""End-to-end parity of hcz_compress / hcz_decompress against the oracle (GPU).

Both sides start from the same generator output and model.  The autoencoder runs in FP32
on the GPU and FP64 in the oracle, so codes may differ only where the oracle's latent sits
within the stated tolerance of a midpoint (counted, bounded); the bound and the QoIs must
hold on the GPU's own output for every histogram.  In the coder-only pipeline (no model)
every record must match the oracle's bit for bit, also at the full 2^20 batch.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import grid, moments, pipeline, pq
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


def check_roundtrip(F, out, flags, tau, g, qtol=1e-10):
    F64 = F.astype(np.float64)
    Hn = F.shape[0]
    th = pipeline.tau_h(F64, pipeline.Params(tau=tau))
    raw = (flags & 4) != 0
    dist = np.sqrt(((out - F64) ** 2).reshape(Hn, -1).sum(1))
    assert np.all(dist[~raw] <= th[~raw]), (dist[~raw] / th[~raw]).max()
    assert np.array_equal(out[raw], F64[raw])
    q0 = moments.qoi(F64, g)
    q1 = moments.qoi(out, g)
    err = moments.qoi_rel_error(q0, q1, g)[~raw]
    assert err.max() < qtol, err.max()
    return dist, th


def near_tie_codes(z_or, C_or, C_gpu, tol):
    """Mask of (h, d) where the oracle latent lies within tol of a midpoint of either codebook."""
    near = np.zeros(z_or.shape, bool)
    for C in (C_or, C_gpu):
        beta = pq.midpoints(C)
        for d in range(z_or.shape[1]):
            idx = np.searchsorted(beta[d], z_or[:, d])
            lo = np.abs(z_or[:, d] - beta[d][np.clip(idx - 1, 0, beta.shape[1] - 1)])
            hi = np.abs(z_or[:, d] - beta[d][np.clip(idx, 0, beta.shape[1] - 1)])
            near[:, d] |= np.minimum(lo, hi) <= tol[d]
    return near


@pytest.mark.parametrize("Hn,dtype,every,bits,compute", [(256, np.float64, 1, 8, "fp32"), (3001, np.float32, 16, 8, "fp32"),
                                                         (1000, np.float32, 4, 4, "fp32"), (3001, np.float32, 16, 8, "bf16"),
                                                         (256, np.float64, 1, 8, "bf16")])
def test_compress_with_model(H, ctx, Hn, dtype, every, bits, compute):
    """compute = "bf16": the BF16 form on both sides (the oracle forms the same bfloat16
    operands and sums in FP64), with the same tolerances as the FP32 form."""
    say("e2e model", Hn, dtype.__name__, every, bits, compute)
    g = grid.make_grid()
    F = synth.histograms(Hn, seed=synth.SEED_PLAIN_SMALL, dtype=dtype)
    W = synth.dense_ae_weights()
    mu, sd = oracle.ae.norm_stats(F)
    mu, sd = mu.astype(np.float32), sd.astype(np.float32)
    plan = H.Plan(ctx)
    model = H.Model(plan, W, mu, sd, compute=compute)
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    cz = H.Compressor(plan, model, Hn, H.params(tau=1e-3, fit_codebook=True, sample_every=every), bits=bits, in_dtype=tdt)
    x = torch.from_numpy(F).cuda()
    comp = cz.compress(x)
    out = cz.decompress(comp, Hn, in_dtype=tdt).cpu().numpy()
    st = comp.stats()
    flags = comp.flags.cpu().numpy()
    codes = comp.codes.cpu().numpy()
    Cg = cz.centroids.cpu().numpy()
    check_roundtrip(F, out, flags, 1e-3, g)
    assert st["n_hist"] == Hn and st["overflow"] == 0
    # oracle pipeline on the same inputs
    model_o = dict(W=W, mu=mu.astype(np.float64), sd=sd.astype(np.float64),
                   compute="bf16" if compute == "bf16" else "fp64")
    ref = pipeline.compress(F, g, model_o, None, pipeline.Params(tau=1e-3), fit_codebook=True,
                            bits=bits, sample_every=every)
    Co = ref["codebook"]
    rng_z = np.abs(ref["z"]).max(axis=0) + 1.0
    assert np.allclose(Cg, Co, rtol=0, atol=1e-4 * rng_z.max())
    tol = 2e-5 * rng_z + np.abs(Cg - Co).max(axis=1)
    near = near_tie_codes(ref["z"], Co, Cg, tol)
    # a sample smaller than the codebook leaves duplicate centroids, whose indices may
    # differ while the dequantized values agree: compare what is unique, the values
    d = np.arange(16)[None, :]
    vdiff = np.abs(Cg[d, codes] - Co[d, ref["codes"]]) > tol[None, :]
    assert not np.any(vdiff & ~near), np.argwhere(vdiff & ~near)[:5]
    assert vdiff.sum() <= max(2, 1e-3 * vdiff.size)
    # the same histograms need a residual (decisions far from the threshold)
    assert abs(int((flags & 1).sum()) - int((ref["flags"] & 1).sum())) <= max(1, Hn // 500)
    # residual sizes agree in aggregate (the reconstructions differ by FP32 rounding only)
    assert abs(st["stream_bytes"] - len(ref["stream"])) <= 0.01 * len(ref["stream"]) + 64


def test_compress_without_model_bit_exact(H, ctx):
    say("e2e coder-only")
    g = grid.make_grid()
    F = synth.histograms(700, seed=41, dtype=np.float32)
    plan = H.Plan(ctx)
    cz = H.Compressor(plan, None, 700, H.params(tau=1e-3))
    comp = cz.compress(torch.from_numpy(F).cuda())
    out = cz.decompress(comp, 700).cpu().numpy()
    ref = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    assert comp.stream_bytes() == ref["stream"]
    assert np.array_equal(comp.offsets.cpu().numpy().astype(np.uint64), ref["offsets"])
    assert np.array_equal(comp.flags.cpu().numpy(), ref["flags"])
    assert np.allclose(out, ref["fc"], rtol=1e-12, atol=1e-14 * np.abs(F).max())
    check_roundtrip(F, out, comp.flags.cpu().numpy(), 1e-3, g)


def test_verbatim_records_bit_exact(H, ctx):
    """FP64 input with verbatim records mixed in (non-finite cells, empty histograms): the
    12,168-byte records go through the stream compaction several 2,048-byte passes at a
    time, and the stream, offsets and flags are the oracle's byte for byte; decompression
    returns the verbatim histograms bit for bit."""
    say("e2e verbatim records")
    g = grid.make_grid()
    n = 300
    F = synth.histograms(n, seed=47, dtype=np.float64)
    F[::7, 3, 5] = np.inf
    F[1::11, 20, 2] = np.nan
    F[5::13] = 0.0
    plan = H.Plan(ctx)
    cz = H.Compressor(plan, None, n, H.params(tau=1e-3), in_dtype=torch.float64)
    comp = cz.compress(torch.from_numpy(F).cuda())
    ref = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    raw = (ref["flags"] & 4) != 0
    assert raw.sum() >= 60
    assert comp.stream_bytes() == ref["stream"]
    assert np.array_equal(comp.offsets.cpu().numpy().astype(np.uint64), ref["offsets"])
    assert np.array_equal(comp.flags.cpu().numpy(), ref["flags"])
    out = cz.decompress(comp, n).cpu().numpy()
    assert out[raw].tobytes() == F[raw].tobytes()
    check_roundtrip(F[~raw], out[~raw], comp.flags.cpu().numpy()[~raw], 1e-3, g)


@pytest.mark.parametrize("lambda_fp32,no_positivity", [(True, False), (False, True)])
def test_stage5_variants_end_to_end(H, ctx, lambda_fp32, no_positivity):
    """Compress and decompress with FP32 multipliers or without positivity: the stream is
    the oracle's byte for byte, the bound holds, and the QoIs are restored to the
    variant's accuracy (FP32 multipliers: about 1e-8, Section I)."""
    say("e2e stage-5 variant", lambda_fp32, no_positivity)
    g = grid.make_grid()
    F = synth.histograms(300, seed=45, dtype=np.float32)
    plan = H.Plan(ctx)
    hp = H.params(tau=1e-3, lambda_fp32=lambda_fp32, no_positivity=no_positivity)
    cz = H.Compressor(plan, None, 300, hp)
    comp = cz.compress(torch.from_numpy(F).cuda())
    out = cz.decompress(comp, 300).cpu().numpy()
    p = pipeline.Params(tau=1e-3, lambda_fp32=lambda_fp32, positivity=not no_positivity)
    ref = pipeline.compress(F, g, None, None, p)
    assert comp.stream_bytes() == ref["stream"]
    assert np.array_equal(comp.flags.cpu().numpy(), ref["flags"])
    refout = pipeline.decompress(ref, g, None, None, 300)
    assert np.allclose(out, refout, rtol=1e-6, atol=1e-9 * np.abs(F).max())
    raw = (ref["flags"] & 4) != 0
    F64 = F.astype(np.float64)
    th = pipeline.tau_h(F64, p)
    dist = np.sqrt(((out - F64) ** 2).reshape(300, -1).sum(1))
    assert np.all(dist[~raw] <= th[~raw])
    err = moments.qoi_rel_error(moments.qoi(F64, g), moments.qoi(out, g), g)[~raw].max(axis=1)
    if lambda_fp32:
        assert 1e-11 < np.median(err) < 1e-5
    else:
        assert err.max() < 1e-10
        assert (out < 0).any()


def test_determinism_and_empty_batch(H, ctx):
    say("determinism")
    F = synth.histograms(500, seed=42, dtype=np.float32)
    W = synth.dense_ae_weights()
    mu, sd = oracle.ae.norm_stats(F)
    plan = H.Plan(ctx)
    model = H.Model(plan, W, mu, sd)
    x = torch.from_numpy(F).cuda()
    res = []
    for _ in range(2):
        cz = H.Compressor(plan, model, 500, H.params(tau=1e-3, fit_codebook=True, sample_every=2))
        c = cz.compress(x)
        res.append((c.codes.cpu().numpy(), c.lam.cpu().numpy(), c.stream_bytes(), cz.centroids.cpu().numpy(),
                    cz.decompress(c, 500).cpu().numpy()))
    for a, b in zip(res[0], res[1]):
        if isinstance(a, bytes):
            assert a == b
        else:
            assert np.array_equal(a, b)
    say("empty batch")
    cz = H.Compressor(plan, model, 4, H.params(tau=1e-3))
    c = cz.compress(x[:0])
    assert c.stats()["n_hist"] == 0 and int(c.offsets[0].item()) == 0


@pytest.mark.parametrize("with_model", [False, True])
def test_full_scale_batch(H, ctx, with_model):
    """2^20 histograms of 39x39 FP32, the configuration the benchmark times."""
    Hn = 1 << 20
    say("full scale", "model" if with_model else "coder-only", Hn)
    g = grid.make_grid()
    F = synth.histograms(Hn, seed=synth.SEED_PLAIN_LARGE, dtype=np.float32)
    plan = H.Plan(ctx)
    W = synth.dense_ae_weights()
    model = model_o = None
    if with_model:
        x = torch.from_numpy(F).cuda()
        mu, sd = oracle.ae.norm_stats(F[::16])
        mu, sd = mu.astype(np.float32), sd.astype(np.float32)
        model = H.Model(plan, W, mu, sd)
        model_o = dict(W=W, mu=mu.astype(np.float64), sd=sd.astype(np.float64))
    else:
        x = torch.from_numpy(F).cuda()
    cz = H.Compressor(plan, model, Hn, H.params(tau=1e-3, fit_codebook=with_model, sample_every=16))
    comp = cz.compress(x)
    st = comp.stats()
    assert st["n_hist"] == Hn and st["overflow"] == 0
    out = cz.decompress(comp, Hn)
    # bound and QoIs on every histogram, evaluated on the device from the GPU's own output
    _, q0, n0 = H.qoi(plan, x)
    _, q1, _ = H.qoi(plan, out)
    ok = (comp.flags & 4) == 0
    dist = (out - x.double()).reshape(Hn, -1).norm(dim=1)
    assert bool(((dist <= 1e-3 * n0) | ~ok).all())
    den = torch.stack([q0[:, 0].abs(), torch.maximum(q0[:, 1].abs(), q0[:, 3].abs().sqrt()),
                       q0[:, 2].abs(), q0[:, 3].abs()], 1)
    assert ((q1 - q0).abs() / den)[ok].max().item() < 1e-10
    rng = np.random.default_rng(43)
    sample = np.sort(rng.choice(Hn, 128, replace=False))
    off = comp.offsets.cpu().numpy().astype(np.int64)
    flags = comp.flags.cpu().numpy()
    # the same bound and QoIs on the sampled histograms by the oracle's own formulas (FP64,
    # NumPy) rather than the library's moment kernel
    Fs = F[sample].astype(np.float64)
    outs = out[torch.from_numpy(sample).cuda()].cpu().numpy()
    oks = (flags[sample] & 4) == 0
    th = pipeline.tau_h(Fs, pipeline.Params(tau=1e-3))
    d = np.sqrt(((outs - Fs) ** 2).reshape(len(sample), -1).sum(1))
    assert np.all(d[oks] <= th[oks])
    assert moments.qoi_rel_error(moments.qoi(Fs, g), moments.qoi(outs, g), g)[oks].max() < 1e-10
    if not with_model:
        ref = pipeline.compress(F[sample], g, None, None, pipeline.Params(tau=1e-3))
        stream = comp.stream
        for k, h in enumerate(sample):
            rec = bytes(stream[off[h]:off[h + 1]].cpu().numpy().tobytes())
            assert rec == ref["stream"][int(ref["offsets"][k]):int(ref["offsets"][k + 1])], h
        assert np.array_equal(flags[sample], ref["flags"])
        lam = comp.lam.cpu().numpy()[sample]
        assert np.allclose(lam, ref["lam"], rtol=1e-7, atol=1e-9 * np.abs(ref["lam"]).max())
    else:
        # codebook: the oracle fits it on the oracle's latents of the same every-16th sample
        Zs = oracle.ae.dense_encode(oracle.ae.normalize(F[::16], model_o["mu"], model_o["sd"]), W)
        Co = pq.fit(Zs, 8, 1)
        Cg = cz.centroids.cpu().numpy()
        rng_z = np.abs(Zs).max(axis=0) + 1.0
        close = np.isclose(Cg, Co, rtol=0, atol=1e-4 * rng_z[:, None])
        assert close.mean() > 0.99, close.mean()
        zs = oracle.ae.dense_encode(oracle.ae.normalize(F[sample], model_o["mu"], model_o["sd"]), W)
        codes_o = pq.encode(zs, Co)
        codes = comp.codes.cpu().numpy()[sample]
        tol = 2e-5 * rng_z + np.abs(Cg - Co).max(axis=1)
        near = near_tie_codes(zs, Co, Cg, tol)
        diff = codes != codes_o
        assert not np.any(diff & ~near)


@pytest.mark.parametrize("shape,tau,variant,Hn", [((39, 39), 1e-2, "auto", 400), ((39, 39), 1e-3, "auto", 400),
                                                  ((33, 37), 1e-2, "auto", 400),
                                                  ((39, 39), 1e-2, "block_256x6", 400),
                                                  ((49, 49), 1e-2, "auto", 120)])
def test_kl_correction_end_to_end(H, ctx, shape, tau, variant, Hn):
    """The KL reading of Stage 5 (kept where it keeps the bound, the L2 projection
    elsewhere), coder-only, on the wave kernels (39 x 39 compiled, 33 x 37 run-time tables)
    and the workgroup kernel (39 x 39 by its variant, 49 x 49, which the wave-team kernels
    leave to it for this reading): records byte-exact, flags equal to the oracle's wherever
    the KL bound decision is not a near-tie, multipliers to 1e-7, the bound, the QoIs and
    non-negativity on the GPU's own output."""
    n_perp, n_par = shape
    say("kl", shape, tau, variant)
    g = grid.make_grid(n_par, n_perp)
    F = synth.histograms(Hn, n_par, n_perp, seed=44, dtype=np.float32)
    plan = H.Plan(ctx, n_par, n_perp)
    plan.set_variant(variant)
    cz = H.Compressor(plan, None, Hn, H.params(tau=tau, kl=True))
    comp = cz.compress(torch.from_numpy(F).cuda())
    out = cz.decompress(comp, Hn).cpu().numpy()
    flags = comp.flags.cpu().numpy()
    ref = pipeline.compress(F, g, None, None, pipeline.Params(tau=tau, kl=True))
    assert comp.stream_bytes() == ref["stream"]
    # where the oracle's KL result sits within 1e-9 of the bound the decision may differ
    F64 = F.astype(np.float64)
    th = pipeline.tau_h(F64, pipeline.Params(tau=tau))
    A = g.A()
    near = np.zeros(Hn, bool)
    for h in range(Hn):
        if ref["flags"][h] & 4:
            continue
        ft = ref["ft"][h].reshape(-1)
        r = oracle.newton.project_kl(ft.reshape(n_perp, n_par), A @ F64[h].reshape(-1), g)
        if r["status"] < 2:
            d = np.sqrt(((F64[h].reshape(-1) - r["x"].reshape(-1)) ** 2).sum())
            near[h] = abs(d - (1 - 2.0 ** -20) * th[h]) <= 1e-9 * th[h]
    same = flags == ref["flags"]
    assert np.all(same | near), np.nonzero(~same & ~near)[0][:5]
    kl = (flags & 32) != 0
    assert kl.any() and not kl.all()
    ok = same & ((flags & 4) == 0)
    lam = comp.lam.cpu().numpy()
    assert np.allclose(lam[ok], ref["lam"][ok], rtol=1e-7, atol=1e-9 * np.abs(ref["lam"][ok]).max())
    check_roundtrip(F, out, flags, tau, g)
    assert np.all(out[kl] >= 0)
    assert np.allclose(out[ok], ref["fc"][ok], rtol=1e-10, atol=1e-13 * np.abs(F).max())


@pytest.mark.parametrize("with_model", [False, True])
def test_container_round_trip_through_decompression(H, ctx, with_model):
    """Compress, copy to the host, pack the container with rANS, unpack, copy back and
    decompress: the same histograms bit for bit as decompressing the original arrays."""
    say("container", with_model)
    Hn = 2000
    F = synth.histograms(Hn, seed=45, dtype=np.float32)
    plan = H.Plan(ctx)
    model, kw = None, {}
    if with_model:
        W = synth.dense_ae_weights()
        mu, sd = oracle.ae.norm_stats(F)
        mu, sd = mu.astype(np.float32), sd.astype(np.float32)
        model = H.Model(plan, W, mu, sd)
        kw = dict(weights=H.pack_dense_weights(W), norm_mean=mu, norm_std=sd, arch="dense", compute="fp32")
    cz = H.Compressor(plan, model, Hn, H.params(tau=1e-3, fit_codebook=with_model, sample_every=4))
    comp = cz.compress(torch.from_numpy(F).cuda())
    ref = cz.decompress(comp, Hn).cpu().numpy()
    off = comp.offsets.cpu().numpy().astype(np.uint64)
    if with_model:
        kw.update(codes=comp.codes.cpu().numpy(), centroids=cz.centroids.cpu().numpy())
    buf = H.container_pack(39, 39, comp.flags.cpu().numpy(), off, np.frombuffer(comp.stream_bytes(), np.uint8),
                           comp.lam.cpu().numpy(), entropy=True, **kw)
    plain = H.container_pack(39, 39, comp.flags.cpu().numpy(), off, np.frombuffer(comp.stream_bytes(), np.uint8),
                             comp.lam.cpu().numpy(), entropy=False, **kw)
    assert len(buf) < len(plain)
    d = H.container_unpack(buf)
    back = H.alloc_compressed(Hn, plan.N, "cuda")
    back.flags.copy_(torch.from_numpy(d["flags"]))
    back.offsets.copy_(torch.from_numpy(d["res_offset"].astype(np.int64)))
    back.stream[:d["res_bytes"].size].copy_(torch.from_numpy(d["res_bytes"]))
    back.lam.copy_(torch.from_numpy(d["lam"]))
    if with_model:
        back.codes.copy_(torch.from_numpy(d["codes"]))
        m2 = H.Model(plan, H.unpack_dense_weights(d["weights"], plan.N), d["norm_mean"], d["norm_std"])
        cz2 = H.Compressor(plan, m2, Hn, H.params(tau=1e-3))
        cz2.centroids.copy_(torch.from_numpy(d["centroids"]))
    else:
        cz2 = cz
    out = cz2.decompress(back, Hn).cpu().numpy()
    assert np.array_equal(out, ref)


@pytest.mark.parametrize("bits", [12, 30])
def test_multiplier_truncation(H, ctx, bits):
    """Multipliers rounded to `bits` mantissa bits: at most that many bits set, equal to the
    oracle's rounded multipliers up to the Newton tolerance and one unit in the last kept
    place, records byte-exact, QoI error of the order of 2^-bits."""
    say("lambda bits", bits)
    g = grid.make_grid()
    F = synth.histograms(500, seed=46, dtype=np.float32)
    cz = H.Compressor(H.Plan(ctx), None, 500, H.params(tau=1e-3, lambda_bits=bits))
    comp = cz.compress(torch.from_numpy(F).cuda())
    lam = comp.lam.cpu().numpy()
    assert np.all((lam.view(np.uint64) & np.uint64((1 << (52 - bits)) - 1)) == 0)
    ref = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3, lambda_bits=bits))
    assert comp.stream_bytes() == ref["stream"]
    ok = (ref["flags"] & 4) == 0
    # the unrounded multipliers agree to the Newton tolerance (1e-7 relative, 1e-9 of the
    # largest), the rounding adds at most one unit in the last kept place
    scale = np.abs(ref["lam"][ok]).max()
    assert np.all(np.abs(lam[ok] - ref["lam"][ok]) <= (2.0 ** -bits + 1e-7) * np.abs(ref["lam"][ok]) + 1e-9 * scale)
    out = cz.decompress(comp, 500).cpu().numpy()
    err = moments.qoi_rel_error(moments.qoi(F.astype(np.float64), g), moments.qoi(out, g), g)[ok]
    assert 2.0 ** -(bits + 12) < err.max() < 2.0 ** -(bits - 10)


@pytest.mark.parametrize("shape,level", [((39, 39), 0), ((39, 39), 7), ((39, 39), 40), ((33, 37), 3),
                                         ((65, 65), 0), ((65, 65), 9)])
def test_user_specified_step_end_to_end(H, ctx, shape, level):
    """The 'ub' setting (the coder's step given, no search) on the compiled 39 x 39 wave
    kernel, the run-time-table wave kernel (33 x 37) and the workgroup kernel (65 x 65),
    coder-only: records and flags byte-exact against the oracle, k* equal to the level on
    every coded histogram, decompressed data equal to the oracle's, and at level 0 the
    bound and the QoIs on the GPU's own output."""
    n_perp, n_par = shape
    say("ub", shape, level)
    g = grid.make_grid(n_par, n_perp)
    Hn = 300
    F = synth.histograms(Hn, n_par, n_perp, seed=47, dtype=np.float32)
    cz = H.Compressor(H.Plan(ctx, n_par, n_perp), None, Hn, H.params(tau=1e-3, ub_level=level))
    comp = cz.compress(torch.from_numpy(F).cuda())
    ref = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3, ub_level=level))
    flags = comp.flags.cpu().numpy()
    assert comp.stream_bytes() == ref["stream"]
    assert np.array_equal(flags, ref["flags"])
    coded = (flags & 5) == 1
    assert coded.any() and np.all(ref["kstar"][coded] == level)
    out = cz.decompress(comp, Hn).cpu().numpy()
    refout = pipeline.decompress(ref, g, None, None, Hn)
    assert np.allclose(out, refout, rtol=1e-10, atol=1e-13 * np.abs(F).max())
    if level == 0:
        check_roundtrip(F, out, flags, 1e-3, g)


@pytest.mark.parametrize("shape,search", [((39, 39), "bisect"), ((39, 39), "guided"), ((33, 37), "bisect"),
                                          ((65, 65), "bisect"), ((65, 65), "guided")])
def test_search_modes_end_to_end(H, ctx, shape, search):
    """Both ways of searching the coder's step (exponential search from the predicted index,
    or bisection over the whole ladder) on the three kernel paths, coder-only, at a tight
    and a loose bound: records, offsets and flags byte-exact against the oracle's same
    search, the bound and the QoIs on the GPU's own output."""
    n_perp, n_par = shape
    g = grid.make_grid(n_par, n_perp)
    Hn = 300
    F = synth.histograms(Hn, n_par, n_perp, seed=48, dtype=np.float32)
    for tau in (1e-4, 3e-2):
        say("search", shape, search, tau)
        cz = H.Compressor(H.Plan(ctx, n_par, n_perp), None, Hn, H.params(tau=tau, search=search))
        comp = cz.compress(torch.from_numpy(F).cuda())
        ref = pipeline.compress(F, g, None, None, pipeline.Params(tau=tau, search=search))
        assert comp.stream_bytes() == ref["stream"]
        assert np.array_equal(comp.offsets.cpu().numpy().astype(np.uint64), ref["offsets"])
        assert np.array_equal(comp.flags.cpu().numpy(), ref["flags"])
        check_roundtrip(F, cz.decompress(comp, Hn).cpu().numpy(), comp.flags.cpu().numpy(), tau, g)


@pytest.mark.parametrize("Hn,dtype,every", [(256, np.float64, 1), (1000, np.float32, 4)])
def test_fp64_form_end_to_end(H, ctx, Hn, dtype, every):
    """The FP64 form of the autoencoder (every layer in FP64, z and fhat stored as FP32)
    against the oracle's FP64 model with the same FP32 staging: the two sum in different
    orders, so a stored value may differ in its last FP32 place only where the FP64 sums
    straddle a rounding boundary.  Where z agrees everywhere (the expected case) the
    codebook, every code, every flag and every record byte must agree; the bound and the
    QoIs hold on the GPU's own output."""
    say("e2e fp64 form", Hn, dtype.__name__, every)
    g = grid.make_grid()
    F = synth.histograms(Hn, seed=synth.SEED_PLAIN_SMALL, dtype=dtype)
    W = synth.dense_ae_weights()
    mu, sd = oracle.ae.norm_stats(F)
    mu, sd = mu.astype(np.float32), sd.astype(np.float32)
    plan = H.Plan(ctx)
    model = H.Model(plan, W, mu, sd, compute="fp64")
    model_o = dict(W=W, mu=mu.astype(np.float64), sd=sd.astype(np.float64), compute="fp64_staged")
    tdt = torch.float64 if dtype == np.float64 else torch.float32
    x = torch.from_numpy(F).cuda()
    z = H.encode(model, x).cpu().numpy().astype(np.float64)
    z_o = pipeline.encode_ae(F.astype(np.float64), model_o)
    zdiff = z != z_o
    assert zdiff.sum() <= 2
    assert np.all(np.abs(z - z_o)[zdiff] <= np.spacing(np.abs(z_o[zdiff]).astype(np.float32)))
    cz = H.Compressor(plan, model, Hn, H.params(tau=1e-3, fit_codebook=True, sample_every=every), in_dtype=tdt)
    comp = cz.compress(x)
    out = cz.decompress(comp, Hn, in_dtype=tdt).cpu().numpy()
    flags = comp.flags.cpu().numpy()
    check_roundtrip(F, out, flags, 1e-3, g)
    ref = pipeline.compress(F, g, model_o, None, pipeline.Params(tau=1e-3), fit_codebook=True, bits=8,
                            sample_every=every)
    Cg = cz.centroids.cpu().numpy()
    codes = comp.codes.cpu().numpy()
    if not zdiff.any():
        assert np.array_equal(Cg, ref["codebook"].astype(np.float32))
        assert np.array_equal(codes, ref["codes"])
        # the decoder's FP32 fhat may also differ in a last place where the FP64 sums
        # straddle a rounding boundary; every histogram whose fhat agrees must agree byte
        # for byte
        fh = H.decode(model, comp.codes, cz.centroids).cpu().numpy().astype(np.float64)
        same = (fh.reshape(Hn, -1) == ref["fhat"].reshape(Hn, -1)).all(axis=1)
        assert same.mean() >= 0.99
        assert np.array_equal(flags[same], ref["flags"][same])
        off_g, off_o = comp.offsets.cpu().numpy().astype(np.int64), ref["offsets"].astype(np.int64)
        st_g, st_o = comp.stream_bytes(), ref["stream"]
        for h in np.nonzero(same)[0]:
            assert st_g[off_g[h]:off_g[h + 1]] == st_o[off_o[h]:off_o[h + 1]], h
        if same.all():
            assert st_g == st_o
