"""The convolutional autoencoder (BF16 form, 39 x 39 grids) on the GPU against the oracle:
encoder and decoder within bounds derived from the FP32 accumulations, and the whole
compress / decompress path with it (GPU)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import conv, grid, pipeline, pq
from paper_2212_10733_amd import synth

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -24


@pytest.fixture(scope="module")
def H():
    from paper_2212_10733_amd import hcz
    return hcz


@pytest.fixture(scope="module")
def ctx(H):
    return H.Context(0)


def say(*a):
    print("[case]", *a, flush=True)


def model(H, plan, F, seed=0):
    W = synth.conv_ae_weights(seed)
    rng = np.random.default_rng(seed + 200)
    for k in ("c1b", "c2b", "fb", "db", "t1b", "t2b"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    mu, sd = oracle.ae.norm_stats(F.astype(np.float64))
    mu, sd = mu.astype(np.float32), sd.astype(np.float32)
    return W, mu, sd, H.Model(plan, W, mu, sd, compute="bf16", arch="conv")


def absconv(x, w, b):
    return conv.conv2d_s2(np.abs(x), np.abs(np.asarray(w, np.float64)), np.abs(np.asarray(b, np.float64)))


@pytest.mark.parametrize("Hn,dtype,pad", [(200, np.float32, 0), (77, np.float64, 0), (50, np.float32, 5),
                                          (16384 + 37, np.float32, 0)])
def test_conv_encode_parity(H, ctx, Hn, dtype, pad):
    """conv1 and its bfloat16 rounding are the oracle's bit for bit (same FP32 chain), so z
    differs only by FP32 accumulation: at most ~25 roundings of conv2's running sums (18
    matrix-core steps plus the instruction's own) and ~3,200 in the dense layer (a
    matrix-core accumulation over K = 6400 in steps of two)."""
    say("conv encode", Hn, dtype.__name__, pad)
    plan = H.Plan(ctx)
    F = synth.histograms(Hn, seed=60, dtype=dtype)
    F[2, 5, 7] = np.inf
    W, mu, sd, m = model(H, plan, F[3:])
    x = torch.from_numpy(F).cuda()
    if pad:
        xp = torch.zeros((Hn, 39, 39 + pad), dtype=x.dtype, device=x.device)
        xp[:, :, :39] = x
        x = xp[:, :, :39]
    z = H.encode(m, x).cpu().numpy()
    rsd = np.float32(1) / sd
    if Hn > 1000:   # a batch spanning two internal chunks: check rows around the boundary
        rows = np.r_[0:40, 16384 - 40:min(Hn, 16384 + 40), Hn - 10:Hn]
        z, F = z[rows], F[rows]
        Hn = len(rows)
    zo = conv.encode_bf16(F.astype(np.float32), mu, rsd, W)
    h1b = conv.bf16(conv.conv1_fp32(conv._x32(F.astype(np.float32), mu, rsd), W["c1w"], W["c1b"])).astype(np.float64)
    w2b = conv.bf16(W["c2w"]).astype(np.float64)
    s2 = absconv(h1b, w2b, W["c2b"]).reshape(Hn, 6400)
    h2 = np.maximum(conv.conv2d_s2(h1b, w2b, W["c2b"]), 0).reshape(Hn, 6400)
    fw = np.abs(W["fw"].astype(np.float64))
    bound = 30 * EPS * (s2 @ fw.T) + 3300 * EPS * (np.abs(h2) @ fw.T + np.abs(W["fb"]))
    err = np.abs(z - zo)
    assert np.all(err <= bound), (err / bound).max()


def test_conv_decode_parity(H, ctx):
    """hd and its bfloat16 rounding are the oracle's bit for bit; fhat differs by FP32
    accumulation in the transposed convolutions and the final sigma y + mu."""
    say("conv decode")
    plan = H.Plan(ctx)
    F = synth.histograms(64, seed=61, dtype=np.float32)
    W, mu, sd, m = model(H, plan, F)
    C = synth.sorted_codebook(16, 8, seed=62)
    codes = synth.codes(300, 16, 8, seed=63)
    fh = H.decode(m, torch.from_numpy(codes).cuda(), torch.from_numpy(C).cuda()).cpu().numpy().reshape(300, -1)
    Zh = pq.decode(codes, C)
    ref = conv.decode_bf16(Zh, W, mu, sd)
    hdb = conv.bf16(conv.dec_hidden_fp32(Zh, W)).astype(np.float64).reshape(300, 64, 10, 10)
    t1b = conv.bf16(W["t1w"]).astype(np.float64)
    s3 = conv.conv_t2d_s2(np.abs(hdb), np.abs(t1b), np.abs(W["t1b"].astype(np.float64)), 20)
    h3 = np.maximum(conv.conv_t2d_s2(hdb, t1b, W["t1b"], 20), 0)
    aw = np.abs(W["t2w"].astype(np.float64))
    prop = conv.conv_t2d_s2(s3, aw, np.zeros(1), 39).reshape(300, -1)
    direct = conv.conv_t2d_s2(np.abs(h3), aw, np.abs(W["t2b"].astype(np.float64)), 39).reshape(300, -1)
    bound = sd * (25 * EPS * prop + 140 * EPS * direct) + 2 * EPS * np.abs(ref) + 1e-30
    err = np.abs(fh - ref)
    assert np.all(err <= bound), (err / bound).max()
    fh2 = H.decode(m, torch.from_numpy(codes).cuda(), torch.from_numpy(C).cuda()).cpu().numpy().reshape(300, -1)
    assert np.array_equal(fh, fh2)


def test_conv_compress_end_to_end(H, ctx):
    """hcz_compress / hcz_decompress with the convolutional model: the bound and QoIs on
    every histogram, codes equal to the oracle's away from near-ties, the same
    histograms coded and a residual stream of the same size."""
    say("conv e2e")
    g = grid.make_grid()
    Hn = 1500
    F = synth.histograms(Hn, seed=64, dtype=np.float32)
    W, mu, sd, m = model(H, H.Plan(ctx), F)
    plan = m.plan
    cz = H.Compressor(plan, m, Hn, H.params(tau=1e-3, fit_codebook=True, sample_every=4))
    comp = cz.compress(torch.from_numpy(F).cuda())
    out = cz.decompress(comp, Hn).cpu().numpy()
    flags = comp.flags.cpu().numpy()
    th = pipeline.tau_h(F.astype(np.float64), pipeline.Params(tau=1e-3))
    raw = (flags & 4) != 0
    dist = np.sqrt(((out - F.astype(np.float64)) ** 2).reshape(Hn, -1).sum(1))
    assert np.all(dist[~raw] <= th[~raw])
    from oracle import moments
    err = moments.qoi_rel_error(moments.qoi(F.astype(np.float64), g), moments.qoi(out, g), g)[~raw]
    assert err.max() < 1e-10
    ref = pipeline.compress(F, g, dict(arch="conv", W=W, mu=mu.astype(np.float64), sd=sd.astype(np.float64)),
                            None, pipeline.Params(tau=1e-3), fit_codebook=True, sample_every=4)
    Cg, Co = cz.centroids.cpu().numpy(), ref["codebook"]
    rng_z = np.abs(ref["z"]).max(axis=0) + 1.0
    assert np.allclose(Cg, Co, rtol=0, atol=1e-4 * rng_z.max())
    codes = comp.codes.cpu().numpy()
    d = np.arange(16)[None, :]
    tol = 2e-5 * rng_z + np.abs(Cg - Co).max(axis=1)
    vdiff = np.abs(Cg[d, codes] - Co[d, ref["codes"]]) > tol[None, :]
    assert vdiff.sum() <= max(2, 1e-3 * vdiff.size)
    assert abs(int((flags & 1).sum()) - int((ref["flags"] & 1).sum())) <= max(1, Hn // 500)
    st = comp.stats()
    assert abs(st["stream_bytes"] - len(ref["stream"])) <= 0.01 * len(ref["stream"]) + 64
