"""The learned part on the GPU: the dense autoencoder's hand-written forward/backward
kernels against the oracle (FP64) and central finite differences, Adam, the z-score
statistics, and what training buys in compression (GPU)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import grid, moments
from paper_2212_10733_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def T():
    from paper_2212_10733_amd import hcz, train
    return hcz, train


def say(*a):
    print("[case]", *a, flush=True)


def weights(N, seed=5):
    W = synth.dense_ae_weights(N, seed=seed)
    rng = np.random.default_rng(seed)
    for k in ("b1", "b2", "b3", "b4"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    return W


def inputs(B, N, seed=6):
    F = synth.histograms(B, seed=seed, dtype=np.float32).reshape(B, -1)[:, :N]
    mu, sd = oracle.ae.norm_stats(F)
    return ((F - mu) / sd).astype(np.float32)


@pytest.mark.parametrize("B", [64, 200])
def test_forward_backward_parity(T, B):
    hcz, train = T
    N = 1521
    say("ae fwd/bwd", B)
    W = weights(N)
    X = inputs(B, N)
    p = train.pack(W).requires_grad_(True)
    x = torch.from_numpy(X).cuda()
    z, xh = train.DenseAE.apply(x, p)
    loss = train.mse(xh, x)
    loss.backward()
    torch.cuda.synchronize()
    W64 = {k: v.astype(np.float64) for k, v in W.items()}
    cache = oracle.ae.dense_forward_train(X.astype(np.float64), W64)
    assert np.allclose(z.detach().cpu().numpy(), cache["z"], rtol=1e-4, atol=1e-4 * np.abs(cache["z"]).max())
    assert np.allclose(xh.detach().cpu().numpy(), cache["xh"], rtol=1e-4, atol=1e-4 * np.abs(cache["xh"]).max())
    assert loss.item() == pytest.approx(oracle.ae.mse(cache["xh"], X.astype(np.float64)), rel=1e-5)
    g_or = oracle.ae.dense_backward(cache, W64)
    g = train.unpack(p.grad, N)
    for k in train.KEYS:
        scale = np.abs(g_or[k]).max() + 1e-30
        err = np.abs(g[k] - g_or[k]).max() / scale
        assert err < 2e-4, (k, err)
    # central finite differences of the FP64 loss at sampled coordinates
    rng = np.random.default_rng(7)
    for k in train.KEYS:
        for _ in range(2):
            idx = tuple(rng.integers(0, s) for s in W64[k].shape)
            Wp = {kk: vv.copy() for kk, vv in W64.items()}
            Wm = {kk: vv.copy() for kk, vv in W64.items()}
            h = 1e-6 * max(1.0, abs(W64[k][idx]))
            Wp[k][idx] += h
            Wm[k][idx] -= h
            fd = (oracle.ae.dense_loss(X.astype(np.float64), Wp) - oracle.ae.dense_loss(X.astype(np.float64), Wm)) / (2 * h)
            assert g[k][idx] == pytest.approx(fd, rel=2e-3, abs=2e-4 * (np.abs(g_or[k]).max() + 1e-12)), (k, idx)


def test_latent_and_input_gradients(T):
    hcz, train = T
    say("dz / dx")
    N, B = 1521, 48
    W = weights(N, seed=8)
    X = inputs(B, N, seed=9)
    dz = np.random.default_rng(10).normal(size=(B, 16)).astype(np.float32)
    p = train.pack(W).requires_grad_(True)
    x = torch.from_numpy(X).cuda().requires_grad_(True)
    z, xh = train.DenseAE.apply(x, p)
    ((z * torch.from_numpy(dz).cuda()).sum() + train.mse(xh, x.detach())).backward()
    # reference: torch autograd on the CPU in FP64 (library routine)
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in W.items()}
    xt = torch.tensor(X, dtype=torch.float64, requires_grad=True)
    h1 = torch.relu(xt @ t["W1"].T + t["b1"])
    zt = h1 @ t["W2"].T + t["b2"]
    xht = torch.relu(zt @ t["W3"].T + t["b3"]) @ t["W4"].T + t["b4"]
    ((zt * torch.tensor(dz, dtype=torch.float64)).sum() + ((xht - xt.detach()) ** 2).mean()).backward()
    assert np.allclose(x.grad.cpu().numpy(), xt.grad.numpy(), rtol=1e-3, atol=2e-4 * np.abs(xt.grad.numpy()).max())
    g = train.unpack(p.grad, N)
    for k in train.KEYS:
        ref = t[k].grad.numpy()
        assert np.abs(g[k] - ref).max() <= 2e-4 * (np.abs(ref).max() + 1e-30), k


def test_adam_and_norm_stats(T):
    hcz, train = T
    say("adam")
    rng = np.random.default_rng(11)
    p0 = rng.normal(size=5000).astype(np.float32)
    tr = train.Trainer(torch.from_numpy(p0).cuda(), lr=1e-2)
    params = {"w": p0.astype(np.float64)}
    state = {}
    for _ in range(5):
        gr = rng.normal(size=5000).astype(np.float32)
        tr.step(torch.from_numpy(gr).cuda())
        oracle.ae.adam_step(params, {"w": gr.astype(np.float64)}, state, lr=1e-2)
    assert np.allclose(tr.p.cpu().numpy(), params["w"], rtol=1e-5, atol=1e-6)
    say("norm stats")
    ctx = hcz.Context(0)
    plan = hcz.Plan(ctx)
    F = synth.histograms(1000, seed=12, dtype=np.float32)
    F[:, 0, 0] = 0.5                      # a constant pixel gets the floored std
    mu, sd = hcz.norm_stats(plan, torch.from_numpy(F).cuda())
    mo, so = oracle.ae.norm_stats(F)
    assert np.allclose(mu.cpu().numpy(), mo, rtol=1e-6, atol=1e-12)
    assert np.allclose(sd.cpu().numpy(), so, rtol=1e-5, atol=1e-18)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_column_stats_and_normalize(T, dtype):
    """Column statistics of a strided matrix against the oracle's z-score statistics, and
    the FP32 z-scoring of training rows bit for bit against NumPy's FP32 subtraction and
    division (both IEEE round to nearest)."""
    hcz, train = T
    say("column stats / normalize", dtype.__name__)
    rng = np.random.default_rng(13)
    X = (rng.standard_normal((3000, 37)) * rng.random(37) * 5 + rng.standard_normal(37)).astype(dtype)
    X[:, 4] = 1.5                                          # constant column: floored std
    pad = np.zeros((3000, 40), dtype)
    pad[:, :37] = X
    xd = torch.from_numpy(pad).cuda()[:, :37]              # row stride 40
    mu, sd = hcz.column_stats(xd)
    mo, so = oracle.ae.norm_stats(X)
    assert np.allclose(mu.cpu().numpy(), mo, rtol=1e-6, atol=1e-7)
    assert np.allclose(sd.cpu().numpy(), so, rtol=1e-5, atol=1e-18)
    out = hcz.column_normalize(xd, mu, sd).cpu().numpy()
    m32, s32 = mu.cpu().numpy(), sd.cpu().numpy()
    want = (X.astype(np.float32) - m32) / s32
    assert out.dtype == np.float32 and np.array_equal(out, want)
    out = hcz.column_normalize(xd, None, sd).cpu().numpy()
    assert np.array_equal(out, X.astype(np.float32) / s32)
    F = synth.histograms(50, seed=14, dtype=np.float32)
    x = torch.from_numpy(F).cuda()
    m, s = hcz.column_stats(x)
    assert np.array_equal(hcz.column_normalize(x, m, s).cpu().numpy(),
                          (F.reshape(50, -1) - m.cpu().numpy()) / s.cpu().numpy())


def test_training_reduces_loss_and_residuals(T):
    hcz, train = T
    say("training")
    ctx = hcz.Context(0)
    plan = hcz.Plan(ctx)
    Ftr = torch.from_numpy(synth.histograms(16384, seed=synth.SEED_TRAIN, dtype=np.float32)).cuda()
    Fte = torch.from_numpy(synth.histograms(4096, seed=synth.SEED_HELDOUT, dtype=np.float32)).cuda()
    mu, sd = hcz.norm_stats(plan, Ftr)
    X = ((Ftr.reshape(16384, -1) - mu) / sd).contiguous()
    W0 = synth.dense_ae_weights()
    tr = train.Trainer(train.pack(W0), lr=1e-3)
    losses = tr.fit(X, epochs=8, batch=1024)
    assert losses[-1] < 0.5 * losses[0]
    res = {}
    for name, W in (("untrained", W0), ("trained", train.unpack(tr.p, 1521))):
        model = hcz.Model(plan, W, mu.cpu().numpy(), sd.cpu().numpy())
        cz = hcz.Compressor(plan, model, 4096, hcz.params(tau=1e-2, fit_codebook=True, sample_every=1))
        c = cz.compress(Fte)
        st = c.stats()
        res[name] = (st["n_coded"], st["stream_bytes"])
        out = cz.decompress(c, 4096).cpu().numpy()
        g = grid.make_grid()
        F = Fte.cpu().numpy().astype(np.float64)
        q0, q1 = moments.qoi(F, g), moments.qoi(out, g)
        assert moments.qoi_rel_error(q0, q1, g).max() < 1e-10
    assert res["trained"][0] <= res["untrained"][0]
    assert res["trained"][1] < 0.9 * res["untrained"][1]


def test_mlp_kernels_match_oracle(T):
    hcz, train = T
    from oracle import mlp as omlp
    say("mlp fwd/bwd/predict")
    P = synth.mlp_weights()
    rng = np.random.default_rng(13)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.normal(0, 0.1, P[k].shape).astype(np.float32)
    Z = rng.normal(size=(300, 16)).astype(np.float32)
    Tg = rng.normal(size=(300, 4)).astype(np.float32)
    p = train.mlp_pack(P).requires_grad_(True)
    out = train.MlpNet.apply(torch.from_numpy(Z).cuda(), p)
    loss = train.mse(out, torch.from_numpy(Tg).cuda())
    loss.backward()
    P64 = {k: v.astype(np.float64) for k, v in P.items()}
    cache = omlp.forward(Z.astype(np.float64), P64)
    assert np.allclose(out.detach().cpu().numpy(), cache["out"], rtol=1e-4, atol=1e-5)
    g_or = omlp.backward(cache, Tg.astype(np.float64), P64)
    g = train.mlp_unpack(p.grad)
    for k in train.MLP_KEYS:
        assert np.abs(g[k] - g_or[k]).max() <= 2e-4 * (np.abs(g_or[k]).max() + 1e-30), k
    # inference kernel on codes + codebook, with the output scale
    ctx = hcz.Context(0)
    C = synth.sorted_codebook(16, 8, seed=14)
    codes = synth.codes(500, 16, 8, seed=15)
    scale = np.array([1e-3, 2e-2, 3.0, 4e-1])
    net = hcz.Mlp(ctx, train.mlp_pack(P).cpu().numpy(), scale)
    lam0 = net.predict(torch.from_numpy(codes).cuda(), torch.from_numpy(C).cuda()).cpu().numpy()
    ref = omlp.predict(oracle.pq.decode(codes, C), P64, scale)
    assert np.allclose(lam0, ref, rtol=1e-4, atol=1e-5 * np.abs(ref).max(axis=0))
    zq = hcz.dequantize(torch.from_numpy(codes).cuda(), torch.from_numpy(C).cuda()).cpu().numpy()
    assert np.array_equal(zq, oracle.pq.decode(codes, C).astype(np.float32))


def test_warm_start_network_cuts_newton_iterations(T):
    """Train the warm-start network on the multipliers of a training batch, then compress
    held-out data cold and warm: same multipliers and QoIs, fewer Newton updates."""
    hcz, train = T
    say("warm-start training")
    ctx = hcz.Context(0)
    plan = hcz.Plan(ctx)
    Ftr = torch.from_numpy(synth.histograms(32768, seed=synth.SEED_TRAIN, dtype=np.float32)).cuda()
    Fte = torch.from_numpy(synth.histograms(8192, seed=synth.SEED_HELDOUT, dtype=np.float32)).cuda()
    mu, sd = hcz.norm_stats(plan, Ftr)
    W = synth.dense_ae_weights()
    model = hcz.Model(plan, W, mu.cpu().numpy(), sd.cpu().numpy())
    # targets: cold-start multipliers of the training batch (tau large: most histograms uncoded)
    p_cold = hcz.params(tau=0.5, fit_codebook=True, sample_every=4)
    cz = hcz.Compressor(plan, model, 32768, p_cold)
    c = cz.compress(Ftr)
    lam = c.lam.clone()
    codes = c.codes.clone()
    cent = cz.centroids.clone()
    ok = (c.flags & 4) == 0
    scale = lam[ok].std(dim=0).clamp_min(1e-30)
    Z = hcz.dequantize(codes, cent)[ok]
    Tt = (lam[ok] / scale).float()
    # the latent of an untrained autoencoder explains about half of the multipliers'
    # variance (a CPU fit of the same network plateaus near 0.45 of the initial loss)
    params, losses = train.fit_mlp(Z, Tt, synth.mlp_weights(), epochs=40, batch=256, lr=3e-3)
    assert losses[-1] < 0.7 * losses[0], losses
    net = hcz.Mlp(ctx, params.cpu().numpy(), scale.cpu().numpy())
    res = {}
    for name, p in (("cold", hcz.params(tau=0.5)), ("warm", hcz.params(tau=0.5, mlp=net))):
        cz2 = hcz.Compressor(plan, model, 8192, p)
        cz2.centroids.copy_(cent)
        c2 = cz2.compress(Fte)
        st = c2.stats()
        out = cz2.decompress(c2, 8192).cpu().numpy()
        g = grid.make_grid()
        F = Fte.cpu().numpy().astype(np.float64)
        assert moments.qoi_rel_error(moments.qoi(F, g), moments.qoi(out, g), g).max() < 1e-10
        res[name] = (st["newton_iters_total"], c2.lam.cpu().numpy(), c2.flags.cpu().numpy())
    assert res["warm"][0] < res["cold"][0], (res["warm"][0], res["cold"][0])
    both = ((res["warm"][2] & 4) == 0) & ((res["cold"][2] & 4) == 0)
    assert np.allclose(res["warm"][1][both], res["cold"][1][both], rtol=1e-6,
                       atol=1e-9 * np.abs(res["cold"][1]).max())
    print(f"[warm-start] Newton updates cold {res['cold'][0]} warm {res['warm'][0]} "
          f"rejected {int(((res['warm'][2] & 8) != 0).sum())}", flush=True)


def test_incremental_training(T):
    """Incremental training (Section IV-D) on a drifting series: a model trained on step 0
    and continued for 2 epochs on step 1 (rows chosen one per mesh node, column-random-
    index style) fits step 1 better than before the update and better than 2 epochs from
    scratch; its first update is the oracle's Adam step from the same weights."""
    hcz, train = T
    say("incremental training")
    ctx = hcz.Context(0)
    plan = hcz.Plan(ctx)
    planes, nodes = 4, 4096
    sets = []
    for t in range(2):
        F = torch.from_numpy(synth.series(t, planes, nodes)).cuda()
        Fs = F.reshape(planes * nodes, -1)[torch.from_numpy(train.colrandind(planes, nodes, seed=t)).cuda()]
        mu, sd = hcz.norm_stats(plan, Fs.reshape(nodes, 39, 39))
        sets.append(((Fs - mu) / sd).contiguous())
    X0, X1 = sets
    W0 = synth.dense_ae_weights()
    tr0 = train.Trainer(train.pack(W0), lr=1e-3)
    tr0.fit(X0, epochs=8, batch=256)

    def loss_of(p, X):
        with torch.no_grad():
            _, xh = train.DenseAE.apply(X, p)
            return train.mse(xh, X).item()

    before = loss_of(tr0.p, X1)
    tri, li = train.incremental(tr0.p, X1, epochs=2, batch=256)
    trs, ls = train.incremental(train.pack(W0), X1, epochs=2, batch=256)
    after, scratch = loss_of(tri.p, X1), loss_of(trs.p, X1)
    assert after < before and after < 0.8 * scratch, (before, after, scratch)
    # parity of the first incremental update against the oracle (FP64 gradient, Adam)
    xb = X1[:256].contiguous()
    tr = train.Trainer(tr0.p, lr=1e-3)
    tr.train_step(xb)
    P0 = train.unpack(tr0.p, 1521)
    P1 = train.unpack(tr.p, 1521)
    W64 = {k: v.astype(np.float64) for k, v in P0.items()}
    cache = oracle.ae.dense_forward_train(xb.cpu().numpy().astype(np.float64), W64)
    g = oracle.ae.dense_backward(cache, W64)
    ref = oracle.ae.adam_step(dict(W64), g, {}, lr=1e-3)
    for k in train.KEYS:
        sure = np.abs(g[k]) > 1e-3 * np.abs(g[k]).max()     # the FP32 gradient has the same sign
        d = np.abs(P1[k].astype(np.float64) - ref[k])[sure]
        # the step is lr g / (|g| + eps): within 0.5 % of lr where the sign is sure
        tol = 5e-6 + 4 * np.finfo(np.float32).eps * np.abs(W64[k][sure])
        assert np.all(d <= tol), (k, (d / tol).max())


def test_conv_model_forward_backward_and_training(T):
    """The convolutional model's FP32 training kernels against the oracle's FP64 forward and
    backward (plus an extra dL/dz), and a few epochs of training lower the loss."""
    hcz, train = T
    say("conv training")
    from oracle import conv as oconv
    rng = np.random.default_rng(90)
    W = synth.conv_ae_weights(4)
    for k in ("c1b", "c2b", "fb", "db", "t1b", "t2b"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    B = 96
    X = inputs(B, 1521, seed=91)
    p = train.pack_conv(W).requires_grad_(True)
    x = torch.from_numpy(X).cuda()
    z, xh = train.ConvAE.apply(x, p)
    dz = torch.from_numpy(rng.standard_normal((B, 16)).astype(np.float32) * 1e-3).cuda()
    loss = train.mse(xh, x)
    (loss + (z * dz).sum()).backward()
    torch.cuda.synchronize()
    cache = oconv.forward_train(X.astype(np.float64), W)
    assert np.allclose(z.detach().cpu().numpy(), cache["z"], rtol=1e-4, atol=1e-4 * np.abs(cache["z"]).max())
    assert np.allclose(xh.detach().cpu().numpy(), cache["xh"], rtol=1e-4, atol=1e-4 * np.abs(cache["xh"]).max())
    dxh = 2 * (cache["xh"] - X.astype(np.float64)) / X.size
    g_or = oconv.backward(cache, W, dxh, dz.cpu().numpy().astype(np.float64))
    g = train.unpack_conv(p.grad)
    for k in hcz.CONV_KEYS:
        scale = np.abs(g_or[k]).max() + 1e-30
        err = np.abs(g[k] - g_or[k]).max() / scale
        assert err < 2e-4, (k, err)
    # training on 2,048 z-scored histograms lowers the loss
    F = synth.histograms(2048, seed=92, dtype=np.float32).reshape(2048, -1)
    mu, sd = oracle.ae.norm_stats(F)
    Xt = torch.from_numpy(((F - mu) / sd).astype(np.float32)).cuda()
    tr = train.Trainer(train.pack_conv(synth.conv_ae_weights()), lr=1e-3, arch="conv")
    losses = tr.fit(Xt, epochs=6, batch=256)
    assert losses[-1] < 0.7 * losses[0], losses


def _bf(a):
    return oracle.ae.bf16(np.asarray(a, np.float32)).astype(np.float64)


def _product_ok(got, A, B, add=None, what=""):
    """got (the kernel's FP32 result) against bf16(A) @ bf16(B) (+ add) in FP64.  The matrix
    cores multiply bfloat16 operands exactly and only the FP32 sums round: at most one
    rounding of 2^-24 of the running sum per term of the K-long sum, so
    |got - exact| <= K 2^-24 (|bf16 A| @ |bf16 B|), plus one rounding of the result."""
    a, b = _bf(A), _bf(B)
    exact = a @ b + (0.0 if add is None else add)
    K = a.shape[1]
    tol = K * 2.0 ** -23 * (np.abs(a) @ np.abs(b)) + 2.0 ** -22 * np.abs(exact) + 1e-30
    err = np.abs(got.astype(np.float64) - exact)
    assert np.all(err <= tol), (what, float((err / tol).max()))
    return exact


def test_bf16_training_products_stage_exact(T):
    """BF16 training form, stage by stage through the C-ABI: every product of the forward
    and backward pass is checked against the oracle's bfloat16-operand product of the
    kernel's own inputs (exact in FP64) within the FP32 summation bound; bias gradients
    against FP64 column sums."""
    hcz, train = T
    N, B, Hd, Ld = 1521, 200, 128, 16
    say("bf16 training products", B)
    C = train.C
    W = weights(N, seed=13)
    X = inputs(B, N, seed=14)
    rng = np.random.default_rng(15)
    dxh = (rng.normal(size=(B, N)) * 1e-3).astype(np.float32)
    dz_in = (rng.normal(size=(B, Ld)) * 1e-2).astype(np.float32)
    p = train.pack(W)
    x = torch.from_numpy(X).cuda()
    nbytes = C.c_size_t()
    train._check(train.LIB.hcz_ae_saved_bytes(N, B, C.byref(nbytes)))
    saved = torch.zeros(nbytes.value // 4, dtype=torch.float32, device="cuda")
    z = torch.empty((B, Ld), dtype=torch.float32, device="cuda")
    xh = torch.empty((B, N), dtype=torch.float32, device="cuda")
    train._check(train.LIB.hcz_ae_forward(N, hcz.COMPUTE_BF16, train._ptr(p), train._ptr(x), B, train._ptr(z),
                                          train._ptr(xh), train._ptr(saved), nbytes.value, None))
    torch.cuda.synchronize()
    s = saved.cpu().numpy()
    h1, h3 = s[:B * Hd].reshape(B, Hd), s[B * Hd:2 * B * Hd].reshape(B, Hd)
    zg, xhg = z.cpu().numpy(), xh.cpu().numpy()
    # h1 = relu(.): compare the pre-activation where it is positive, zero elsewhere
    ex1 = _bf(X) @ _bf(W["W1"].T) + W["b1"]
    tol1 = N * 2.0 ** -23 * (np.abs(_bf(X)) @ np.abs(_bf(W["W1"].T))) + 2.0 ** -22 * np.abs(ex1)
    assert np.all(np.abs(h1 - np.maximum(ex1, 0)) <= tol1)
    _product_ok(zg, h1, W["W2"].T, W["b2"], "z")
    ex3 = _bf(zg) @ _bf(W["W3"].T) + W["b3"]
    tol3 = Ld * 2.0 ** -23 * (np.abs(_bf(zg)) @ np.abs(_bf(W["W3"].T))) + 2.0 ** -22 * np.abs(ex3)
    assert np.all(np.abs(h3 - np.maximum(ex3, 0)) <= tol3)
    _product_ok(xhg, h3, W["W4"].T, W["b4"], "xhat")
    # backward with dL/dxhat = dxh and an extra dL/dz = dz_in
    grad = torch.empty_like(p)
    dx = torch.empty_like(x)
    dxh_d, dz_d = torch.from_numpy(dxh).cuda(), torch.from_numpy(dz_in).cuda()
    train._check(train.LIB.hcz_ae_backward(N, hcz.COMPUTE_BF16, train._ptr(p), train._ptr(x), B, train._ptr(dz_d),
                                           train._ptr(dxh_d), train._ptr(saved), nbytes.value, train._ptr(grad),
                                           train._ptr(dx), None))
    torch.cuda.synchronize()
    s = saved.cpu().numpy()
    d3 = s[2 * B * Hd:3 * B * Hd].reshape(B, Hd)
    d1 = s[3 * B * Hd:4 * B * Hd].reshape(B, Hd)
    dz = s[4 * B * Hd:4 * B * Hd + B * Ld].reshape(B, Ld)
    g = train.unpack(grad, N)
    _product_ok(g["W4"], dxh.T, h3, None, "dW4")
    assert np.allclose(g["b4"], dxh.astype(np.float64).sum(0), rtol=2.0 ** -23, atol=1e-30)
    mask3 = h3 > 0
    ed3 = _bf(dxh) @ _bf(W["W4"])
    td3 = N * 2.0 ** -23 * (np.abs(_bf(dxh)) @ np.abs(_bf(W["W4"])))
    assert np.all(np.abs(d3 - ed3 * mask3) <= td3 + 1e-30)
    _product_ok(g["W3"], d3.T, zg, None, "dW3")
    _product_ok(dz, d3, W["W3"], dz_in, "dz")
    _product_ok(g["W2"], dz.T, h1, None, "dW2")
    assert np.allclose(g["b2"], dz.astype(np.float64).sum(0), rtol=2.0 ** -23, atol=1e-30)
    ed1 = _bf(dz) @ _bf(W["W2"])
    td1 = Ld * 2.0 ** -23 * (np.abs(_bf(dz)) @ np.abs(_bf(W["W2"])))
    assert np.all(np.abs(d1 - ed1 * (h1 > 0)) <= td1 + 1e-30)
    _product_ok(g["W1"], d1.T, X, None, "dW1")
    assert np.allclose(g["b1"], d1.astype(np.float64).sum(0), rtol=2.0 ** -23, atol=1e-30)
    _product_ok(dx.cpu().numpy(), d1, W["W1"], None, "dx")


def test_bf16_training_end_to_end(T):
    """BF16 training against the oracle: the gradients of one step agree with the oracle's
    BF16 form (FP64 sums; its own rounding decisions) to 1e-2 in norm and with the FP64
    gradients to 3e-2, and training with bfloat16 operands follows FP32 training."""
    hcz, train = T
    N, B = 1521, 256
    say("bf16 training end to end")
    W = weights(N, seed=16)
    X = inputs(B, N, seed=17)
    x = torch.from_numpy(X).cuda()
    p = train.pack(W).requires_grad_(True)
    _, xh = train.DenseAE.apply(x, p, hcz.COMPUTE_BF16)
    loss = train.mse(xh, x)
    loss.backward()
    g = train.unpack(p.grad, N)
    c16 = oracle.ae.dense_forward_train(X, W, rnd=oracle.ae.bf16)
    g16 = oracle.ae.dense_backward(c16, W, rnd=oracle.ae.bf16)
    W64 = {k: v.astype(np.float64) for k, v in W.items()}
    g64 = oracle.ae.dense_backward(oracle.ae.dense_forward_train(X.astype(np.float64), W64), W64)
    assert loss.item() == pytest.approx(oracle.ae.mse(c16["xh"], X.astype(np.float64)), rel=1e-4)
    for k in train.KEYS:
        n16 = np.linalg.norm(g[k] - g16[k]) / np.linalg.norm(g16[k])
        n64 = np.linalg.norm(g[k] - g64[k]) / np.linalg.norm(g64[k])
        assert n16 < 1e-2 and n64 < 3e-2, (k, n16, n64)
    say("bf16 training run")
    ctx = hcz.Context(0)
    plan = hcz.Plan(ctx)
    Ftr = torch.from_numpy(synth.histograms(8192, seed=synth.SEED_TRAIN, dtype=np.float32)).cuda()
    mu, sd = hcz.norm_stats(plan, Ftr)
    Xt = ((Ftr.reshape(8192, -1) - mu) / sd).contiguous()
    W0 = synth.dense_ae_weights()
    l32 = train.Trainer(train.pack(W0), lr=1e-3).fit(Xt, epochs=8, batch=512)
    l16 = train.Trainer(train.pack(W0), lr=1e-3, compute="bf16").fit(Xt, epochs=8, batch=512)
    say("losses fp32", l32, "bf16", l16)
    assert l16[-1] < 0.6 * l16[0]
    assert abs(l16[-1] - l32[-1]) < 0.15 * l32[-1], (l16, l32)
    with pytest.raises(ValueError):
        train.Trainer(train.pack(W0), compute="fp16")


def test_conv_bf16_training(T):
    """BF16 training of the convolutional model: one step's gradients (with an extra dL/dz)
    against the oracle's BF16 form (bfloat16 operands of every product, its own rounding
    decisions on FP64 activations) within 2e-2 in norm and against the FP64 gradients
    within 1e-1, the loss against the oracle's BF16 forward, and a short training run in
    BF16 that follows the FP32 run."""
    hcz, train = T
    say("conv bf16 training")
    from oracle import conv as oconv
    rng = np.random.default_rng(93)
    W = synth.conv_ae_weights(6)
    for k in ("c1b", "c2b", "fb", "db", "t1b", "t2b"):
        W[k] = rng.normal(0, 0.05, W[k].shape).astype(np.float32)
    B = 96
    X = inputs(B, 1521, seed=94)
    p = train.pack_conv(W).requires_grad_(True)
    x = torch.from_numpy(X).cuda()
    z, xh = train.ConvAE.apply(x, p, hcz.COMPUTE_BF16)
    dz = torch.from_numpy(rng.standard_normal((B, 16)).astype(np.float32) * 1e-3).cuda()
    loss = train.mse(xh, x)
    (loss + (z * dz).sum()).backward()
    torch.cuda.synchronize()
    X64 = X.astype(np.float64)
    c16 = oconv.forward_train(X64, W, rnd=oracle.ae.bf16)
    assert loss.item() == pytest.approx(float(np.mean((c16["xh"] - X64) ** 2)), rel=1e-3)
    dz64 = dz.cpu().numpy().astype(np.float64)
    g16 = oconv.backward(c16, W, 2 * (c16["xh"] - X64) / X.size, dz64, rnd=oracle.ae.bf16)
    c64 = oconv.forward_train(X64, W)
    g64 = oconv.backward(c64, W, 2 * (c64["xh"] - X64) / X.size, dz64)
    g = train.unpack_conv(p.grad)
    for k in hcz.CONV_KEYS:
        n16 = np.linalg.norm(g[k] - g16[k]) / np.linalg.norm(g16[k])
        n64 = np.linalg.norm(g[k] - g64[k]) / np.linalg.norm(g64[k])
        assert n16 < 2e-2 and n64 < 1e-1, (k, n16, n64)
    F = synth.histograms(2048, seed=95, dtype=np.float32).reshape(2048, -1)
    mu, sd = oracle.ae.norm_stats(F)
    Xt = torch.from_numpy(((F - mu) / sd).astype(np.float32)).cuda()
    W0 = synth.conv_ae_weights()
    l32 = train.Trainer(train.pack_conv(W0), lr=1e-3, arch="conv").fit(Xt, epochs=6, batch=256)
    l16 = train.Trainer(train.pack_conv(W0), lr=1e-3, arch="conv", compute="bf16").fit(Xt, epochs=6, batch=256)
    say("conv losses fp32", l32, "bf16", l16)
    assert l16[-1] < 0.7 * l16[0]
    assert abs(l16[-1] - l32[-1]) < 0.15 * l32[-1], (l16, l32)
