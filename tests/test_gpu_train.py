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
    """Incremental training (Section IV-C) on a drifting series: a model trained on step 0
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
