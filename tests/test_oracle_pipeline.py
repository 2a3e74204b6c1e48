"""Whole-pipeline properties of the oracle (Section III): bound, QoIs, edge cases."""
import numpy as np
import pytest

import oracle
from oracle import coder, grid, moments, pipeline
from paper_2212_10733_amd import synth


def make_model(F, N=1521):
    W = synth.dense_ae_weights(N)
    mu, sd = oracle.ae.norm_stats(F)
    return dict(W=W, mu=mu, sd=sd)


def check_bound_and_qoi(F, out, comp, g, tau):
    F64 = F.astype(np.float64)
    err = np.sqrt(((out - F64) ** 2).sum((1, 2)))
    th = comp["tau_h"]
    raw = (comp["flags"] & pipeline.FLAG_RAW) != 0
    assert np.all(err[~raw] <= th[~raw])
    assert np.all(out[raw] == F64[raw])
    q0 = moments.qoi(F64, g)
    q1 = moments.qoi(out, g)
    assert moments.qoi_rel_error(q0, q1, g).max() < 1e-10


@pytest.mark.parametrize("use_model", [True, False])
@pytest.mark.parametrize("tau", [1e-2, 1e-3])
def test_roundtrip_bound_and_qoi(use_model, tau):
    g = grid.make_grid()
    F = synth.histograms(12, seed=1, dtype=np.float64)
    model = make_model(F) if use_model else None
    comp = pipeline.compress(F, g, model, None, pipeline.Params(tau=tau), fit_codebook=use_model,
                             sample_every=1, bits=3)
    out = pipeline.decompress(comp, g, model, comp["codebook"], 12, np.float64)
    check_bound_and_qoi(F, out, comp, g, tau)
    assert np.array_equal(out, comp["fc"])
    assert int(comp["offsets"][-1]) == len(comp["stream"])


def test_nrmse_mode_and_fp32_input():
    g = grid.make_grid()
    F = synth.histograms(6, seed=2, dtype=np.float32)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3, tau_mode="nrmse"))
    out = pipeline.decompress(comp, g, None, None, 6, np.float32)
    check_bound_and_qoi(F, out, comp, g, 1e-3)
    X = F.reshape(6, -1).astype(np.float64)
    assert np.allclose(comp["tau_h"], 1e-3 * 39 * (X.max(1) - X.min(1)))


def test_edge_cases_go_verbatim():
    g = grid.make_grid()
    F = synth.histograms(5, seed=3, dtype=np.float64)
    F[0, 3, 4] = np.nan              # non-finite input
    F[1] = 0.0                        # empty histogram (n = 0)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    assert comp["flags"][0] == pipeline.FLAG_RAW and comp["flags"][1] == pipeline.FLAG_RAW
    out = pipeline.decompress(comp, g, None, None, 5, np.float64)
    assert np.isnan(out[0, 3, 4]) and np.all(out[1] == 0)
    assert np.all(comp["flags"][2:] == pipeline.FLAG_CODED)


def test_tau_zero_is_lossless():
    g = grid.make_grid()
    F = synth.histograms(3, seed=4, dtype=np.float64)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=0.0))
    assert np.all(comp["flags"] == pipeline.FLAG_RAW)
    out = pipeline.decompress(comp, g, None, None, 3, np.float64)
    assert np.array_equal(out, F)


def test_forced_newton_failure_goes_round2_then_verbatim():
    g = grid.make_grid()
    F = synth.histograms(3, seed=5, dtype=np.float64)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-2, newton_max_iter=0, newton_max_iter2=0))
    assert np.all(comp["flags"] == pipeline.FLAG_RAW | pipeline.FLAG_ROUND2)


def test_uncoded_when_reconstruction_is_good():
    g = grid.make_grid()
    F = synth.histograms(4, seed=6, dtype=np.float64)
    model = make_model(F)
    comp = pipeline.compress(F, g, model, None, pipeline.Params(tau=100.0), fit_codebook=True,
                             sample_every=1, bits=2)
    assert np.all(comp["flags"] == 0) and len(comp["stream"]) == 0
    out = pipeline.decompress(comp, g, model, comp["codebook"], 4, np.float64)
    check_bound_and_qoi(F, out, comp, g, 100.0)


def test_record_layout_in_stream():
    g = grid.make_grid()
    F = synth.histograms(3, seed=7, dtype=np.float64)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    lay = coder.layout(39, 39)
    for h in range(3):
        rec = comp["stream"][int(comp["offsets"][h]):int(comp["offsets"][h + 1])]
        q, Delta, k = coder.unpack(rec, lay)
        assert k == comp["kstar"][h]
        assert Delta == coder.ladder(coder.delta0(comp["tau_h"][h:h + 1], lay), np.array([k]))[0]


def test_warm_start_network_keeps_the_solution():
    from oracle import mlp
    g = grid.make_grid()
    F = synth.histograms(10, seed=8, dtype=np.float64)
    model = make_model(F)
    cold = pipeline.compress(F, g, model, None, pipeline.Params(tau=0.5), fit_codebook=True,
                             sample_every=1, bits=3)
    P = synth.mlp_weights()
    warm = pipeline.compress(F, g, model, None, pipeline.Params(tau=0.5), fit_codebook=True,
                             sample_every=1, bits=3, warm=(P, np.abs(cold["lam"]).max(axis=0)))
    ok = (cold["flags"] & pipeline.FLAG_RAW) == 0
    assert np.allclose(warm["fc"][ok], cold["fc"][ok], rtol=1e-10, atol=1e-13)
    assert warm["stream"] == cold["stream"]


@pytest.mark.parametrize("lambda_fp32,positivity", [(True, True), (False, False), (True, False)])
def test_stage5_variants_roundtrip(lambda_fp32, positivity):
    """FP32 multipliers (the paper's float storage: QoIs to ~1e-8 rather than ~1e-14) and
    the correction without positivity (flag bit 4): the bound holds on every histogram."""
    g = grid.make_grid()
    F = synth.histograms(24, seed=24, dtype=np.float64)
    p = pipeline.Params(tau=1e-3, lambda_fp32=lambda_fp32, positivity=positivity)
    comp = pipeline.compress(F, g, None, None, p)
    assert comp["lam"].dtype == (np.float32 if lambda_fp32 else np.float64)
    raw = (comp["flags"] & pipeline.FLAG_RAW) != 0
    assert np.all(((comp["flags"] & pipeline.FLAG_NOCLIP) != 0) == (~raw & (not positivity)))
    out = pipeline.decompress(comp, g, None, None, 24, np.float64)
    th = pipeline.tau_h(F, p)
    dist = np.sqrt(((out - F) ** 2).reshape(24, -1).sum(1))
    assert np.all(dist[~raw] <= th[~raw])
    err = moments.qoi_rel_error(moments.qoi(F, g), moments.qoi(out, g), g)[~raw].max(axis=1)
    if lambda_fp32:
        assert 1e-11 < np.median(err) < 1e-5
    else:
        assert err.max() < 1e-11
    if not positivity:
        assert (out < 0).any()                     # negative values survive without positivity


def test_bf16_form_roundtrip():
    """The BF16 autoencoder form changes only the reconstruction fhat: the bound and the
    QoIs hold as in the FP64 form, decompression rebuilds the compressor's f_c exactly,
    and the reconstruction stays within a few bfloat16 roundings of the FP64 model's."""
    g = grid.make_grid()
    F = synth.histograms(16, seed=27, dtype=np.float32)
    model = make_model(F.astype(np.float64))
    m16 = dict(model, compute="bf16")
    comp = pipeline.compress(F, g, m16, None, pipeline.Params(tau=1e-3), fit_codebook=True,
                             sample_every=1, bits=3)
    out = pipeline.decompress(comp, g, m16, comp["codebook"], 16, np.float32)
    check_bound_and_qoi(F, out, comp, g, 1e-3)
    assert np.array_equal(out, comp["fc"])
    C = comp["codebook"]
    f16 = pipeline.reconstruct_ae(comp["codes"], C, m16, F.shape)
    f64 = pipeline.reconstruct_ae(comp["codes"], C, model, F.shape)
    scale = np.abs(f64).max()
    assert 1e-6 * scale < np.abs(f16 - f64).max() < 3e-2 * scale


def test_per_histogram_tau_is_the_scalar_form_per_subdomain():
    """Subdomains with their own bounds in one batch: every histogram's record, flags and
    multipliers are those of compressing its subdomain alone with the scalar bound; a
    negative or NaN bound stores the histogram verbatim."""
    g = grid.make_grid(33, 33)
    F = synth.histograms(30, 33, 33, seed=28, dtype=np.float32)
    counts, taus = [7, 0, 11, 4, 8], [1e-2, 5e-3, 1e-4, -1.0, np.nan]
    tau = np.repeat(taus, counts)
    comp = pipeline.compress(F, g, None, None, pipeline.Params(tau=tau))
    start = np.concatenate([[0], np.cumsum(counts)])
    for s, t in enumerate(taus):
        lo, hi = start[s], start[s + 1]
        if hi == lo:
            continue
        if not (t >= 0):
            assert np.all(comp["flags"][lo:hi] == pipeline.FLAG_RAW)
            assert np.array_equal(comp["fc"][lo:hi], F[lo:hi].astype(np.float64))
            continue
        one = pipeline.compress(F[lo:hi], g, None, None, pipeline.Params(tau=t))
        assert np.array_equal(comp["flags"][lo:hi], one["flags"])
        assert np.array_equal(comp["lam"][lo:hi], one["lam"])
        assert comp["stream"][comp["offsets"][lo]:comp["offsets"][hi]] == one["stream"]


def test_conv_model_roundtrip():
    """The convolutional model (BF16 form) in the pipeline: bound, QoIs and exact
    decompression as with the dense model."""
    g = grid.make_grid()
    F = synth.histograms(10, seed=29, dtype=np.float32)
    mu, sd = oracle.ae.norm_stats(F.astype(np.float64))
    model = dict(arch="conv", W=synth.conv_ae_weights(), mu=mu, sd=sd)
    comp = pipeline.compress(F, g, model, None, pipeline.Params(tau=1e-3), fit_codebook=True,
                             sample_every=1, bits=3)
    assert comp["codes"].shape == (10, 16)
    out = pipeline.decompress(comp, g, model, comp["codebook"], 10, np.float32)
    check_bound_and_qoi(F, out, comp, g, 1e-3)
    assert np.array_equal(out, comp["fc"])


def test_multiplier_truncation():
    """Rounding to m mantissa bits is nearest-even (at m = 23 it equals the FP32 conversion
    for normal values); the QoI error of the decompressed data grows like 2^-m while the
    bound still holds."""
    rng = np.random.default_rng(30)
    v = rng.standard_normal(10000) * 10.0 ** rng.integers(-30, 30, 10000)
    assert np.array_equal(pipeline.round_mantissa(v, 23), v.astype(np.float32).astype(np.float64))
    assert np.array_equal(pipeline.round_mantissa(v, 0), v)
    # ties: 1 + 2^-11 at 10 bits goes to the even 1, 1 + 3 * 2^-11 up to 1 + 2^-9
    t = np.array([1 + 2.0 ** -11, 1 + 3 * 2.0 ** -11])
    assert np.array_equal(pipeline.round_mantissa(t, 10), np.array([1.0, 1 + 2.0 ** -9]))
    g = grid.make_grid()
    F = synth.histograms(12, seed=31, dtype=np.float64)
    errs = []
    for bits in (0, 30, 12):
        p = pipeline.Params(tau=1e-3, lambda_bits=bits)
        comp = pipeline.compress(F, g, None, None, p)
        out = pipeline.decompress(comp, g, None, None, 12, np.float64)
        dist = np.sqrt(((out - F) ** 2).reshape(12, -1).sum(1))
        assert np.all(dist <= 1.0001 * pipeline.tau_h(F, p))
        errs.append(moments.qoi_rel_error(moments.qoi(F, g), moments.qoi(out, g), g).max())
    assert errs[0] < 1e-11 and errs[0] < errs[1] < errs[2] < 1e-2


def _records(comp, H):
    off = comp["offsets"].astype(np.int64)
    return [comp["stream"][off[h]:off[h + 1]] for h in range(H)]


def test_user_specified_step():
    """The 'ub' setting (Section IV-F): the coder's step is given, not searched.
    * level 0 keeps the bound: every cell's coder error is at most (L+1) Delta_0 / 2 (each
      level adds at most Delta/2 to a convex combination of coarser errors), so
      ||f - f~|| <= sqrt(N) (L+1) Delta_0 / 2 < tau_h, and the projection only shrinks it;
    * on histograms where the bisection chose k, the step k given by the user gives the
      same record byte for byte;
    * a finer step never gives a shorter record (|rint(d / Delta)| is non-increasing in
      Delta, so is every group's bit width)."""
    g = grid.make_grid()
    H = 16
    F = synth.histograms(H, seed=41, dtype=np.float64)
    lay = coder.layout(g.n_par, g.n_perp)
    ab = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3))
    ub0 = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3, ub_level=0))
    coded = (ab["flags"] & pipeline.FLAG_CODED) != 0
    assert coded.all() and np.array_equal(ub0["flags"] & pipeline.FLAG_CODED, ab["flags"] & pipeline.FLAG_CODED)
    assert np.all(ub0["kstar"][coded] == 0)
    d0 = coder.delta0(ub0["tau_h"], lay)
    cell = np.abs((F - ub0["ft"]).reshape(H, -1)).max(axis=1)
    assert np.all(cell <= (lay.L + 1) * d0 / 2 * (1 + 1e-12))
    out = pipeline.decompress(ub0, g, None, None, H, np.float64)
    check_bound_and_qoi(F, out, ub0, g, 1e-3)
    ra, r0 = _records(ab, H), _records(ub0, H)
    assert all(len(x) >= len(y) for x, y in zip(r0, ra))
    assert sum(map(len, r0)) > sum(map(len, ra))
    for k in np.unique(ab["kstar"][coded]):
        uk = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3, ub_level=int(k)))
        rk = _records(uk, H)
        for h in np.nonzero(coded & (ab["kstar"] == k))[0]:
            assert rk[h] == ra[h]
            assert np.array_equal(uk["lam"][h], ab["lam"][h])
        assert np.all(uk["kstar"][coded] == k)
    # a step far above the search's choice loses the bound on the primary data
    big = pipeline.compress(F, g, None, None, pipeline.Params(tau=1e-3, ub_level=40))
    dist = np.sqrt(((big["ft"] - F) ** 2).reshape(H, -1).sum(1))
    assert np.any(dist > big["tau_h"])


def test_fp64_staged_form():
    """The library's FP64 form stores z and fhat as FP32: the oracle's staged form equals
    torch's float32 rounding of the FP64 model's z and fhat, and the pipeline keeps the
    bound and the QoIs with it."""
    import torch
    g = grid.make_grid()
    F = synth.histograms(10, seed=33, dtype=np.float64)
    model = make_model(F)
    model["mu"] = model["mu"].astype(np.float32).astype(np.float64)
    model["sd"] = model["sd"].astype(np.float32).astype(np.float64)
    staged = dict(model, compute="fp64_staged")
    z64 = pipeline.encode_ae(F, model)
    z32 = pipeline.encode_ae(F, staged)
    assert np.array_equal(z32, torch.from_numpy(z64).float().double().numpy())
    assert not np.array_equal(z32, z64)
    comp = pipeline.compress(F, g, staged, None, pipeline.Params(tau=1e-3), fit_codebook=True, sample_every=1)
    f64 = pipeline.reconstruct_ae(comp["codes"], comp["codebook"], model, F.shape)
    assert np.array_equal(comp["fhat"], torch.from_numpy(f64).float().double().numpy())
    out = pipeline.decompress(comp, g, staged, comp["codebook"], 10, np.float64)
    check_bound_and_qoi(F, out, comp, g, 1e-3)
