"""Throughput of the hybrid compressor's hot path on one MI355X.

Workload (plain method at scale): 1,048,576 synthetic 39x39 FP32 histograms (6.38 GB),
dense FP32 autoencoder 1521-128-16-128-1521 with seeded Xavier weights, 8-bit product
quantizer fitted per batch on every 16th latent vector, per-histogram relative-L2 bound
tau = 1e-3, FP64 residual coder and Newton QoI correction.  One step = one hcz_compress
call (encode, codebook fit, quantize, decode, residual coding, Newton, stream assembly)
with the input already resident in HBM.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the program runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_FP64_VALU_TFLOPS = 78.6


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def residual_flops(N: int, H: int, coded: int, steps_per_coded: float, newton_passes: float) -> float:
    """FP64 operations the residual kernel itself executes, FMA counted as 2, per grid cell:
    13 for the load pass (residual, two squared norms, four moments), per coded histogram
    5 for the decomposition, 12 per bisection step (quantise, interpolate, add, error),
    2 for packing and 10 for the final recomposition with ft = fhat + rhat, and 10 per
    Newton pass (correction, clip, two moment sums, Hessian terms on active cells)."""
    per_cell = 13.0 * H + coded * (5.0 + 12.0 * steps_per_coded + 2.0 + 10.0) + 10.0 * newton_passes
    return per_cell * N


def residual_flops_method(N: int, H: int, coded: int, probes_per_coded: float, passes: float,
                          hessians: float) -> float:
    """FP64 operations of the residual stage as the method's algorithmic count gives them
    (FMA = 2 operations), per grid cell: the four moments, 4 FMA; each Newton pass, 8 FMA
    (correction, clip, gradient sums); each Hessian, 5 masked adds; each coded histogram,
    7 operations per coder step, the steps being the forward decomposition plus one per
    bound evaluation of the ladder search.  passes and hessians are totals over the batch."""
    return N * (8.0 * H + 16.0 * passes + 5.0 * hessians + 7.0 * coded * (1.0 + probes_per_coded))


def search_steps(kstar_hist, start: int | None = 11) -> float:
    """Mean number of bound evaluations of the ladder search for the measured k*
    distribution, counted on a ladder whose feasibility is monotone (k feasible iff k <= k*):
    the exponential search from `start` (the default search; 11 = round(4 log2(L+1)) for
    the 39 x 39 grid, L = 6) followed by bisection, or with start None the bisection over
    the 41-step ladder alone."""
    def steps(k):
        lo, hi, step, n = 0, 41, 1, 0
        phase = 3 if start is None else 0
        while True:
            if phase == 1 and lo + step >= 41:
                phase = 3
            if phase == 2 and hi - step <= 0:
                lo, phase = 0, 3
            if phase == 3 and hi - lo <= 1:
                return n
            t = start if phase == 0 else lo + step if phase == 1 else hi - step if phase == 2 else (lo + hi) >> 1
            ok = t <= k
            n += 1
            if phase == 0:
                lo, hi, phase = (t, hi, 1) if ok else (lo, t, 2)
            elif phase == 1:
                if ok:
                    lo, step = t, step * 2
                else:
                    hi, phase = t, 3
            elif phase == 2:
                if ok:
                    lo, phase = t, 3
                else:
                    hi, step = t, step * 2
            else:
                lo, hi = (t, hi) if ok else (lo, t)
    tot = sum(kstar_hist)
    return sum(c * steps(k) for k, c in enumerate(kstar_hist)) / tot if tot else 0.0


def _sha256(paths) -> str:
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


RESIDUAL_SOURCES = ["paper_2212_10733_amd/csrc/k_wave.hip", "paper_2212_10733_amd/csrc/wave_ops.h",
                    "paper_2212_10733_amd/csrc/hcz_internal.h"]


def residual_traffic(H: int):
    """HBM bytes of one residual launch from the committed counter summary, scaled to H,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "residual_wave_hbm_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    try:
        if vals["kernel source sha256"] != _sha256(RESIDUAL_SOURCES):
            return None
        per_hist = float(vals["calibrated fetch bytes per histogram"]) + float(vals["calibrated write bytes per histogram"])
    except (KeyError, ValueError):
        return None
    return per_hist * H


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_compress_timed(F, W, mu, sd, tau, threads=1):
    """Time the oracle's full compress (encode, codebook fit on every 16th latent, quantize,
    decode, coder, Newton) of the histograms F with `threads` BLAS threads; returns seconds."""
    from threadpoolctl import threadpool_limits

    from oracle import grid, pipeline
    g = grid.make_grid(F.shape[2], F.shape[1])
    model = dict(W=W, mu=np.asarray(mu, np.float64), sd=np.asarray(sd, np.float64))
    with threadpool_limits(limits=threads):
        t0 = time.perf_counter()
        pipeline.compress(F, g, model, None, pipeline.Params(tau=tau), fit_codebook=True, bits=8, sample_every=16)
        return time.perf_counter() - t0


def _oracle_worker(a):
    return _oracle_compress_timed(*a)


def cpu_baseline(F: np.ndarray, W: dict, mu, sd, tau: float, n: int, gpu_check=None, precision=None) -> dict:
    """The FP64 oracle timed on this host's cores on samples of the same workload: every
    sample runs the whole compress.  Headline: all cores, one worker process per core (at
    most 16), each on its own n histograms with one BLAS thread (16 n histograms, 65,536 at
    the default n), at tau; the same at 1e-2 and 1e-4.  Beside it: one thread on n
    histograms, every BLAS thread on n/2 (the oracle's products are the only multithreaded
    part), and the 256-histogram FP64 case.
    gpu_check: (b, q_in, q_out, f_c) of the GPU on the first histograms of the batch
    (moments of f, QoIs of f and of the decompressed f_c), compared here with the oracle's.
    precision: the GPU's per-stage outputs of the precision forms on a sample
    (precision_sample), compared here with the plain FP64 model."""
    import multiprocessing as mp

    from oracle import grid, moments
    from paper_2212_10733_amd import synth
    cores = os.cpu_count() or 1
    workers = max(1, min(16, cores))
    res = {"cpu_model": _cpu_model(), "host_cores": cores, "kind": "oracle", "unit": "histograms/s"}
    dt = _oracle_compress_timed(F[:n], W, mu, sd, tau, 1)
    res["one_thread"] = {"value": n / dt, "histograms": n, "tau": tau, "seconds": dt}
    m = max(256, n // 2)
    d = _oracle_compress_timed(F[:m], W, mu, sd, tau, cores)
    res["blas_all_threads"] = {"value": m / d, "histograms": m, "threads": cores, "seconds": d}
    F1 = synth.histograms(256, seed=synth.SEED_PLAIN_SMALL, dtype=np.float64)
    from oracle import ae
    m1, s1 = ae.norm_stats(F1)                  # the 256-histogram case's own z-score statistics
    d = _oracle_compress_timed(F1, W, m1, s1, tau, 1)
    res["c1_256_fp64_one_thread"] = {"value": 256 / d, "seconds": d}
    per = min(n, len(F) // workers)
    chunks = [np.ascontiguousarray(F[k * per:(k + 1) * per]) for k in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        pool.map(_oracle_worker, [(c[:64], W, mu, sd, tau, 1) for c in chunks])      # import and warm up
        for t in dict.fromkeys((tau, 1e-2, 1e-4)):
            t0 = time.perf_counter()
            secs = pool.map(_oracle_worker, [(c, W, mu, sd, t, 1) for c in chunks])
            wall = time.perf_counter() - t0
            r = {"value": workers * per / wall, "workers": workers, "histograms": workers * per, "tau": t,
                 "wall_seconds": wall, "max_worker_seconds": max(secs)}
            if t == tau:
                res["value"] = r["value"]
                res["cores"] = workers
                res["all_cores"] = r
            else:
                res[f"all_cores_tau_{t:g}"] = r
            log(f"cpu baseline: all cores at tau {t:g}: {r['value']:.0f} histograms/s")
    res["sample"] = (f"histograms of the same 2^20 batch, full compress (encode, codebook fit on every 16th, "
                     f"quantize, decode, coder, Newton), NumPy FP64: headline {workers} worker processes x {per} "
                     f"histograms at tau {tau:g}, one BLAS thread each; all_cores_tau_* the same at the other "
                     f"bounds; see one_thread, blas_all_threads, c1_256_fp64_one_thread")
    if gpu_check is not None:
        b_gpu, q_in, q_out, fc = gpu_check
        k = len(b_gpu)
        g = grid.make_grid()
        bo = moments.moments(F[:k], g)
        qo_in = moments.qoi(F[:k], g)
        qo_out = moments.qoi(fc, g)
        res["gpu_crosscheck"] = {
            "histograms": k,
            "moments_max_rel_diff": float((np.abs(b_gpu - bo) / np.abs(bo).max(axis=0)).max()),
            "qoi_in_max_rel_err": float(moments.qoi_rel_error(qo_in, q_in, g).max()),
            "qoi_out_vs_oracle_input_max_rel_err": float(moments.qoi_rel_error(qo_in, qo_out, g).max()),
        }
    if precision is not None:
        log("cpu baseline: per-stage error of the precision forms against the FP64 model")
        res["precision_vs_fp64"] = precision_errors(F, precision, tau)
    return res


def precision_sample(hcz, plan, x, forms, tau: float, K: int) -> dict:
    """GPU outputs of each precision form on the first K histograms of the batch, for the
    per-stage comparison with the plain FP64 model (codebook fitted on all K latents, the
    sample's own z-score statistics): z, codebook, codes, fhat, flags, multipliers, record
    sizes and the decompressed FP64 histograms.  forms: name -> (weights, arch, compute)."""
    import torch
    xs = x[:K].contiguous()
    mu, sd = hcz.norm_stats(plan, xs)
    mu, sd = mu.cpu().numpy(), sd.cpu().numpy()
    out = {}
    for name, (W, arch, compute) in forms.items():
        model = hcz.Model(plan, W, mu, sd, compute=compute, arch=arch)
        cz = hcz.Compressor(plan, model, K, hcz.params(tau=tau, fit_codebook=True, sample_every=1))
        comp = cz.compress(xs)
        z = hcz.encode(model, xs)
        fh = hcz.decode(model, comp.codes, cz.centroids)
        fc = cz.decompress(comp, K)
        torch.cuda.synchronize()
        off = comp.offsets.cpu().numpy().astype(np.int64)
        out[name] = {"arch": arch, "compute": compute, "W": W, "z": z.cpu().numpy().astype(np.float64),
                     "centroids": cz.centroids.cpu().numpy().astype(np.float64),
                     "codes": comp.codes.cpu().numpy(), "fhat": fh.cpu().numpy().astype(np.float64).reshape(K, -1),
                     "flags": comp.flags.cpu().numpy(), "lam": comp.lam.cpu().numpy().astype(np.float64),
                     "stream_bytes": int(off[-1]), "fc": fc.cpu().numpy().reshape(K, -1)}
        del model, cz, comp, fc
    return out


def precision_errors(F: np.ndarray, gpu: dict, tau: float) -> dict:
    """Per-stage error of each precision form's GPU outputs against the plain FP64 model run
    by the oracle on the same K histograms (its own z-score statistics and codebook fit):
    latent, codebook, code flip rate, fhat, coded fraction p, stream bytes, multipliers,
    QoI error of each side's output and the final histograms."""
    from oracle import ae, grid, moments, pipeline
    K = next(iter(gpu.values()))["z"].shape[0]
    F64 = np.asarray(F[:K], np.float64)
    g = grid.make_grid()
    mu, sd = ae.norm_stats(F64)
    q_in = moments.qoi(F64, g)
    th = pipeline.tau_h(F64, pipeline.Params(tau=tau))
    res = {"histograms": K, "tau": tau}
    for name, d in gpu.items():
        model = dict(arch=d["arch"], W=d["W"], mu=mu, sd=sd, compute="fp64")
        t0 = time.perf_counter()
        o = pipeline.compress(F64, g, model, None, pipeline.Params(tau=tau), fit_codebook=True, bits=8, sample_every=1)
        t_or = time.perf_counter() - t0
        zo, fo = o["z"], o["fhat"].reshape(K, -1)
        ok = ((d["flags"] & 4) == 0) & ((o["flags"] & 4) == 0)
        lam_o = np.asarray(o["lam"], np.float64)
        lam_rel = np.linalg.norm(d["lam"] - lam_o, axis=1) / np.maximum(np.linalg.norm(lam_o, axis=1), 1e-300)
        fc_o = o["fc"].reshape(K, -1)
        qg = moments.qoi(d["fc"].reshape(F64.shape), g)
        qo = moments.qoi(fc_o.reshape(F64.shape), g)
        span = d["centroids"].max() - d["centroids"].min()
        res[name] = {
            "oracle_seconds": t_or,
            "z_rel_l2": float(np.linalg.norm(d["z"] - zo) / np.linalg.norm(zo)),
            "z_max_abs_over_range": float(np.abs(d["z"] - zo).max() / (zo.max() - zo.min())),
            "codebook_max_abs_over_range": float(np.abs(d["centroids"] - o["codebook"]).max() / span),
            "code_flip_rate": float((d["codes"] != o["codes"]).mean()),
            "fhat_rel_l2": float(np.linalg.norm(d["fhat"] - fo) / np.linalg.norm(fo)),
            "fhat_diff_over_tau_h_median": float(np.median(np.linalg.norm(d["fhat"] - fo, axis=1) / th)),
            "coded_frac": {"gpu": float((d["flags"] & 1).mean()), "oracle": float((o["flags"] & 1).mean())},
            "stream_bytes": {"gpu": d["stream_bytes"], "oracle": len(o["stream"])},
            "lambda_rel_diff_median": float(np.median(lam_rel[ok])), "lambda_rel_diff_max": float(lam_rel[ok].max()),
            "qoi_rel_err_max": {"gpu": float(moments.qoi_rel_error(q_in[ok], qg[ok], g).max()),
                                "oracle": float(moments.qoi_rel_error(q_in[ok], qo[ok], g).max())},
            "final_diff_over_tau_h_max": float((np.linalg.norm(d["fc"] - fc_o, axis=1)[ok] / th[ok]).max()),
            "err_over_tau_h_max": {"gpu": float((np.linalg.norm(d["fc"] - F64.reshape(K, -1), axis=1)[ok] / th[ok]).max()),
                                   "oracle": float((np.linalg.norm(fc_o - F64.reshape(K, -1), axis=1)[ok]
                                                    / th[ok]).max())},
        }
    return res


def time_compress(cz, x, steps):
    import torch
    cz.compress(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        comp = cz.compress(x)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, comp


def _qoi_refs(hcz, plan, x):
    import torch
    _, q0, n0 = hcz.qoi(plan, x)
    den = torch.stack([q0[:, 0].abs(), torch.maximum(q0[:, 1].abs(), q0[:, 3].abs().sqrt()),
                       q0[:, 2].abs(), q0[:, 3].abs()], 1)
    return q0, n0, den


def newton_stats(s: dict, H: int) -> dict:
    """Newton updates per histogram from the device histogram of update counts (its last
    bin holds 63 or more): mean over the non-verbatim histograms, median, 99th percentile
    and maximum."""
    hist = np.asarray(s["newton_iter_hist"], np.int64)
    cum = np.cumsum(hist)
    n = int(cum[-1])

    def pct(q):
        return int(np.searchsorted(cum, q * n)) if n else 0
    return {"mean": s["newton_iters_total"] / max(1, H - s["n_raw"]), "p50": pct(0.5), "p99": pct(0.99),
            "max": int(s["newton_max_iters"])}


DENSE_PARAMS, CONV_PARAMS = 395265, 248785


def _plain_run(hcz, plan, model, x, hp, tau, refs, steps=3, model_floats=DENSE_PARAMS) -> dict:
    """Time one configuration of the full pipeline and report throughput, coded fraction p,
    stream size, compression ratio (codes, FP64 multipliers, flags, residual stream, model,
    codebook and header against the FP32 input), Newton updates, QoI error and the bound on
    the batch."""
    H = x.shape[0]
    q0, n0, den = refs
    cz = hcz.Compressor(plan, model, H, hp)
    dt, comp = time_compress(cz, x, steps)
    s = comp.stats()
    o = cz.decompress(comp, H)
    _, q1, _ = hcz.qoi(plan, o)
    ok = (comp.flags & 4) == 0
    stored = H * 16 + H * 32 + H + s["stream_bytes"] + model_floats * 4 + 16 * 256 * 4 + 44
    over = (o - x.double()).reshape(H, -1).norm(dim=1)[ok] / (tau * n0[ok])
    r = {"value": H / dt, "ms_per_step": dt * 1e3, "coded_frac": s["n_coded"] / H, "raw": s["n_raw"],
         "stream_bytes": s["stream_bytes"], "compression_ratio": H * plan.N * 4 / stored,
         "newton_mean_updates": s["newton_iters_total"] / max(1, H - s["n_raw"]),
         "newton": newton_stats(s, H), "round2": s["n_round2"],
         "warm_rejected": int(((comp.flags & 8) != 0).sum().item()),
         "max_qoi_rel_err": ((q1 - q0).abs() / den)[ok].max().item(),
         "max_err_over_tau_h": over.max().item(), "over_bound": int((over > 1).sum().item())}
    alg = H * (4 * plan.N + 16 + 32 + 1 + 8) + s["stream_bytes"]
    r["hbm_alg_bytes"] = alg
    r["hbm_frac"] = alg / dt / 1e9 / PEAK_HBM_GBS
    del cz, comp, o
    return r


def tau_sweep(hcz, plan, model, x, args) -> dict:
    """The plain form at the other bounds of the workload's tau set."""
    refs = _qoi_refs(hcz, plan, x)
    out = {}
    for tau in (1e-2, 1e-4):
        log(f"tau sweep: {tau}")
        out[f"{tau:g}"] = _plain_run(hcz, plan, model, x, hcz.params(tau=tau, fit_codebook=True, sample_every=16),
                                     tau, refs)
    return out


def ub_form(hcz, plan, model, x, args) -> dict:
    """The plain form with the coder's step given instead of searched (the paper's 'ub'
    against its 'ab'): level 0 is the step whose a-priori estimate keeps the bound, level 4
    doubles it and lets the bound go."""
    refs = _qoi_refs(hcz, plan, x)
    out = {}
    for level in (0, 4):
        log(f"ub form: level {level}")
        out[f"level_{level}"] = _plain_run(hcz, plan, model, x,
                                           hcz.params(tau=args.tau, fit_codebook=True, sample_every=16,
                                                      ub_level=level), args.tau, refs)
    return out


def container_form(hcz, plan, x, W, args, n=131072) -> dict:
    """The output container of the plain form on the first n histograms: bytes without
    entropy coding, with the byte-wise rANS of codes, residual bytes and multipliers, and
    with the residual records coded by their integers, and the host pack / unpack rates
    (single thread) including the device-to-host copies."""
    import torch
    xs = x[:n]
    mu, sd = hcz.norm_stats(plan, xs)
    mu, sd = mu.cpu().numpy(), sd.cpu().numpy()
    model = hcz.Model(plan, W, mu, sd)
    cz = hcz.Compressor(plan, model, n, hcz.params(tau=args.tau, fit_codebook=True, sample_every=16))
    comp = cz.compress(xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    arrays = dict(flags=comp.flags.cpu().numpy(), res_offset=comp.offsets.cpu().numpy().astype(np.uint64),
                  res_bytes=np.frombuffer(comp.stream_bytes(), np.uint8), lam=comp.lam.cpu().numpy(),
                  codes=comp.codes.cpu().numpy(), centroids=cz.centroids.cpu().numpy(),
                  weights=hcz.pack_dense_weights(W), norm_mean=mu, norm_std=sd, arch="dense")
    t_copy = time.perf_counter() - t0
    res = {"histograms": n, "input_bytes": n * plan.N * 4, "d2h_seconds": t_copy}
    for ent, name in ((0, "plain"), (1, "rans"), (2, "rans_integers")):
        t0 = time.perf_counter()
        buf = hcz.container_pack(plan.n_par, plan.n_perp, entropy=ent, **arrays)
        t1 = time.perf_counter()
        d = hcz.container_unpack(buf)
        t2 = time.perf_counter()
        assert np.array_equal(d["res_bytes"], arrays["res_bytes"])
        res[name] = {"bytes": len(buf), "ratio": n * plan.N * 4 / len(buf),
                                           "pack_MBps": len(buf) / (t1 - t0) / 1e6,
                                           "unpack_MBps": len(buf) / (t2 - t1) / 1e6}
    del cz, comp, model
    return res


def stage5_form(hcz, plan, x, args) -> dict:
    """The coder-only pipeline at tau with each reading of the correction: FP32 multipliers,
    no positivity (orthogonal projection onto A x = b), and the KL correction (kept where it
    keeps the bound, the L2 projection elsewhere; it runs on the workgroup kernel)."""
    import torch
    H = x.shape[0]
    _, q0, n0 = hcz.qoi(plan, x)
    den = torch.stack([q0[:, 0].abs(), torch.maximum(q0[:, 1].abs(), q0[:, 3].abs().sqrt()),
                       q0[:, 2].abs(), q0[:, 3].abs()], 1)
    out = {}
    for name, kw in (("fp32_lambda", dict(lambda_fp32=True)), ("no_positivity", dict(no_positivity=True)),
                     ("kl", dict(kl=True))):
        cz = hcz.Compressor(plan, None, H, hcz.params(tau=args.tau, **kw))
        dt, comp = time_compress(cz, x, 2)
        s = comp.stats()
        o = cz.decompress(comp, H)
        _, q1, _ = hcz.qoi(plan, o)
        ok = (comp.flags & 4) == 0
        out[name] = {"value": H / dt, "ms_per_step": dt * 1e3, "raw": s["n_raw"],
                     "kl_kept": int(((comp.flags & 32) != 0).sum().item()),
                     "negative_cells": int((o < 0).sum().item()),
                     "max_qoi_rel_err": ((q1 - q0).abs() / den)[ok].max().item(),
                     "max_err_over_tau_h": ((o - x.double()).reshape(H, -1).norm(dim=1)[ok]
                                            / (args.tau * n0[ok])).max().item()}
        del cz, comp, o
    return out


def bf16_form(hcz, plan, ctx, x, W, args, arch="dense", stats=None) -> dict:
    """The plain workload with the autoencoder's large products on bfloat16 operands
    (FP32 accumulation), dense or convolutional: throughput, per-stage times with the
    encoder's and decoder's HBM rates (4N bytes read, resp. written, per histogram) and
    matrix-core rates, p, stream size, QoI error, bound."""
    import torch
    H, N = x.shape[0], plan.N
    if stats is None:
        mu, sd = hcz.norm_stats(plan, x)
        mu, sd = mu.cpu().numpy(), sd.cpu().numpy()
    else:
        mu, sd = stats
    model = hcz.Model(plan, W, mu, sd, compute="bf16", arch=arch)
    cz = hcz.Compressor(plan, model, H, hcz.params(tau=args.tau, fit_codebook=True, sample_every=16))
    cz.compress(x)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    dt, comp = time_compress(cz, x, 3)
    prof = ctx.profile_read()
    ctx.profile(False)
    stage_ms = {k: v[0] / v[1] for k, v in prof.items() if v[1]}
    s = comp.stats()
    o = cz.decompress(comp, H)
    _, q0, n0 = hcz.qoi(plan, x)
    _, q1, _ = hcz.qoi(plan, o)
    ok = (comp.flags & 4) == 0
    den = torch.stack([q0[:, 0].abs(), torch.maximum(q0[:, 1].abs(), q0[:, 3].abs().sqrt()),
                       q0[:, 2].abs(), q0[:, 3].abs()], 1)
    res = {"value": H / dt, "ms_per_step": dt * 1e3, "coded_frac": s["n_coded"] / H,
           "stream_bytes": s["stream_bytes"], "raw": s["n_raw"],
           "newton_mean_updates": s["newton_iters_total"] / max(1, H - s["n_raw"]),
           "max_qoi_rel_err": ((q1 - q0).abs() / den)[ok].max().item(),
           "max_err_over_tau_h": ((o - x.double()).reshape(H, -1).norm(dim=1)[ok] / (args.tau * n0[ok])).max().item(),
           "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()}}
    # FLOP per histogram and direction: dense 2 (N 128 + 128 16); convolutional 2 (conv1
    # 115,200 + conv2 1,843,200 + dense 102,400) multiply-adds, the decoder mirroring it
    flop = 2 * (N * 128 + 128 * 16) if arch == "dense" else 2 * (115200 + 1843200 + 102400)
    for k in ("encode", "decode"):
        if k in stage_ms:
            res[f"{k}_hbm_GBps"] = H * 4 * N / (stage_ms[k] / 1e3) / 1e9
            res[f"{k}_TFLOPs"] = H * flop / (stage_ms[k] / 1e3) / 1e12
    del cz, comp, o, model
    return res


def batched_form(hcz, ctx, args, n_sub=512, reps=3) -> dict:
    """512 subdomains of uneven sizes (log-uniform 500..20,000 histograms) on 33x33, 39x39,
    49x49 and 65x65 grids, each with its own tau (log-uniform 1e-4..1e-2): one plan, dense
    FP32 model (Xavier, z-score statistics of its grid's histograms) and per-batch codebook
    per grid size.  Reported: whole-batch throughput (histograms/s and input GB/s), and the
    per-subdomain completion time (residual stage done) p50/p99 of the last repetition."""
    import torch

    from paper_2212_10733_amd import batched, synth
    layout = synth.subdomains(n_sub)
    plans, models, inputs = {}, {}, {}
    nbytes = 0
    for n in synth.BATCH_GRIDS:
        Hn = sum(c for g, c, _ in layout if g == n)
        plans[n] = hcz.Plan(ctx, n, n)
        F = synth.histograms(Hn, n, n, seed=synth.SEED_BATCHED * 100 + n, dtype=np.float32)
        x = torch.from_numpy(F).cuda()
        del F
        mu, sd = hcz.norm_stats(plans[n], x)
        models[n] = hcz.Model(plans[n], synth.dense_ae_weights(n * n), mu.cpu().numpy(), sd.cpu().numpy())
        inputs[n] = x
        nbytes += x.numel() * 4
    Htot = sum(c for _, c, _ in layout)
    sb = batched.SubdomainBatch(plans, models, layout)
    sb.compress(inputs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        comps = sb.compress(inputs)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    done = sb.completion_seconds()
    st = {k: c.stats() for k, c in comps.items()}
    # the launch variant of every grid's residual stage from the autotuner, then the whole
    # batch as one HIP graph
    import tempfile
    from paper_2212_10733_amd import autotune
    tuned = {}
    with tempfile.TemporaryDirectory() as td:
        for n in synth.BATCH_GRIDS:
            v = autotune.apply(plans[n], os.path.join(td, "tune.json"), H=16384, reps=3)
            tuned[f"{n}x{n}"] = {"variant": v, "ms_per_16384": autotune.load(os.path.join(td, "tune.json"))[
                autotune.plan_key(plans[n])]["ms"]}
    sb.compress(inputs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.compress(inputs)
    torch.cuda.synchronize()
    dt_tuned = (time.perf_counter() - t0) / reps
    sb.capture(inputs)
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.replay()
    torch.cuda.synchronize()
    dt_graph = (time.perf_counter() - t0) / reps
    small = _small_batch_graph(hcz, batched, synth, plans, torch)
    for n in synth.BATCH_GRIDS:
        plans[n].set_variant("auto")
    # every grid's residual stage in one persistent launch (hcz_compress_batch)
    group_H = {k: g["H"] for k, g in sb.groups.items()}
    del sb
    torch.cuda.empty_cache()
    sbp = batched.SubdomainBatch(plans, models, layout, persistent=True)
    sbp.compress(inputs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sbp.compress(inputs)
    torch.cuda.synchronize()
    dt_p = (time.perf_counter() - t0) / reps
    done_p = sbp.completion_seconds()
    del sbp
    live = np.array([c > 0 for _, c, _ in layout])
    res = {"subdomains": n_sub, "histograms": Htot, "input_bytes": nbytes, "value": Htot / dt,
           "tuned": {"variants": tuned, "value": Htot / dt_tuned, "ms_per_step": dt_tuned * 1e3},
           "graph": {"value": Htot / dt_graph, "ms_per_step": dt_graph * 1e3}, "small_batch": small,
           "persistent": {"value": Htot / dt_p, "ms_per_step": dt_p * 1e3,
                          "completion_ms_p50": float(np.percentile(done_p[live], 50) * 1e3),
                          "completion_ms_p99": float(np.percentile(done_p[live], 99) * 1e3)},
           "unit": "histograms/s", "ms_per_step": dt * 1e3, "input_GBps": nbytes / dt / 1e9,
           "completion_ms_p50": float(np.percentile(done[live], 50) * 1e3),
           "completion_ms_p99": float(np.percentile(done[live], 99) * 1e3),
           "completion_ms_max": float(done[live].max() * 1e3),
           "per_grid": {f"{k}x{k}": {"histograms": group_H[k], "coded_frac": s["n_coded"] / max(1, s["n_hist"]),
                                     "raw": s["n_raw"], "stream_bytes": s["stream_bytes"],
                                     "newton_mean_updates": s["newton_iters_total"] / max(1, s["n_hist"] - s["n_raw"])}
                        for k, s in st.items()}}
    del comps, inputs, models, plans
    torch.cuda.empty_cache()
    return res


def _small_batch_graph(hcz, batched, synth, plans, torch, n_sub=64, reps=20) -> dict:
    """64 small subdomains (50..500 histograms, coder-only) on the four grids: eager calls
    against replays of the captured batch, where launch overhead is a visible share."""
    layout = synth.subdomains(n_sub, seed=55, count_range=(50, 500))
    inputs = {}
    for n in synth.BATCH_GRIDS:
        Hn = sum(c for g, c, _ in layout if g == n)
        inputs[n] = torch.from_numpy(synth.histograms(max(Hn, 1), n, n, seed=56 + n, dtype=np.float32)[:Hn]).cuda()
    sb = batched.SubdomainBatch(plans, {}, layout)
    Htot = sum(c for _, c, _ in layout)
    sb.compress(inputs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.compress(inputs)
    torch.cuda.synchronize()
    dt_e = (time.perf_counter() - t0) / reps
    sb.capture(inputs)
    t0 = time.perf_counter()
    for _ in range(reps):
        sb.replay()
    torch.cuda.synchronize()
    dt_g = (time.perf_counter() - t0) / reps
    del sb
    sbp = batched.SubdomainBatch(plans, {}, layout, persistent=True)
    sbp.compress(inputs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        sbp.compress(inputs)
    torch.cuda.synchronize()
    dt_pe = (time.perf_counter() - t0) / reps
    sbp.capture(inputs)
    t0 = time.perf_counter()
    for _ in range(reps):
        sbp.replay()
    torch.cuda.synchronize()
    dt_pg = (time.perf_counter() - t0) / reps
    return {"subdomains": n_sub, "histograms": Htot, "eager_ms": dt_e * 1e3, "graph_ms": dt_g * 1e3,
            "eager_value": Htot / dt_e, "graph_value": Htot / dt_g,
            "persistent_eager_ms": dt_pe * 1e3, "persistent_graph_ms": dt_pg * 1e3,
            "persistent_graph_value": Htot / dt_pg}


def incremental_form(hcz, plan, H, W, args, steps=4, planes=8) -> dict:
    """Incremental training (Section IV-D) on a drifting synthetic series: at every step a
    batch of planes x nodes = H / 4 histograms (262,144 at H = 2^20), training rows chosen
    one per node (column-random-index: 32,768), the model of step 0 trained from
    scratch for --epochs, every later step either continued from the previous model for 2
    epochs or trained from scratch for --epochs.  Reported per step: training seconds, final
    training loss, and the residual stream of the whole batch at tau (what the model buys)."""
    import torch

    from paper_2212_10733_amd import synth, train
    nodes = max(1024, H // 4 // planes)
    n = planes * nodes
    res = []
    prev = None
    for t in range(steps):
        F = torch.from_numpy(synth.series(t, planes, nodes)).cuda()
        sel = torch.from_numpy(train.colrandind(planes, nodes, seed=t)).cuda()
        Fs = F.reshape(n, -1)[sel]
        mu, sd = hcz.norm_stats(plan, Fs.reshape(nodes, plan.n_perp, plan.n_par))
        X = hcz.column_normalize(Fs, mu, sd)
        row = {"step": t}
        runs = [("scratch", train.pack(W), args.epochs)]
        if prev is not None:
            runs.insert(0, ("incremental", prev, 2))
        for name, p0, ep in runs:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            tr, losses = train.incremental(p0, X, epochs=ep, batch=1024)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            model = hcz.Model(plan, train.unpack(tr.p, plan.N), mu.cpu().numpy(), sd.cpu().numpy())
            cz = hcz.Compressor(plan, model, n, hcz.params(tau=args.tau, fit_codebook=True, sample_every=16))
            s = cz.compress(F).stats()
            row[name] = {"epochs": ep, "train_seconds": dt, "final_loss": losses[-1],
                         "coded_frac": s["n_coded"] / n, "stream_bytes_per_hist": s["stream_bytes"] / n}
            if name == "incremental" or prev is None:
                nxt = tr.p
            del cz, model
        prev = nxt
        res.append(row)
        del F, Fs, X
    return {"planes": planes, "nodes": nodes, "train_rows_per_step": nodes, "steps": res}


def other_forms(hcz, plan, ctx, x, F, W, args, plain_value, plain_stats) -> dict:
    """The same batch and tau through (a) the coder-only pipeline and (b) the learned form:
    the autoencoder trained by the library's kernels on held-apart synthetic histograms,
    plus the warm-start network trained on the training batch's multipliers."""
    import torch

    from paper_2212_10733_amd import synth, train
    H = x.shape[0]
    out = {}
    if "coder" in args.forms:
        log("form: coder-only")
        cz = hcz.Compressor(plan, None, H, hcz.params(tau=args.tau))
        dt, comp = time_compress(cz, x, 3)
        s = comp.stats()
        out["coder_only"] = {"value": H / dt, "ms_per_step": dt * 1e3, "coded_frac": s["n_coded"] / H,
                             "stream_bytes": s["stream_bytes"], "newton_mean_updates": s["newton_iters_total"] / H}
        del cz, comp
    if "bf16" in args.forms:
        log("form: BF16 autoencoder")
        out["bf16_ae"] = bf16_form(hcz, plan, ctx, x, W, args)
    if "stage5" in args.forms:
        log("form: Stage-5 variants")
        out["stage5_variants"] = stage5_form(hcz, plan, x, args)
    if "container" in args.forms:
        log("form: container")
        out["container"] = container_form(hcz, plan, x, W, args)
    if "conv" in args.forms:
        log("form: convolutional autoencoder (BF16)")
        out["conv_ae"] = bf16_form(hcz, plan, ctx, x, synth.conv_ae_weights(), args, arch="conv")
    if "batched" in args.forms:
        log("form: batched uneven subdomains")
        out["batched"] = batched_form(hcz, ctx, args)
    if "incremental" in args.forms:
        log("form: incremental training series")
        out["incremental"] = incremental_form(hcz, plan, x.shape[0], W, args)
    if "learned" in args.forms:
        log(f"form: learned, dense (train {args.epochs} epochs on {args.train_hist})")
        out["learned"] = learned_form(hcz, plan, ctx, W, args, "dense", plain_value, plain_stats, H)
    if "learned_conv" in args.forms:
        log(f"form: learned, convolutional BF16 (train {args.epochs} epochs on {args.train_hist})")
        out["learned_conv"] = learned_form(hcz, plan, ctx, synth.conv_ae_weights(), args, "conv", plain_value,
                                           plain_stats, H)
    return out


def learned_form(hcz, plan, ctx, W0, args, arch, plain_value, plain_stats, H) -> dict:
    """The learned form: the autoencoder trained by the library's kernels (Adam, lr 1e-3,
    batch 1024, `args.epochs` epochs on `args.train_hist` histograms of the training seed,
    z-scored with their own statistics), a warm-start network per bound trained on the
    training batch's cold multipliers, then evaluated on a held-out batch of H histograms
    (held-out seed) at tau = 1e-3 and 1e-2: the untrained model (its z-score statistics from
    the held-out batch), the trained model with cold, analytic-linear and network starts
    (Newton updates mean / p50 / p99 / max, QoI error, bound, p, ratio).  Dense: trained in
    FP32 and, separately, in BF16 (evaluated in the BF16 form, the form whose HBM rate is
    reported as hbm_frac_bf16_dense_trained).  Convolutional: trained in BF16, evaluated in its BF16 form."""
    import torch

    from paper_2212_10733_amd import synth, train
    conv = arch == "conv"
    mf = CONV_PARAMS if conv else DENSE_PARAMS
    Ftr = torch.from_numpy(synth.histograms(args.train_hist, seed=synth.SEED_TRAIN, dtype=np.float32)).cuda()
    mu, sd = hcz.norm_stats(plan, Ftr)
    mu_np, sd_np = mu.cpu().numpy(), sd.cpu().numpy()
    X = hcz.column_normalize(Ftr, mu, sd)
    res = {"train_histograms": args.train_hist, "epochs": args.epochs, "batch": 1024}
    pack = train.pack_conv if conv else train.pack
    unpack = train.unpack_conv if conv else (lambda p: train.unpack(p, plan.N))
    runs = [("bf16", "bf16")] if conv else [("fp32", "fp32"), ("bf16", "bf16")]
    trained = {}
    for name, compute in runs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        tr = train.Trainer(pack(W0), lr=1e-3, arch=arch, compute=compute)
        losses = tr.fit(X, epochs=args.epochs, batch=1024, log=log if conv else None)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        res[f"train_{name}"] = {"seconds": dt, "samples_per_s": args.train_hist * args.epochs / dt,
                                "loss_first_last": [losses[0], losses[-1]]}
        log(f"  trained {arch} in {name}: {dt:.1f} s, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
        trained[name] = unpack(tr.p)
        del tr
    del X
    # the evaluation model: conv and the BF16-trained dense model in their BF16 forms
    main = "bf16" if conv else "fp32"
    model = hcz.Model(plan, trained[main], mu_np, sd_np, compute="bf16" if conv else "fp32", arch=arch)
    model16 = None if conv else hcz.Model(plan, trained["bf16"], mu_np, sd_np, compute="bf16")
    xe = torch.from_numpy(synth.histograms(H, seed=synth.SEED_HELDOUT, dtype=np.float32)).cuda()
    refs = _qoi_refs(hcz, plan, xe)
    mue, sde = hcz.norm_stats(plan, xe)
    untrained = hcz.Model(plan, W0, mue.cpu().numpy(), sde.cpu().numpy(), compute="bf16" if conv else "fp32",
                          arch=arch)
    for tau in (1e-3, 1e-2):
        log(f"  held-out evaluation at tau {tau:g}")
        # warm-start network: targets are the training batch's cold multipliers at this tau
        czt = hcz.Compressor(plan, model, args.train_hist, hcz.params(tau=tau, fit_codebook=True, sample_every=16))
        ct = czt.compress(Ftr)
        ok = (ct.flags & 4) == 0
        lam_ok = ct.lam[ok]
        _, scale = hcz.column_stats(lam_ok)
        Z = hcz.dequantize(ct.codes, czt.centroids)[ok]
        T = hcz.column_normalize(lam_ok, None, scale)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pm, mlosses = train.fit_mlp(Z, T, synth.mlp_weights(), epochs=10, batch=512, lr=3e-3)
        torch.cuda.synchronize()
        t_mlp = time.perf_counter() - t0
        net = hcz.Mlp(ctx, pm.cpu().numpy(), scale.double().cpu().numpy())
        del czt, ct, Z, T
        r = {"mlp_train_seconds": t_mlp, "mlp_loss_first_last": [mlosses[0], mlosses[-1]]}
        base = dict(tau=tau, fit_codebook=True, sample_every=16)
        r["untrained"] = _plain_run(hcz, plan, untrained, xe, hcz.params(**base), tau, refs, 2, mf)
        for start, kw in (("cold", {}), ("analytic", {"analytic_start": True}), ("mlp", {"mlp": net})):
            r[f"trained_{start}"] = _plain_run(hcz, plan, model, xe, hcz.params(**base, **kw), tau, refs, 2, mf)
        if model16 is not None:
            r["bf16_trained_bf16_form"] = _plain_run(hcz, plan, model16, xe, hcz.params(**base), tau, refs, 3, mf)
        res[f"tau_{tau:g}"] = r
        del net
    res["benchmark_batch_untrained_plain"] = {"value": plain_value, "coded_frac": plain_stats["n_coded"] / H,
                                              "stream_bytes": plain_stats["stream_bytes"]}
    del xe, Ftr, model, model16, untrained
    return res


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--H", type=int, default=1 << 20)
    ap.add_argument("--tau", type=float, default=1e-3)
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="histograms per oracle worker (16 workers at most) and of the one-thread run")
    ap.add_argument("--precision-sample", type=int, default=2048,
                    help="histograms of the per-stage comparison of the precision forms with the FP64 model")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the coder-only and learned forms")
    ap.add_argument("--forms", default="tau,ub,coder,stage5,container,bf16,conv,batched,incremental,learned,learned_conv",
                    help="comma list of the other forms to run: tau (sweep), coder (coder-only), "
                         "stage5 (FP32 multipliers, no positivity, KL correction), container (packed "
                         "output with and without rANS), ub (the coder step given, not searched), "
                         "bf16 (BF16 autoencoder), conv (convolutional BF16 autoencoder), "
                         "batched (uneven subdomains on four grids), "
                         "incremental (training series), learned (dense model trained in FP32 and "
                         "BF16, held-out evaluation with cold / analytic / network starts), learned_conv (the "
                         "convolutional model trained in BF16, the same evaluation)")
    ap.add_argument("--train-hist", type=int, default=262144)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the "
                         "reference kernel for scaling HBM byte counters), then exit")
    args = ap.parse_args()
    args.forms = {f.strip() for f in args.forms.split(",") if f.strip()}
    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        a = torch.empty(n, dtype=torch.uint8, device="cuda").fill_(1)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {n} bytes three times")
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on exactly one GPU: the per-histogram path needs no communication, "
              "and this program does not run on several GPUs.", file=sys.stderr)
        return 2

    import torch

    from paper_2212_10733_amd import hcz, synth

    H = args.H
    log(f"generating {H} histograms")
    t0 = time.perf_counter()
    F = synth.histograms(H, seed=synth.SEED_PLAIN_LARGE, dtype=np.float32)
    W = synth.dense_ae_weights()
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    x = torch.from_numpy(F).cuda()
    ctx = hcz.Context(0)
    plan = hcz.Plan(ctx)
    # model preparation (outside the hot path): z-score statistics of the batch
    mu, sd = hcz.norm_stats(plan, x)
    mu, sd = mu.cpu().numpy(), sd.cpu().numpy()
    model = hcz.Model(plan, W, mu, sd)
    p = hcz.params(tau=args.tau, fit_codebook=True, sample_every=16)
    cz = hcz.Compressor(plan, model, H, p, bits=8)
    torch.cuda.synchronize()
    log("warmup")
    for _ in range(args.warmup):
        cz.compress(x)
    torch.cuda.synchronize()
    ctx.profile(True)
    ctx.profile_read()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        comp = cz.compress(x)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile(False)
    st = comp.stats()
    ms_step = dt / args.steps * 1e3
    value = H / (dt / args.steps)
    log(f"{ms_step:.3f} ms/step, {value:.4g} hist/s")

    # per-stage live timing (HIP events on the compress stream)
    stage_ms = {k: (v[0] / v[1] if v[1] else 0.0) for k, v in prof.items() if v[1]}
    N = plan.N
    coded = st["n_coded"]
    steps_coded = search_steps(st["kstar_hist"])
    passes = st["newton_iters_total"] + (H - st["n_raw"])
    ae_flops = 2.0 * H * N * 128 + 2.0 * H * 128 * 16
    method_flops = residual_flops_method(N, H, coded, steps_coded, passes, st["newton_iters_total"])
    cands = {
        "encode": ("mfma", ae_flops / 1e12, PEAK_FP32_MFMA_TFLOPS, "TFLOP/s"),
        "decode": ("mfma", ae_flops / 1e12, PEAK_FP32_MFMA_TFLOPS, "TFLOP/s"),
        "residual": ("alu", method_flops / 1e12, PEAK_FP64_VALU_TFLOPS, "TFLOP/s"),
    }
    dom = max(cands, key=lambda k: stage_ms.get(k, 0.0))
    bound, work, peak, unit = cands[dom]
    achieved = work / (stage_ms[dom] / 1e3)
    roofline = {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": residual_traffic(H) if dom == "residual" else None}
    stream_bytes = st["stream_bytes"]
    alg_bytes = H * (4 * N + 16 + 32 + 1 + 8) + stream_bytes
    kernel_flops = residual_flops(N, H, coded, steps_coded, passes)
    extra = {
        "stage_ms": {k: round(v, 4) for k, v in stage_ms.items()},
        "stage_roofline": {k: {"bound": c[0], "achieved": c[1] / (stage_ms[k] / 1e3), "peak": c[2],
                               "frac": c[1] / (stage_ms[k] / 1e3) / c[2]} for k, c in cands.items() if k in stage_ms},
        "residual_flop_counts": {
            "method_count_per_cell": method_flops / (H * N), "kernel_count_per_cell": kernel_flops / (H * N),
            "kernel_count_frac": kernel_flops / (stage_ms["residual"] / 1e3) / 1e12 / PEAK_FP64_VALU_TFLOPS,
            "search_probes_per_coded": steps_coded, "newton_passes": passes,
            "hbm_alg_bytes": H * (4 * N + 16 + 32 + 1 + 8) + stream_bytes,
            "hbm_frac_of_alg_bytes": (H * (4 * N + 16 + 32 + 1 + 8) + stream_bytes)
                                     / (stage_ms["residual"] / 1e3) / 1e9 / PEAK_HBM_GBS},
        "hbm_whole_step": {"alg_bytes": alg_bytes, "GB/s": alg_bytes / (dt / args.steps) / 1e9,
                           "frac": alg_bytes / (dt / args.steps) / 1e9 / PEAK_HBM_GBS},
        "coded_frac": coded / H, "raw": st["n_raw"], "round2": st["n_round2"],
        "newton_mean_updates": st["newton_iters_total"] / max(1, H - st["n_raw"]),
        "newton_max_updates": st["newton_max_iters"],
        "stream_bytes": stream_bytes,
        "compression_ratio": (H * N * 4) / (H * 16 + H * 32 + H + stream_bytes + 395265 * 4 + 16 * 256 * 4 + 44),
    }
    # QoI restoration and the bound, checked on the whole batch after the timed region
    out = cz.decompress(comp, H, in_dtype=torch.float32, out_dtype=torch.float64)
    _, q0, n0 = hcz.qoi(plan, x)
    _, q1, _ = hcz.qoi(plan, out)
    den = torch.stack([q0[:, 0].abs(), torch.maximum(q0[:, 1].abs(), q0[:, 3].abs().sqrt()),
                       q0[:, 2].abs(), q0[:, 3].abs()], 1)
    flags = comp.flags
    ok = (flags & 4) == 0
    qerr = ((q1 - q0).abs() / den)[ok].max().item()
    dist = (out - x.double()).reshape(H, -1).norm(dim=1)
    bound_ratio = (dist[ok] / (args.tau * n0[ok])).max().item()
    extra["max_qoi_rel_err"] = qerr
    extra["max_err_over_tau_h"] = bound_ratio
    # Eq. 7 applied to each QoI over the batch: u = the QoI of the inputs, f = of the output
    rng_q = (q0[ok].max(0).values - q0[ok].min(0).values)
    nr = ((q1[ok] - q0[ok]) ** 2).mean(0).sqrt() / rng_q
    extra["qoi_nrmse"] = {k: nr[i].item() for i, k in enumerate(("n", "u_par", "T_perp", "T_par"))}
    extra["pd_nrmse"] = ((dist[ok] ** 2).sum() / (int(ok.sum().item()) * N)).sqrt().item() / (x.max() - x.min()).item()
    valid = bool(qerr <= 1e-10 and bound_ratio <= 1.0)
    extra["valid"] = valid
    if not valid:
        log(f"INVALID: max QoI relative error {qerr:.3e} (limit 1e-10) or max ||f-f_c||/tau_h {bound_ratio:.4f} > 1")
    kchk = min(4096, H)
    bchk, qin_chk, _ = hcz.qoi(plan, x[:kchk])
    _, qout_chk, _ = hcz.qoi(plan, out[:kchk])
    gpu_check = (bchk.cpu().numpy(), qin_chk.cpu().numpy(), qout_chk.cpu().numpy(), out[:kchk].cpu().numpy())
    # decompression (dequantize + decode + residual records + correction) on its own, into
    # the same FP64 output: reads codes, multipliers, flags, offsets and records, writes 8N
    ctx.profile(True)
    ctx.profile_read()
    reps = 3
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        cz.decompress_into(comp, H, out, in_dtype=torch.float32)
    e1.record()
    e1.synchronize()
    dms = e0.elapsed_time(e1) / reps
    dprof = ctx.profile_read()
    ctx.profile(False)
    dbytes = H * (16 + 32 + 1 + 8 + 8 * N) + stream_bytes
    extra["decompress"] = {"value": H / (dms / 1e3), "unit": "histograms/s", "ms": dms,
                           "stage_ms": {k: round(v[0] / v[1], 4) for k, v in dprof.items() if v[1]},
                           "alg_bytes": dbytes, "GB/s": dbytes / (dms / 1e3) / 1e9,
                           "hbm_frac": dbytes / (dms / 1e3) / 1e9 / PEAK_HBM_GBS}
    del out

    log("measured ceilings")
    extra["ceilings"] = hcz.ceilings()
    forms = {}
    if not args.no_forms:
        if "tau" in args.forms:
            forms["tau_sweep"] = tau_sweep(hcz, plan, model, x, args)
        if "ub" in args.forms:
            forms["ub"] = ub_form(hcz, plan, model, x, args)
        forms.update(other_forms(hcz, plan, ctx, x, F, W, args, value, st))

    cpu = None
    if not args.no_cpu:
        log(f"precision forms on {args.precision_sample} histograms")
        prec = precision_sample(hcz, plan, x, {"fp32_dense": (W, "dense", "fp32"), "bf16_dense": (W, "dense", "bf16"),
                                               "bf16_conv": (synth.conv_ae_weights(), "conv", "bf16")},
                                args.tau, args.precision_sample)
        log(f"cpu baseline on {args.cpu_sample} histograms per worker")
        cpu = cpu_baseline(F, W, mu, sd, args.tau, args.cpu_sample, gpu_check, prec)

    lf = forms.get("learned", {}).get(f"tau_{args.tau:g}", {}).get("bf16_trained_bf16_form")
    if lf:
        # the HBM rate of the BF16-trained dense model in its BF16 form,
        # on the held-out batch, algorithmic bytes (f read once, outputs, stream) per step
        extra["hbm_frac_bf16_dense_trained"] = {"value": lf["value"], "hbm_frac": lf["hbm_frac"],
                                                "GB/s": lf["hbm_frac"] * PEAK_HBM_GBS}
    line = {
        "metric": "histograms/s (compress+QoI-correct)", "value": value, "unit": "histograms/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {"workload": "plain method at scale: 1048576 x 39x39 FP32 histograms, dense FP32 AE "
                               "1521-128-16 (Xavier), 8-bit PQ fitted per batch, tau=1e-3 rel-L2, FP64 coder + Newton",
                   "H": H, "grid": "39x39", "tau": args.tau, "tau_mode": "rel_l2", "pq_bits": 8,
                   "sample_every": 16},
        "roofline": roofline, "cpu_baseline": cpu, **extra, "forms": forms,
    }
    print(json.dumps(line), flush=True)
    return 0 if valid else 3


if __name__ == "__main__":
    sys.exit(main())
