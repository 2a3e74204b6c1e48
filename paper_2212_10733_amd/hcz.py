"""ctypes binding of libhcz (C ABI in include/hcz.h), with torch tensors for device memory.

Every function here marshals arguments and calls the library; all compute runs in the
HIP kernels.  Import fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhcz.so")

F32, F64 = 0, 1
ARCH_DENSE, ARCH_CONV = 1, 2
CONV_KEYS = ("c1w", "c1b", "c2w", "c2b", "fw", "fb", "dw", "db", "t1w", "t1b", "t2w", "t2b")
COMPUTE_FP32, COMPUTE_BF16, COMPUTE_FP64 = 0, 1, 2
_COMPUTE = {"fp32": COMPUTE_FP32, "bf16": COMPUTE_BF16, "fp64": COMPUTE_FP64}
TAU_REL_L2, TAU_NRMSE = 0, 1
FALLBACK_BACKTRACK, FALLBACK_PAPER = 0, 1
FLAG_CODED, FLAG_ROUND2, FLAG_RAW, FLAG_WARM_REJECTED, FLAG_NOCLIP, FLAG_KL = 1, 2, 4, 8, 16, 32
WARM_COLD, WARM_MLP, WARM_ANALYTIC = 0, 1, 2
BOUND_AB, BOUND_UB = 0, 1
SEARCH_GUIDED, SEARCH_BISECT = 0, 1
HIDDEN, LATENT = 128, 16

STATUS = {0: "HCZ_OK", -1: "HCZ_EINVAL", -2: "HCZ_ENOMEM", -3: "HCZ_EHIP",
          -4: "HCZ_EUNSUPPORTED", -5: "HCZ_ECAPACITY", -6: "HCZ_EWORKSPACE"}


class HczError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Grid(C.Structure):
    _fields_ = [("n_par", C.c_int32), ("n_perp", C.c_int32), ("vpar_lo", C.c_double),
                ("vpar_hi", C.c_double), ("vperp_lo", C.c_double), ("vperp_hi", C.c_double),
                ("mass", C.c_double), ("vol", C.POINTER(C.c_double))]


class ModelDesc(C.Structure):
    _fields_ = [("arch", C.c_int32), ("latent", C.c_int32), ("hidden", C.c_int32),
                ("weights", C.POINTER(C.c_float)), ("norm_mean", C.POINTER(C.c_float)),
                ("norm_std", C.POINTER(C.c_float)), ("compute", C.c_int32)]


class ContainerInfo(C.Structure):
    _fields_ = [("H", C.c_int64), ("n_par", C.c_int32), ("n_perp", C.c_int32), ("arch", C.c_int32),
                ("compute", C.c_int32), ("latent", C.c_int32), ("bits", C.c_int32), ("lambda_fp32", C.c_int32),
                ("entropy", C.c_int32), ("n_weights", C.c_int64), ("res_bytes", C.c_uint64),
                ("total_bytes", C.c_uint64)]


class ContainerIn(C.Structure):
    _fields_ = [("info", ContainerInfo), ("weights", C.c_void_p), ("norm_mean", C.c_void_p),
                ("norm_std", C.c_void_p), ("codes", C.c_void_p), ("centroids", C.c_void_p), ("flags", C.c_void_p),
                ("res_offset", C.c_void_p), ("res_bytes", C.c_void_p), ("lambda_", C.c_void_p)]


class ContainerOut(C.Structure):
    _fields_ = [("weights", C.c_void_p), ("norm_mean", C.c_void_p), ("norm_std", C.c_void_p),
                ("codes", C.c_void_p), ("centroids", C.c_void_p), ("flags", C.c_void_p),
                ("res_offset", C.c_void_p), ("res_bytes", C.c_void_p), ("lambda_", C.c_void_p)]


class Codebook(C.Structure):
    _fields_ = [("bits", C.c_int32), ("centroids", C.c_void_p)]


class Params(C.Structure):
    _fields_ = [("tau", C.c_double), ("tau_mode", C.c_int32), ("newton_s", C.c_double),
                ("newton_max_iter", C.c_int32), ("newton_max_iter2", C.c_int32),
                ("fallback", C.c_int32), ("fit_codebook", C.c_int32), ("sample_every", C.c_int32),
                ("warm_start", C.c_int32), ("mlp", C.c_void_p), ("lambda_fp32", C.c_int32),
                ("no_positivity", C.c_int32), ("tau_hist", C.c_void_p), ("kl", C.c_int32),
                ("lambda_bits", C.c_int32), ("bound_mode", C.c_int32), ("ub_level", C.c_int32),
                ("search", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_hist", C.c_uint64), ("n_coded", C.c_uint64), ("n_round2", C.c_uint64),
                ("n_raw", C.c_uint64), ("stream_bytes", C.c_uint64), ("overflow", C.c_uint64),
                ("newton_max_iters", C.c_uint64), ("newton_iters_total", C.c_uint64),
                ("newton_iter_hist", C.c_uint64 * 64), ("kstar_hist", C.c_uint64 * 48)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_[:8]}
        d["newton_iter_hist"] = list(self.newton_iter_hist)
        d["kstar_hist"] = list(self.kstar_hist)
        return d


class CompressedC(C.Structure):
    _fields_ = [("codes", C.c_void_p), ("lambda_", C.c_void_p), ("flags", C.c_void_p),
                ("res_offset", C.c_void_p), ("res_bytes", C.c_void_p),
                ("res_capacity", C.c_uint64), ("stats", C.c_void_p), ("lambda_fp32", C.c_int32),
                ("t_done", C.c_void_p)]


class BatchSegmentC(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("model", C.c_void_p), ("codebook", C.POINTER(Codebook)),
                ("params", C.POINTER(Params)), ("hist", C.c_void_p), ("dtype", C.c_int32), ("H", C.c_int64),
                ("hist_stride", C.c_int64), ("row_stride", C.c_int64), ("out", C.POINTER(CompressedC)),
                ("ws", C.c_void_p), ("ws_bytes", C.c_size_t)]


BATCH_MAX_SEGMENTS = 4
BATCH_WORKSPACE_BYTES = 256


def _load() -> C.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2212_10733_amd.build` "
                          "(there is no CPU fallback)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    sig = {
        "hcz_create": [C.c_int, C.POINTER(vp)],
        "hcz_plan_create": [vp, C.POINTER(Grid), C.POINTER(vp)],
        "hcz_model_load": [vp, C.POINTER(ModelDesc), C.POINTER(vp)],
        "hcz_qoi": [vp, vp, i32, i64, i64, i64, vp, vp, vp, vp],
        "hcz_encode": [vp, vp, i32, i64, i64, i64, vp, vp],
        "hcz_codebook_fit_workspace": [i64, i32, i64, C.POINTER(sz)],
        "hcz_codebook_fit": [vp, i64, i32, i64, C.POINTER(Codebook), vp, sz, vp],
        "hcz_quantize": [vp, i64, i32, C.POINTER(Codebook), vp, vp],
        "hcz_decode": [vp, vp, C.POINTER(Codebook), i64, vp, vp],
        "hcz_residual": [vp, C.POINTER(Params), vp, i32, i64, i64, i64, vp, vp, C.POINTER(CompressedC), vp, sz, vp],
        "hcz_mlp_load": [vp, vp, vp, C.POINTER(vp)],
        "hcz_mlp_param_count": [C.POINTER(i64)],
        "hcz_mlp_saved_bytes": [i64, C.POINTER(sz)],
        "hcz_mlp_forward": [vp, vp, i64, vp, vp, sz, vp],
        "hcz_mlp_backward": [vp, vp, i64, vp, vp, sz, vp, vp],
        "hcz_dequantize": [vp, i64, i32, C.POINTER(Codebook), vp, vp],
        "hcz_mlp_predict": [vp, vp, C.POINTER(Codebook), i64, vp, vp],
        "hcz_compress_workspace": [vp, vp, i64, C.POINTER(Params), C.POINTER(sz)],
        "hcz_decompress_workspace": [vp, vp, i64, C.POINTER(sz)],
        "hcz_compress": [vp, vp, C.POINTER(Codebook), C.POINTER(Params), vp, i32, i64, i64, i64,
                         C.POINTER(CompressedC), vp, sz, vp],
        "hcz_compress_static": [vp, vp, C.POINTER(Codebook), C.POINTER(Params), vp, i32, i64, i64, i64,
                                C.POINTER(CompressedC), vp],
        "hcz_compress_batch": [C.POINTER(BatchSegmentC), i32, vp, sz, vp],
        "hcz_decompress": [vp, vp, C.POINTER(Codebook), C.POINTER(CompressedC), i32, i64, vp, i32, vp, sz, vp],
        "hcz_stats_read": [vp, C.POINTER(Stats), vp],
        "hcz_ae_param_count": [i32, C.POINTER(i64)],
        "hcz_ae_saved_bytes": [i32, i64, C.POINTER(sz)],
        "hcz_ae_forward": [i32, i32, vp, vp, i64, vp, vp, vp, sz, vp],
        "hcz_ae_backward": [i32, i32, vp, vp, i64, vp, vp, vp, sz, vp, vp, vp],
        "hcz_mse_workspace": [C.POINTER(sz)],
        "hcz_mse": [vp, vp, i64, vp, vp, vp, sz, vp],
        "hcz_adam_step": [vp, vp, vp, vp, i64, C.c_double, C.c_double, C.c_double, C.c_double, i64, vp],
        "hcz_norm_stats_workspace": [vp, i64, C.POINTER(sz)],
        "hcz_norm_stats": [vp, vp, i32, i64, i64, i64, vp, vp, vp, sz, vp],
        "hcz_column_stats_workspace": [i64, i64, C.POINTER(sz)],
        "hcz_column_stats": [vp, i32, i64, i64, i64, vp, vp, vp, sz, vp],
        "hcz_column_normalize": [vp, i32, i64, i64, i64, vp, vp, vp, vp],
        "hcz_plan_path": [vp, C.POINTER(i32)],
        "hcz_plan_variants": [vp, C.POINTER(i32), C.POINTER(i32)],
        "hcz_probe_sink_bytes": [C.POINTER(sz)],
        "hcz_probe_copy": [vp, vp, sz, vp],
        "hcz_probe_compute": [i32, i64, vp, C.POINTER(C.c_double), vp],
        "hcz_plan_set_variant": [vp, i32],
        "hcz_profile_enable": [vp, C.c_int],
        "hcz_profile_read": [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
        "hcz_segment_tau": [vp, vp, i32, i64, vp, vp],
        "hcz_segment_max": [vp, i32, i64, vp, vp, vp],
        "hcz_timestamp": [vp, vp],
        "hcz_wall_clock_hz": [C.c_int, C.POINTER(C.c_double)],
        "hcz_conv_ae_param_count": [C.POINTER(i64)],
        "hcz_conv_ae_saved_bytes": [i64, C.POINTER(sz)],
        "hcz_conv_ae_forward": [i32, vp, vp, i64, vp, vp, vp, sz, vp],
        "hcz_conv_ae_backward": [i32, vp, vp, i64, vp, vp, vp, sz, vp, vp],
        "hcz_container_bound": [C.POINTER(ContainerIn), C.POINTER(sz)],
        "hcz_container_pack": [C.POINTER(ContainerIn), vp, sz, C.POINTER(sz)],
        "hcz_container_read_info": [vp, sz, C.POINTER(ContainerInfo)],
        "hcz_container_unpack": [vp, sz, C.POINTER(ContainerOut)],
        "hcz_rans_bound": [sz, C.POINTER(sz)],
        "hcz_rans_encode": [vp, sz, vp, sz, C.POINTER(sz)],
        "hcz_rans_decode": [vp, sz, vp, sz],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    for name in ("hcz_destroy", "hcz_plan_destroy", "hcz_model_free", "hcz_mlp_free"):
        getattr(lib, name).argtypes = [vp]
        getattr(lib, name).restype = None
    lib.hcz_last_error.restype = C.c_char_p
    lib.hcz_version.restype = C.c_char_p
    return lib


LIB = _load()

# Every symbol the C header declares (checked by the CPU tests).
EXPORTS = ["hcz_create", "hcz_destroy", "hcz_last_error", "hcz_version", "hcz_plan_create",
           "hcz_plan_destroy", "hcz_plan_path", "hcz_plan_variants", "hcz_plan_set_variant", "hcz_probe_sink_bytes", "hcz_probe_copy", "hcz_probe_compute", "hcz_model_load", "hcz_model_free", "hcz_qoi", "hcz_encode",
           "hcz_codebook_fit_workspace", "hcz_codebook_fit", "hcz_quantize", "hcz_decode",
           "hcz_residual", "hcz_compress_workspace", "hcz_decompress_workspace", "hcz_compress",
           "hcz_decompress", "hcz_stats_read", "hcz_profile_enable", "hcz_profile_read",
           "hcz_ae_param_count", "hcz_ae_saved_bytes", "hcz_ae_forward", "hcz_ae_backward",
           "hcz_mse_workspace", "hcz_mse", "hcz_adam_step", "hcz_norm_stats_workspace", "hcz_norm_stats",
           "hcz_mlp_load", "hcz_mlp_free", "hcz_mlp_param_count", "hcz_mlp_saved_bytes", "hcz_mlp_forward",
           "hcz_mlp_backward", "hcz_dequantize", "hcz_mlp_predict", "hcz_segment_tau", "hcz_segment_max",
           "hcz_timestamp", "hcz_wall_clock_hz", "hcz_container_bound", "hcz_container_pack",
           "hcz_container_read_info", "hcz_container_unpack", "hcz_rans_bound", "hcz_rans_encode",
           "hcz_rans_decode", "hcz_conv_ae_param_count", "hcz_conv_ae_saved_bytes", "hcz_conv_ae_forward",
           "hcz_conv_ae_backward", "hcz_column_stats_workspace", "hcz_column_stats", "hcz_column_normalize",
           "hcz_compress_static", "hcz_compress_batch"]

STAGES = ["encode", "codebook", "quantize", "decode", "residual", "scan", "compact", "stats", "decompress",
          "warmstart"]


def _check(status: int) -> None:
    if status != 0:
        raise HczError(status, LIB.hcz_last_error().decode())


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return F32
    if t.dtype == torch.float64:
        return F64
    raise TypeError(f"histograms must be float32 or float64, not {t.dtype}")


def _strides(hist: torch.Tensor):
    if hist.dim() != 3:
        raise ValueError("hist must be (H, n_perp, n_par)")
    if hist.numel() == 0:                 # an empty batch has no layout of its own
        return hist.shape[0], hist.shape[1] * hist.shape[2], hist.shape[2]
    if hist.stride(2) != 1:
        raise ValueError("the v_par axis must be contiguous")
    return hist.shape[0], hist.stride(0), hist.stride(1)


class Context:
    def __init__(self, device: int = 0):
        h = C.c_void_p()
        _check(LIB.hcz_create(device, C.byref(h)))
        self.h = h
        self.device = device

    def profile(self, enable: bool = True) -> None:
        _check(LIB.hcz_profile_enable(self.h, int(enable)))

    def profile_read(self) -> dict:
        """{stage: (total ms, calls)} since the last read (waits for the recorded events)."""
        ms = (C.c_double * len(STAGES))()
        calls = (C.c_int64 * len(STAGES))()
        _check(LIB.hcz_profile_read(self.h, ms, calls))
        return {s: (ms[i], calls[i]) for i, s in enumerate(STAGES)}

    def __del__(self):
        if getattr(self, "h", None) and LIB is not None:   # LIB is None during interpreter shutdown
            LIB.hcz_destroy(self.h)
            self.h = None


class Plan:
    """Device tables of one velocity grid."""

    def __init__(self, ctx: Context, n_par=39, n_perp=39, vpar=(-4.0, 4.0), vperp=(0.0, 4.0),
                 mass=1.0, vol: np.ndarray | None = None):
        self.ctx = ctx
        self.n_par, self.n_perp = n_par, n_perp
        self.N = n_par * n_perp
        self._vol = None if vol is None else np.ascontiguousarray(vol, np.float64).reshape(-1)
        g = Grid(n_par, n_perp, vpar[0], vpar[1], vperp[0], vperp[1], mass,
                 None if self._vol is None else self._vol.ctypes.data_as(C.POINTER(C.c_double)))
        h = C.c_void_p()
        _check(LIB.hcz_plan_create(ctx.h, C.byref(g), C.byref(h)))
        self.h = h
        self.variant = "auto"

    PATHS = {0: "block", 1: "wave", 2: "wave_fixed", 3: "team2", 4: "team4"}

    @property
    def path(self) -> str:
        """Kernel family serving this grid: 'block', 'wave', 'wave_fixed', 'team2' or 'team4'."""
        v = C.c_int32()
        _check(LIB.hcz_plan_path(self.h, C.byref(v)))
        return self.PATHS[v.value]

    VARIANTS = ("auto", "wave_fixed", "wave", "block_256x6", "block_512x5", "block_512x9", "team2", "team4")

    def variants(self) -> list:
        """Launch variants of the residual stage valid for this grid (names of VARIANTS)."""
        buf = (C.c_int32 * 8)()
        n = C.c_int32()
        _check(LIB.hcz_plan_variants(self.h, buf, C.byref(n)))
        return [self.VARIANTS[buf[i]] for i in range(n.value)]

    def set_variant(self, name: str) -> None:
        """Make a variant (a name of VARIANTS) this plan's residual launch for later calls."""
        _check(LIB.hcz_plan_set_variant(self.h, self.VARIANTS.index(name)))
        self.variant = name

    def __del__(self):
        if getattr(self, "h", None) and LIB is not None:   # LIB is None during interpreter shutdown
            LIB.hcz_plan_destroy(self.h)
            self.h = None


DENSE_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3", "W4", "b4")


def pack_dense_weights(W: dict) -> np.ndarray:
    return np.concatenate([np.ascontiguousarray(W[k], np.float32).ravel() for k in DENSE_KEYS])


def unpack_dense_weights(blob: np.ndarray, N: int) -> dict:
    shapes = dict(W1=(HIDDEN, N), b1=(HIDDEN,), W2=(LATENT, HIDDEN), b2=(LATENT,), W3=(HIDDEN, LATENT),
                  b3=(HIDDEN,), W4=(N, HIDDEN), b4=(N,))
    out, o = {}, 0
    for k in DENSE_KEYS:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(blob[o:o + n], np.float32).reshape(shapes[k])
        o += n
    if o != blob.size:
        raise ValueError("weight blob size does not match the dense model of this grid")
    return out


class Model:
    """A dense autoencoder copied to the device for one plan."""

    def __init__(self, plan: Plan, W: dict, mu: np.ndarray, sd: np.ndarray, compute: str = "fp32",
                 arch: str = "dense"):
        """arch "dense" (W1..b4) or "conv" (the convolutional model of 39 x 39 grids, keys
        CONV_KEYS, compute "bf16" only); compute "fp32", "bf16" or "fp64" (dense: every
        layer in FP64, z and fhat stored as FP32)."""
        if compute not in ("fp32", "bf16", "fp64"):
            raise ValueError(f"compute must be 'fp32', 'bf16' or 'fp64', not {compute!r}")
        if arch not in ("dense", "conv"):
            raise ValueError(f"arch must be 'dense' or 'conv', not {arch!r}")
        self.plan = plan
        self.compute = compute
        self.arch = arch
        if arch == "conv":
            blob = np.concatenate([np.ascontiguousarray(W[k], np.float32).ravel() for k in CONV_KEYS])
        else:
            blob = pack_dense_weights(W)
        mu = np.ascontiguousarray(mu, np.float32)
        sd = np.ascontiguousarray(sd, np.float32)
        fp = C.POINTER(C.c_float)
        d = ModelDesc(ARCH_CONV if arch == "conv" else ARCH_DENSE, LATENT, HIDDEN, blob.ctypes.data_as(fp),
                      mu.ctypes.data_as(fp),
                      sd.ctypes.data_as(fp), _COMPUTE[compute])
        h = C.c_void_p()
        _check(LIB.hcz_model_load(plan.h, C.byref(d), C.byref(h)))
        self.h = h
        self.latent = LATENT

    def __del__(self):
        if getattr(self, "h", None) and LIB is not None:   # LIB is None during interpreter shutdown
            LIB.hcz_model_free(self.h)
            self.h = None


def params(tau=1e-3, tau_mode=TAU_REL_L2, newton_s=1.0, newton_max_iter=50, newton_max_iter2=400,
           fallback=FALLBACK_BACKTRACK, fit_codebook=False, sample_every=16, mlp=None, lambda_fp32=False,
           no_positivity=False, tau_hist: torch.Tensor | None = None, kl=False, lambda_bits: int = 0,
           ub_level: int | None = None, search: str = "guided", analytic_start: bool = False) -> Params:
    """tau_hist: optional per-histogram bounds (device, float64, one per histogram), used in
    place of tau.  ub_level: None searches the coder's step per histogram ('ab'); an
    integer 0..40 quantises every coded histogram with that ladder step ('ub').  search:
    "guided" (exponential search from the predicted ladder index, then bisection) or
    "bisect" (bisection over the whole ladder).  analytic_start: Newton starts from
    (A A^T)^-1 (A f~ - b) under the warm-start acceptance rule (not with mlp)."""
    if analytic_start and mlp is not None:
        raise ValueError("analytic_start and a warm-start network exclude each other")
    if search not in ("guided", "bisect"):
        raise ValueError("search must be 'guided' or 'bisect'")
    if tau_hist is not None and (tau_hist.dtype != torch.float64 or not tau_hist.is_cuda
                                 or not tau_hist.is_contiguous()):
        raise ValueError("tau_hist must be a contiguous float64 device tensor")
    p = Params(tau, tau_mode, newton_s, newton_max_iter, newton_max_iter2, fallback,
               int(fit_codebook), sample_every,
               WARM_MLP if mlp is not None else WARM_ANALYTIC if analytic_start else WARM_COLD,
               None if mlp is None else mlp.h, int(lambda_fp32), int(no_positivity),
               None if tau_hist is None else tau_hist.data_ptr(), int(kl), int(lambda_bits),
               BOUND_AB if ub_level is None else BOUND_UB, 0 if ub_level is None else int(ub_level),
               SEARCH_BISECT if search == "bisect" else SEARCH_GUIDED)
    p._mlp = mlp          # keep the network and the bounds alive as long as the parameters
    p._tau_hist = tau_hist
    return p


class Mlp:
    """The warm-start multiplier network on the device (inference)."""

    def __init__(self, ctx: Context, params: np.ndarray, scale):
        self.ctx = ctx
        w = np.ascontiguousarray(params, np.float32)
        sc = np.ascontiguousarray(scale, np.float64)
        h = C.c_void_p()
        _check(LIB.hcz_mlp_load(ctx.h, w.ctypes.data_as(C.c_void_p), sc.ctypes.data_as(C.c_void_p), C.byref(h)))
        self.h = h

    def predict(self, codes: torch.Tensor, centroids: torch.Tensor) -> torch.Tensor:
        H = codes.shape[0]
        out = torch.empty((H, 4), dtype=torch.float64, device=codes.device)
        cb = _cb(centroids)
        _check(LIB.hcz_mlp_predict(self.h, _ptr(codes.contiguous()), C.byref(cb), H, _ptr(out), _stream()))
        return out

    def __del__(self):
        if getattr(self, "h", None) and LIB is not None:   # LIB is None during interpreter shutdown
            LIB.hcz_mlp_free(self.h)
            self.h = None


def dequantize(codes: torch.Tensor, centroids: torch.Tensor) -> torch.Tensor:
    n, L = codes.shape
    z = torch.empty((n, L), dtype=torch.float32, device=codes.device)
    cb = _cb(centroids)
    _check(LIB.hcz_dequantize(_ptr(codes.contiguous()), n, L, C.byref(cb), _ptr(z), _stream()))
    return z


@dataclass
class Compressed:
    codes: torch.Tensor        # (H, latent) uint8
    lam: torch.Tensor          # (H, 4) float64, or float32 for FP32 multipliers
    flags: torch.Tensor        # (H,) uint8
    offsets: torch.Tensor      # (H + 1,) int64 (u64 bits)
    stream: torch.Tensor       # (capacity,) uint8
    stats_dev: torch.Tensor    # sizeof(hcz_stats) bytes
    t_done: torch.Tensor | None = None   # (H,) int64 (u64 bits): wall clock per histogram
    in_dtype: torch.dtype | None = None  # element type the batch was compressed from

    def cstruct(self) -> CompressedC:
        return CompressedC(self.codes.data_ptr(), self.lam.data_ptr(), self.flags.data_ptr(),
                           self.offsets.data_ptr(), self.stream.data_ptr(), self.stream.numel(),
                           self.stats_dev.data_ptr(), int(self.lam.dtype == torch.float32),
                           None if self.t_done is None else self.t_done.data_ptr())

    def stats(self) -> dict:
        s = Stats()
        st = LIB.hcz_stats_read(C.c_void_p(self.stats_dev.data_ptr()), C.byref(s), _stream())
        d = s.as_dict()
        if st not in (0, -5):
            _check(st)
        return d

    def stream_bytes(self) -> bytes:
        n = int(self.offsets[-1].item())
        return bytes(self.stream[:n].cpu().numpy().tobytes())


def alloc_compressed(H: int, N: int, device, latent=LATENT, capacity: int | None = None,
                     in_bytes: int = 4, lambda_fp32: bool = False, timestamps: bool = False) -> Compressed:
    if capacity is None:
        capacity = H * (24 + in_bytes * N)
    return Compressed(
        t_done=torch.zeros(H, dtype=torch.int64, device=device) if timestamps else None,
        codes=torch.zeros((H, latent), dtype=torch.uint8, device=device),
        lam=torch.zeros((H, 4), dtype=torch.float32 if lambda_fp32 else torch.float64, device=device),
        flags=torch.zeros(H, dtype=torch.uint8, device=device),
        offsets=torch.zeros(H + 1, dtype=torch.int64, device=device),
        stream=torch.empty(max(capacity, 16), dtype=torch.uint8, device=device),
        stats_dev=torch.zeros(C.sizeof(Stats), dtype=torch.uint8, device=device),
    )


def workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---- stage entry points --------------------------------------------------------------

def qoi(plan: Plan, hist: torch.Tensor):
    H, hs, rs = _strides(hist)
    dev = hist.device
    b = torch.empty((H, 4), dtype=torch.float64, device=dev)
    q = torch.empty((H, 4), dtype=torch.float64, device=dev)
    n = torch.empty(H, dtype=torch.float64, device=dev)
    _check(LIB.hcz_qoi(plan.h, _ptr(hist), _dtype_code(hist), H, hs, rs, _ptr(b), _ptr(q), _ptr(n), _stream()))
    return b, q, n


def encode(model: Model, hist: torch.Tensor) -> torch.Tensor:
    H, hs, rs = _strides(hist)
    z = torch.empty((H, model.latent), dtype=torch.float32, device=hist.device)
    _check(LIB.hcz_encode(model.h, _ptr(hist), _dtype_code(hist), H, hs, rs, _ptr(z), _stream()))
    return z


def codebook_fit(z: torch.Tensor, bits: int = 8, sample_every: int = 1) -> torch.Tensor:
    z = z.contiguous()
    n, L = z.shape
    nbytes = C.c_size_t()
    _check(LIB.hcz_codebook_fit_workspace(n, L, sample_every, C.byref(nbytes)))
    ws = workspace(nbytes.value, z.device)
    cent = torch.empty((L, 1 << bits), dtype=torch.float32, device=z.device)
    cb = Codebook(bits, cent.data_ptr())
    _check(LIB.hcz_codebook_fit(_ptr(z), n, L, sample_every, C.byref(cb), _ptr(ws), ws.numel(), _stream()))
    return cent


def _cb(centroids: torch.Tensor) -> Codebook:
    k = centroids.shape[1]
    bits = int(k).bit_length() - 1
    if 1 << bits != k:
        raise ValueError("codebook size must be a power of two")
    return Codebook(bits, centroids.data_ptr())


def quantize(z: torch.Tensor, centroids: torch.Tensor) -> torch.Tensor:
    z = z.contiguous()
    n, L = z.shape
    codes = torch.empty((n, L), dtype=torch.uint8, device=z.device)
    cb = _cb(centroids)
    _check(LIB.hcz_quantize(_ptr(z), n, L, C.byref(cb), _ptr(codes), _stream()))
    return codes


def decode(model: Model, codes: torch.Tensor, centroids: torch.Tensor) -> torch.Tensor:
    H = codes.shape[0]
    out = torch.empty((H, model.plan.n_perp, model.plan.n_par), dtype=torch.float32, device=codes.device)
    cb = _cb(centroids)
    _check(LIB.hcz_decode(model.h, _ptr(codes.contiguous()), C.byref(cb), H, _ptr(out), _stream()))
    return out


def residual(plan: Plan, p: Params, hist: torch.Tensor, fhat: torch.Tensor | None,
             capacity: int | None = None, lam0: torch.Tensor | None = None) -> Compressed:
    H, hs, rs = _strides(hist)
    nbytes = C.c_size_t()
    _check(LIB.hcz_compress_workspace(plan.h, None, H, C.byref(p), C.byref(nbytes)))
    ws = workspace(nbytes.value, hist.device)
    out = alloc_compressed(H, plan.N, hist.device, capacity=capacity, in_bytes=hist.element_size(),
                           lambda_fp32=bool(p.lambda_fp32))
    out.in_dtype = hist.dtype
    cs = out.cstruct()
    fh = None if fhat is None else fhat.contiguous()
    l0 = None if lam0 is None else lam0.contiguous()
    _check(LIB.hcz_residual(plan.h, C.byref(p), _ptr(hist), _dtype_code(hist), H, hs, rs, _ptr(fh), _ptr(l0),
                            C.byref(cs), _ptr(ws), ws.numel(), _stream()))
    out._ws = ws
    return out


# ---- whole path ------------------------------------------------------------------------

class Compressor:
    """Preallocated compress/decompress for batches of up to H histograms (no allocation per call)."""

    def __init__(self, plan: Plan, model: Model | None, H: int, p: Params, bits: int = 8,
                 in_dtype=torch.float32, capacity: int | None = None, device="cuda", timestamps: bool = False):
        self.plan, self.model, self.H, self.p = plan, model, H, p
        nbytes = C.c_size_t()
        _check(LIB.hcz_compress_workspace(plan.h, None if model is None else model.h, H, C.byref(p),
                                          C.byref(nbytes)))
        self.ws = workspace(nbytes.value, device)
        _check(LIB.hcz_decompress_workspace(plan.h, None if model is None else model.h, H, C.byref(nbytes)))
        self.dws = workspace(nbytes.value, device)
        esz = 4 if in_dtype == torch.float32 else 8
        self.out = alloc_compressed(H, plan.N, device, capacity=capacity, in_bytes=esz,
                                    lambda_fp32=bool(p.lambda_fp32), timestamps=timestamps)
        self.centroids = torch.zeros((LATENT, 1 << bits), dtype=torch.float32, device=device)
        self.bits = bits
        self.in_dtype = in_dtype

    def compress(self, hist: torch.Tensor) -> Compressed:
        H, hs, rs = _strides(hist)
        if H > self.H:
            raise ValueError("batch larger than the compressor was sized for")
        if hist.dtype == torch.float64 and self.in_dtype != torch.float64:
            raise ValueError("FP64 input needs a compressor built with in_dtype=torch.float64 "
                             "(its verbatim records take 8N bytes)")
        self.out.in_dtype = hist.dtype
        cb = Codebook(self.bits, self.centroids.data_ptr())
        cs = self.out.cstruct()
        _check(LIB.hcz_compress(self.plan.h, None if self.model is None else self.model.h, C.byref(cb),
                                C.byref(self.p), _ptr(hist), _dtype_code(hist), H, hs, rs, C.byref(cs),
                                _ptr(self.ws), self.ws.numel(), _stream()))
        return self.out

    def decompress(self, comp: Compressed, H: int, in_dtype=None,
                   out_dtype=torch.float64) -> torch.Tensor:
        out = torch.empty((H, self.plan.n_perp, self.plan.n_par), dtype=out_dtype, device=comp.lam.device)
        return self.decompress_into(comp, H, out, in_dtype)

    def decompress_into(self, comp: Compressed, H: int, out: torch.Tensor, in_dtype=None):
        """in_dtype: the element type the batch was compressed from (its verbatim records);
        by default the one the batch records, else the compressor's.  A value that
        contradicts the batch's own is refused."""
        if in_dtype is None:
            in_dtype = comp.in_dtype if comp.in_dtype is not None else self.in_dtype
        elif comp.in_dtype is not None and in_dtype != comp.in_dtype:
            raise ValueError(f"batch was compressed from {comp.in_dtype}, not {in_dtype}")
        cb = Codebook(self.bits, self.centroids.data_ptr())
        cs = comp.cstruct()
        _check(LIB.hcz_decompress(self.plan.h, None if self.model is None else self.model.h, C.byref(cb),
                                  C.byref(cs), F32 if in_dtype == torch.float32 else F64, H, _ptr(out),
                                  _dtype_code(out), _ptr(self.dws), self.dws.numel(), _stream()))
        return out


def compress_batch(compressors: list, hists: list, batch_ws: torch.Tensor | None = None) -> list:
    """hcz_compress_batch: compressors[k] compresses hists[k] (grids may differ), with one
    persistent launch of the residual stage for all of them; returns each compressor's
    Compressed.  batch_ws: a device buffer of BATCH_WORKSPACE_BYTES (allocated here if None)."""
    if len(compressors) != len(hists):
        raise ValueError("one input per compressor")
    n = len(compressors)
    segs = (BatchSegmentC * max(n, 1))()
    keep = []
    for k, (cz, hist) in enumerate(zip(compressors, hists)):
        H, hs, rs = _strides(hist)
        if H > cz.H:
            raise ValueError("batch larger than the compressor was sized for")
        if hist.dtype == torch.float64 and cz.in_dtype != torch.float64:
            raise ValueError("FP64 input needs a compressor built with in_dtype=torch.float64")
        cz.out.in_dtype = hist.dtype
        cb = Codebook(cz.bits, cz.centroids.data_ptr())
        cs = cz.out.cstruct()
        keep += [cb, cs]
        segs[k] = BatchSegmentC(cz.plan.h, None if cz.model is None else cz.model.h, C.pointer(cb),
                                C.pointer(cz.p), hist.data_ptr(), _dtype_code(hist), H, hs, rs, C.pointer(cs),
                                cz.ws.data_ptr(), cz.ws.numel())
    if batch_ws is None:
        dev = hists[0].device if hists else torch.device("cuda")
        batch_ws = torch.empty(BATCH_WORKSPACE_BYTES, dtype=torch.uint8, device=dev)
    _check(LIB.hcz_compress_batch(segs, n, _ptr(batch_ws), batch_ws.numel(), _stream()))
    return [cz.out for cz in compressors]


def norm_stats(plan: Plan, hist: torch.Tensor):
    """Per-pixel z-score statistics (mean, std) of a batch, as FP32 numpy arrays."""
    H, hs, rs = _strides(hist)
    nbytes = C.c_size_t()
    _check(LIB.hcz_norm_stats_workspace(plan.h, H, C.byref(nbytes)))
    ws = workspace(nbytes.value, hist.device)
    mu = torch.empty(plan.N, dtype=torch.float32, device=hist.device)
    sd = torch.empty(plan.N, dtype=torch.float32, device=hist.device)
    _check(LIB.hcz_norm_stats(plan.h, _ptr(hist), _dtype_code(hist), H, hs, rs, _ptr(mu), _ptr(sd),
                              _ptr(ws), ws.numel(), _stream()))
    return mu, sd


def _matrix(x: torch.Tensor):
    """(rows, cols, row stride) of a 2-D view whose columns are contiguous (any trailing
    dimensions of a contiguous tensor are flattened into the columns)."""
    if x.dim() != 2:
        x = x.reshape(x.shape[0], -1)
    if x.stride(1) != 1:
        raise ValueError("columns must be contiguous")
    return x, x.shape[0], x.shape[1], x.stride(0)


def column_stats(x: torch.Tensor):
    """Per-column mean and population std (std floored at 1e-12 of the largest) of a matrix
    (rows x cols, FP32 or FP64), as FP32 device tensors."""
    x, rows, cols, ld = _matrix(x)
    nbytes = C.c_size_t()
    _check(LIB.hcz_column_stats_workspace(rows, cols, C.byref(nbytes)))
    ws = workspace(nbytes.value, x.device)
    mu = torch.empty(cols, dtype=torch.float32, device=x.device)
    sd = torch.empty(cols, dtype=torch.float32, device=x.device)
    _check(LIB.hcz_column_stats(_ptr(x), _dtype_code(x), rows, cols, ld, _ptr(mu), _ptr(sd), _ptr(ws), ws.numel(),
                                _stream()))
    return mu, sd


def column_normalize(x: torch.Tensor, mean: torch.Tensor | None, std: torch.Tensor) -> torch.Tensor:
    """(x - mean) / std per column in FP32 (mean None: x / std), as a dense FP32 matrix of
    x's rows; histograms (H, n_perp, n_par) are taken as rows of N values."""
    x, rows, cols, ld = _matrix(x)
    out = torch.empty((rows, cols), dtype=torch.float32, device=x.device)
    m = None if mean is None else mean.contiguous().float()
    sd = std.contiguous().float()
    _check(LIB.hcz_column_normalize(_ptr(x), _dtype_code(x), rows, cols, ld, _ptr(m), _ptr(sd), _ptr(out),
                                    _stream()))
    return out


# ---- batches of subdomains --------------------------------------------------------------

PROBE_FP64_FMA, PROBE_FP32_MFMA, PROBE_BF16_MFMA = 0, 1, 2


def ceilings(copy_bytes: int = 1 << 31, reps: int = 5, iters: dict | None = None) -> dict:
    """Measured ceilings of the current device: streaming-copy rate (bytes read + written
    per second) and FP64 FMA, FP32 and BF16 matrix-core rates of the probe kernels, each the
    best of `reps` launches timed with events on the current stream."""
    iters = iters or {PROBE_FP64_FMA: 100000, PROBE_FP32_MFMA: 10000, PROBE_BF16_MFMA: 10000}
    src = torch.empty(copy_bytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)

    def best(fn):
        t = []
        for _ in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            e1.synchronize()
            t.append(e0.elapsed_time(e1) / 1e3)
        return min(t[1:])

    out = {"copy_bytes": copy_bytes,
           "hbm_copy_GBps": 2 * copy_bytes / best(lambda: _check(LIB.hcz_probe_copy(_ptr(src), _ptr(dst), copy_bytes,
                                                                                     _stream()))) / 1e9}
    del src, dst
    nb = C.c_size_t()
    _check(LIB.hcz_probe_sink_bytes(C.byref(nb)))
    sink = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    fl = C.c_double()
    for kind, name in ((PROBE_FP64_FMA, "fp64_fma_TFLOPs"), (PROBE_FP32_MFMA, "fp32_mfma_TFLOPs"),
                       (PROBE_BF16_MFMA, "bf16_mfma_TFLOPs")):
        dt = best(lambda: _check(LIB.hcz_probe_compute(kind, iters[kind], _ptr(sink), C.byref(fl), _stream())))
        out[name] = fl.value / dt / 1e12
    return out


def segment_tau(seg_start: torch.Tensor, seg_tau: torch.Tensor, H: int) -> torch.Tensor:
    """Per-histogram bounds of a batch of subdomains: histogram h of subdomain s (rows
    seg_start[s] .. seg_start[s+1]-1) gets seg_tau[s]."""
    nseg = seg_tau.numel()
    if seg_start.dtype != torch.int64 or seg_start.numel() != nseg + 1 or seg_tau.dtype != torch.float64:
        raise ValueError("seg_start: int64 [nseg+1], seg_tau: float64 [nseg]")
    out = torch.empty(H, dtype=torch.float64, device=seg_tau.device)
    _check(LIB.hcz_segment_tau(_ptr(seg_start.contiguous()), _ptr(seg_tau.contiguous()), nseg, H, _ptr(out),
                               _stream()))
    return out


def segment_max(seg_start: torch.Tensor, t: torch.Tensor) -> torch.Tensor:
    """Per-subdomain maximum of a per-histogram u64 array (int64 bits), e.g. t_done."""
    nseg = seg_start.numel() - 1
    out = torch.empty(nseg, dtype=torch.int64, device=t.device)
    _check(LIB.hcz_segment_max(_ptr(seg_start.contiguous()), nseg, t.numel(), _ptr(t), _ptr(out), _stream()))
    return out


def timestamp(device="cuda") -> torch.Tensor:
    """A one-element int64 tensor set to the device wall clock when the stream gets there."""
    out = torch.zeros(1, dtype=torch.int64, device=device)
    _check(LIB.hcz_timestamp(_ptr(out), _stream()))
    return out


def wall_clock_hz(device: int = 0) -> float:
    hz = C.c_double()
    _check(LIB.hcz_wall_clock_hz(device, C.byref(hz)))
    return hz.value


# ---- output container and rANS (host) ----------------------------------------------------

def _np_ptr(a):
    return None if a is None else C.c_void_p(a.ctypes.data)


def rans_encode(data: bytes | np.ndarray) -> bytes:
    a = np.frombuffer(bytes(data), np.uint8) if not isinstance(data, np.ndarray) else np.ascontiguousarray(data, np.uint8)
    nb = C.c_size_t()
    _check(LIB.hcz_rans_bound(a.size, C.byref(nb)))
    out = np.empty(nb.value, np.uint8)
    w = C.c_size_t()
    _check(LIB.hcz_rans_encode(_np_ptr(a) if a.size else C.c_void_p(out.ctypes.data), a.size, _np_ptr(out), out.size,
                               C.byref(w)))
    return out[:w.value].tobytes()


def rans_decode(block: bytes, n: int) -> np.ndarray:
    b = np.frombuffer(block, np.uint8)
    out = np.empty(max(n, 1), np.uint8)
    _check(LIB.hcz_rans_decode(_np_ptr(b), b.size, _np_ptr(out), n))
    return out[:n]


def container_pack(n_par: int, n_perp: int, flags, res_offset, res_bytes, lam, codes=None, centroids=None,
                   weights=None, norm_mean=None, norm_std=None, arch: str | None = None, compute: str = "fp32",
                   entropy: int = 0) -> bytes:
    """Pack host (numpy) arrays of one compressed batch into the container (see hcz.h);
    entropy 0 (none), 1 (byte-wise rANS) or 2 (rANS of the residual integers by group)."""
    flags = np.ascontiguousarray(flags, np.uint8)
    H = flags.size
    res_offset = np.ascontiguousarray(res_offset, np.uint64)
    res_bytes = np.ascontiguousarray(res_bytes, np.uint8)
    lam = np.ascontiguousarray(lam)
    info = ContainerInfo(H, n_par, n_perp, 0 if arch is None else (ARCH_CONV if arch == "conv" else ARCH_DENSE),
                         _COMPUTE[compute], 0, 0, int(lam.dtype == np.float32),
                         int(entropy), 0, 0, 0)
    keep = [flags, res_offset, res_bytes, lam]
    cin = ContainerIn(info, None, None, None, None, None, _np_ptr(flags), _np_ptr(res_offset),
                      _np_ptr(res_bytes) if res_bytes.size else None, _np_ptr(lam))
    if arch is not None:
        codes = np.ascontiguousarray(codes, np.uint8)
        centroids = np.ascontiguousarray(centroids, np.float32)
        weights = np.ascontiguousarray(weights, np.float32)
        norm_mean = np.ascontiguousarray(norm_mean, np.float32)
        norm_std = np.ascontiguousarray(norm_std, np.float32)
        keep += [codes, centroids, weights, norm_mean, norm_std]
        cin.info.latent = codes.shape[1]
        cin.info.bits = int(np.log2(centroids.shape[1]))
        cin.info.n_weights = weights.size
        cin.weights, cin.norm_mean, cin.norm_std = _np_ptr(weights), _np_ptr(norm_mean), _np_ptr(norm_std)
        cin.codes, cin.centroids = _np_ptr(codes), _np_ptr(centroids)
    nb = C.c_size_t()
    _check(LIB.hcz_container_bound(C.byref(cin), C.byref(nb)))
    out = np.empty(nb.value, np.uint8)
    w = C.c_size_t()
    _check(LIB.hcz_container_pack(C.byref(cin), _np_ptr(out), out.size, C.byref(w)))
    del keep
    return out[:w.value].tobytes()


def container_unpack(buf: bytes) -> dict:
    """The arrays of a packed container (numpy) and its header fields."""
    b = np.frombuffer(buf, np.uint8)
    info = ContainerInfo()
    _check(LIB.hcz_container_read_info(_np_ptr(b), b.size, C.byref(info)))
    H, N = info.H, info.n_par * info.n_perp
    d = dict(H=H, n_par=info.n_par, n_perp=info.n_perp, entropy=int(info.entropy),
             flags=np.empty(H, np.uint8), res_offset=np.empty(H + 1, np.uint64),
             res_bytes=np.empty(max(int(info.res_bytes), 1), np.uint8),
             lam=np.empty((H, 4), np.float32 if info.lambda_fp32 else np.float64))
    out = ContainerOut(None, None, None, None, None, _np_ptr(d["flags"]), _np_ptr(d["res_offset"]),
                       _np_ptr(d["res_bytes"]), _np_ptr(d["lam"]))
    if info.arch:
        d.update(arch="conv" if info.arch == ARCH_CONV else "dense",
                 compute={v: k for k, v in _COMPUTE.items()}[info.compute],
                 weights=np.empty(info.n_weights, np.float32), norm_mean=np.empty(N, np.float32),
                 norm_std=np.empty(N, np.float32), codes=np.empty((H, info.latent), np.uint8),
                 centroids=np.empty((info.latent, 1 << info.bits), np.float32))
        out.weights, out.norm_mean, out.norm_std = _np_ptr(d["weights"]), _np_ptr(d["norm_mean"]), _np_ptr(d["norm_std"])
        out.codes, out.centroids = _np_ptr(d["codes"]), _np_ptr(d["centroids"])
    else:
        d["arch"] = None
    _check(LIB.hcz_container_unpack(_np_ptr(b), b.size, C.byref(out)))
    d["res_bytes"] = d["res_bytes"][:int(info.res_bytes)]
    return d
