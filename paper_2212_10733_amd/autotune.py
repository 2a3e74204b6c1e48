"""Autotuner of the residual stage's launch per grid (the kernel family and its shape:
one wave per histogram with the slot structure compiled in or read at run time, or one
workgroup of 256 or 512 threads with 6, 5 or 9 nodes per thread).

Every variant produces the same bytes, so the choice is speed only.  `tune` times the
coder-only compress of synthetic histograms of the plan's grid (the seeded generator of
`synth`) with each variant valid for the grid and returns the milliseconds per call;
`best` picks the fastest.  Choices are cached in a JSON file keyed by the GPU
architecture, the grid, the input dtype and whether the cell volumes are uniform;
`apply` sets a plan's variant from the cache and tunes on a miss.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import hcz, synth


def key(arch: str, n_perp: int, n_par: int, dtype: str, uniform: bool) -> str:
    """Cache key: architecture (without feature suffixes), grid, input dtype, volumes."""
    return f"{arch.split(':')[0]}|{n_perp}x{n_par}|{dtype}|{'uniform' if uniform else 'vol'}"


def plan_key(plan: hcz.Plan, dtype: torch.dtype = torch.float32) -> str:
    arch = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    return key(arch, plan.n_perp, plan.n_par, "f32" if dtype == torch.float32 else "f64", plan._vol is None)


def load(path: str) -> dict:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as f:
        data = json.load(f)
    if not isinstance(data, dict):
        raise ValueError(f"{path}: not an autotuner cache")
    return data


def save(path: str, cache: dict) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def best(times: dict) -> str:
    """The fastest variant; ties go to the first in the plan's order (auto first)."""
    return min(times, key=lambda v: (times[v], list(times).index(v)))


def tune(plan: hcz.Plan, dtype: torch.dtype = torch.float32, H: int = 32768, tau: float = 1e-3,
         reps: int = 3, seed: int = 7) -> dict:
    """Milliseconds per coder-only compress of H synthetic histograms for each valid
    variant (median of `reps` timed calls after one warm-up); the plan's variant is restored."""
    npd = np.float32 if dtype == torch.float32 else np.float64
    x = torch.from_numpy(synth.histograms(H, plan.n_par, plan.n_perp, seed=seed, dtype=npd)).cuda()
    cz = hcz.Compressor(plan, None, H, hcz.params(tau=tau), in_dtype=dtype)
    before = plan.variant
    times = {}
    try:
        for v in plan.variants():
            plan.set_variant(v)
            cz.compress(x)
            ms = []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                cz.compress(x)
                e1.record()
                e1.synchronize()
                ms.append(e0.elapsed_time(e1))
            times[v] = float(np.median(ms))
    finally:
        plan.set_variant(before)
    return times


def apply(plan: hcz.Plan, path: str | None = None, dtype: torch.dtype = torch.float32, **tune_kw) -> str:
    """Set the plan's variant from the cache at `path` (tuning and recording it when the key
    is missing or names a variant the grid does not allow); returns the variant."""
    cache = load(path) if path else {}
    k = plan_key(plan, dtype)
    entry = cache.get(k)
    if not entry or entry.get("variant") not in plan.variants():
        times = tune(plan, dtype, **tune_kw)
        entry = {"variant": best(times), "ms": times}
        cache[k] = entry
        if path:
            save(path, cache)
    plan.set_variant(entry["variant"])
    return entry["variant"]
