"""Batches of subdomains of uneven sizes over several velocity grids, each subdomain with
its own bound (the paper's per-rank subdomains of the mesh, Section III-A, compressed
together on one device).

The subdomains of one grid size are laid out back to back and compressed by one
hcz_compress call with per-histogram bounds (hcz_segment_tau expands the per-subdomain
tau); every grid size has its own plan, model and codebook.  The residual stage stamps the
device wall clock as each histogram finishes, and hcz_segment_max turns those stamps into
per-subdomain completion times.  Allocation happens at construction; compress() only
launches, so the whole batch (every grid size) can be recorded once into a HIP graph
(capture) and rerun with a single launch (replay).  With a tuning cache, each grid's
residual launch variant comes from the autotuner.  With persistent=True the residual
stage of every grid size runs as one persistent launch (hcz_compress_batch) that serves
the histograms of all grids from one work list, instead of one launch per grid.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hcz


class SubdomainBatch:
    def __init__(self, plans: dict, models: dict, layout: list, bits: int = 8, sample_every: int = 16,
                 device="cuda", tune_cache: str | None = None, persistent: bool = False, **param_kw):
        """plans / models: grid key -> Plan / Model (or None: the coder-only pipeline);
        layout: [(grid key, count, tau)] in batch order; tune_cache: a JSON file of the
        autotuner (read, and extended on a miss) to choose each plan's launch variant;
        persistent: one residual launch for every grid (at most hcz.BATCH_MAX_SEGMENTS grid
        sizes; the launch variants are then those of the batch kernel, not the tuner's)."""
        self.layout = list(layout)
        self.persistent = persistent
        if tune_cache is not None:
            from . import autotune
            for k in plans:
                if any(g == k for g, _, _ in self.layout):
                    autotune.apply(plans[k], tune_cache)
        self.graph = None
        self.keys = [k for k in plans if any(g == k for g, _, _ in self.layout)]
        self.groups = {}
        for k in self.keys:
            idx = [i for i, (g, _, _) in enumerate(self.layout) if g == k]
            counts = np.array([self.layout[i][1] for i in idx], np.int64)
            start = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
            H = int(start[-1])
            tau_buf = torch.empty(max(H, 1), dtype=torch.float64, device=device)
            p = hcz.params(tau_hist=tau_buf, fit_codebook=models.get(k) is not None, sample_every=sample_every,
                           **param_kw)
            self.groups[k] = dict(
                index=idx, H=H, start_host=start,
                start=torch.from_numpy(start).to(device),
                tau=torch.tensor([self.layout[i][2] for i in idx], dtype=torch.float64, device=device),
                tau_buf=tau_buf, params=p,
                cz=hcz.Compressor(plans[k], models.get(k), max(H, 1), p, bits=bits, device=device,
                                  timestamps=True))
        if persistent and len(self.keys) > hcz.BATCH_MAX_SEGMENTS:
            raise ValueError(f"a persistent batch holds at most {hcz.BATCH_MAX_SEGMENTS} grid sizes")
        self.batch_ws = torch.zeros(hcz.BATCH_WORKSPACE_BYTES, dtype=torch.uint8, device=device)
        self.t0 = torch.zeros(1, dtype=torch.int64, device=device)
        self.done = {}

    def compress(self, inputs: dict) -> dict:
        """inputs: grid key -> (H_k, n_perp, n_par) tensor of that grid's subdomains, back to
        back in layout order.  Returns grid key -> Compressed (the compressor's buffers)."""
        out = {}
        hcz._check(hcz.LIB.hcz_timestamp(hcz._ptr(self.t0), hcz._stream()))
        if self.persistent:
            keys = [k for k in self.keys if self.groups[k]["H"] > 0]
            for k in keys:
                g = self.groups[k]
                hcz._check(hcz.LIB.hcz_segment_tau(hcz._ptr(g["start"]), hcz._ptr(g["tau"]), len(g["index"]),
                                                   g["H"], hcz._ptr(g["tau_buf"]), hcz._stream()))
            comps = hcz.compress_batch([self.groups[k]["cz"] for k in keys], [inputs[k] for k in keys],
                                       self.batch_ws)
            for k, comp in zip(keys, comps):
                self.done[k] = hcz.segment_max(self.groups[k]["start"], comp.t_done)
                out[k] = comp
            return out
        for k in self.keys:
            g = self.groups[k]
            if g["H"] == 0:
                continue
            hcz._check(hcz.LIB.hcz_segment_tau(hcz._ptr(g["start"]), hcz._ptr(g["tau"]), len(g["index"]), g["H"],
                                               hcz._ptr(g["tau_buf"]), hcz._stream()))
            comp = g["cz"].compress(inputs[k])
            self.done[k] = hcz.segment_max(g["start"], comp.t_done)
            out[k] = comp
        return out

    def capture(self, inputs: dict) -> dict:
        """Record compress(inputs) into a HIP graph (torch.cuda.CUDAGraph, default stream
        priority) after one eager call; returns the graph's outputs, which replay()
        refreshes.  The inputs must stay at the same device addresses."""
        self.compress(inputs)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.graph_out = self.compress(inputs)
        torch.cuda.synchronize()
        return self.graph_out

    def replay(self) -> dict:
        """Rerun the captured batch (asynchronous); the outputs are those capture() returned."""
        if self.graph is None:
            raise RuntimeError("capture() first")
        self.graph.replay()
        return self.graph_out

    def completion_seconds(self) -> np.ndarray:
        """Seconds from the start of the last compress() to each subdomain's last histogram
        leaving the residual stage, in layout order (synchronises)."""
        hz = hcz.wall_clock_hz(torch.cuda.current_device())
        t0 = int(self.t0.item())
        res = np.zeros(len(self.layout))
        for k, d in self.done.items():
            res[self.groups[k]["index"]] = (d.cpu().numpy() - t0) / hz
        return res

    def decompress(self, comps: dict, in_dtype=None) -> dict:
        return {k: self.groups[k]["cz"].decompress(c, self.groups[k]["H"], in_dtype=in_dtype)
                for k, c in comps.items()}
