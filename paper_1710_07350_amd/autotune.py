"""Autotuner of the batched persistent launch.

Searches the launch schedule of `trk_track_batched` -- particles per thread
(register tile), persistent blocks per compute unit, passes fused per launch
-- by timing each candidate on a scratch copy of the beam for a few passes
with HIP events, and keeps the fastest.  Results are cached per (GPU, beam
segment sizes, lattice length, element families) in memory and, optionally,
in a JSON file.  Every candidate computes the same result; only speed
differs.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
from typing import Dict, Optional

from . import binding as B

DEFAULT_SPACE = {"ppt": (1, 2, 4), "blocks_per_cu": (1, 2, 4, 8), "passes_per_launch": (0, 25)}
_CACHE: Dict[str, dict] = {}


def _key(batch: "B.Batch", passes: int) -> str:
    import torch
    dev = torch.cuda.get_device_properties(0)
    sizes = (batch.seg_off[1:] - batch.seg_off[:-1]).tolist()
    kinds = [e.kind for e in batch.lattices[0].elements]
    raw = json.dumps([getattr(dev, "gcnArchName", dev.name), sizes, kinds, passes])
    return hashlib.sha1(raw.encode()).hexdigest()


def tune_batch(batch: "B.Batch", beam: "B.Beam", probe_passes: int = 4, space=None,
               cache_path: Optional[str] = None, verbose: bool = False) -> dict:
    """Pick the fastest schedule for this batch; returns the tuning dict."""
    import torch
    key = _key(batch, probe_passes)
    if key in _CACHE:
        return dict(_CACHE[key])
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            disk = json.load(fh)
        if key in disk:
            _CACHE[key] = disk[key]
            return dict(disk[key])
    space = space or DEFAULT_SPACE
    scratch = B.Beam.__new__(B.Beam)
    scratch.n = beam.n
    scratch.z = beam.z.clone()
    scratch.id = beam.id.clone()
    scratch.lost_at = beam.lost_at.clone()
    scratch.n_alive = beam.n_alive.clone()
    ws = batch.workspace(64)
    best, best_ms, table = None, float("inf"), []
    for ppt, bpc, ppl in itertools.product(space["ppt"], space["blocks_per_cu"],
                                           space["passes_per_launch"]):
        tune = dict(ppt=ppt, blocks_per_cu=bpc, passes_per_launch=ppl, use_graph=False)
        scratch.z.copy_(beam.z)
        scratch.lost_at.copy_(beam.lost_at)
        B.track_batched(batch, scratch, 1, ws, **tune)            # warm-up
        scratch.z.copy_(beam.z)
        scratch.lost_at.copy_(beam.lost_at)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record()
        B.track_batched(batch, scratch, probe_passes, ws, **tune)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1)
        table.append((ms, tune))
        if verbose:
            print(f"autotune {tune}: {ms:.3f} ms")
        if ms < best_ms:
            best, best_ms = tune, ms
    best = dict(best, use_graph=True, probe_ms=best_ms)
    _CACHE[key] = best
    if cache_path:
        disk = {}
        if os.path.exists(cache_path):
            with open(cache_path) as fh:
                disk = json.load(fh)
        disk[key] = best
        with open(cache_path, "w") as fh:
            json.dump(disk, fh, indent=1)
    return dict(best)
