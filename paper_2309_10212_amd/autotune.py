"""Autotuner of a batched launch.

Chooses, for a set of render requests run as one batch, the speculation cap
(Sec. 4: N_spec = clamp(floor(w*h / N_act), 1, cap)) and the block-raytrace
launch tuning (sorted pairs per workgroup, blocks staged in LDS per tile, or
no staging: each pair reads its corners from the cache slots).
None of these changes an image; they trade passes against per-pass work and
occupancy.  The tuner renders a seeded sample of the requests as one batch
under every candidate, after one untimed warm-up run so that every candidate
sees a warm block cache, and keeps the candidate with the highest rays/s.

Host-side orchestration only: every render runs in libspr's kernels.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import spr

DEFAULT_CAPS = (4, 8, 16, 32, 64)
DEFAULT_TILES = ((256, 0), (128, 16), (128, 32), (256, 16), (256, 32))


@dataclass
class Choice:
    spec_cap: int
    pairs_per_wg: int
    slot_tile: int
    rays_per_s: float
    seconds: float
    passes: int


def run_batch(ctx, vols, reqs, spec_cap: int, poll_every: int = 2):
    """Render reqs (objects with .vol .cam .iso .w .h) as one batch to completion.
    Returns (seconds, rays entered, passes, renders) - renders still allocated.
    The clock runs from before the first render's set-up (initial rays and
    isovalue masks) to the last pass, as a plain render's clock would."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    renders = [spr.Render(vols[q.vol], q.cam, q.iso, q.w, q.h, spec_cap=spec_cap) for q in reqs]
    b = spr.Batch(ctx, renders)
    passes = b.run(poll_every=poll_every)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    b.free()
    rays = sum(r.info()["rays_entered"] for r in renders)
    return dt, rays, passes, renders


def autotune(ctx, vols, reqs, caps=DEFAULT_CAPS, tiles=DEFAULT_TILES, sample: int = 8, seed: int = 0):
    """Returns (best Choice, list of every Choice); leaves ctx tuned to the best."""
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(reqs), min(sample, len(reqs)), replace=False)
    sub = [reqs[i] for i in sorted(idx)]
    _, _, _, rs = run_batch(ctx, vols, sub, caps[-1])   # warm-up: block cache and graph shapes
    for r in rs:
        r.free()
    table = []
    for ppw, st in tiles:
        ctx.set_tuning(ppw, st)
        for cap in caps:
            dt, rays, passes, rs = run_batch(ctx, vols, sub, cap)
            for r in rs:
                r.free()
            table.append(Choice(cap, ppw, st, rays / dt if dt > 0 else 0.0, dt, passes))
    best = max(table, key=lambda c: c.rays_per_s)
    ctx.set_tuning(best.pairs_per_wg, best.slot_tile)
    return best, table
