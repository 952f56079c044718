"""Serving loop: continuous batching of render requests over resident volumes.

Requests (camera + isovalue on one of the loaded volumes) arrive over time.
The server keeps one batch whose members change between passes (requests
join as soon as they are admitted and leave when their last ray terminates),
so requests that arrive while others are on the GPU share their passes
(Sec. 4's single launch over every active ray, here across requests).

Admission is by cache memory (Sec. 3.5): a request is admitted when the
estimated cache slots of the admitted set plus its own fit the cache.  The
estimate of a request is its volume's last observed per-pass active blocks
per request (the active blocks of a pass, shared out over the requests in it
by their active rays), or 8*w*h when the volume has not been observed yet;
an idle server admits the next request regardless.  Requests also need room
in the batch (member and pixel capacity).

Per-pass latency of a request is the time from its previous pass's
completion (from its arrival, for its first pass) to the pass's completion.

Host-side scheduling only: every pass runs in libspr's kernels.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import spr


@dataclass
class Result:
    idx: int
    arrival: float
    admitted: float
    finished: float
    passes: int
    rays_entered: int
    latencies: list = field(default_factory=list)
    hits: np.ndarray | None = None
    image: np.ndarray | None = None


class Server:
    def __init__(self, ctx: spr.Context, volumes, cache_bytes: int, max_requests: int = 32,
                 max_pixels: int | None = None, spec_cap: int = 16):
        self.ctx = ctx
        self.vols = list(volumes)
        self.n_slots = cache_bytes // 256
        self.max_requests = max_requests
        self.max_pixels = max_pixels if max_pixels is not None else max_requests * 1920 * 1080
        self.spec_cap = spec_cap
        self.batch = spr.Batch(ctx, max_requests=max_requests, max_pixels=self.max_pixels)
        self.per_request_blocks = {}   # volume index -> estimated active blocks per request

    def estimate(self, req) -> int:
        est = self.per_request_blocks.get(req.vol)
        return int(est) if est is not None else 8 * req.w * req.h

    def run(self, arrivals, keep_results: bool = False, clock=time.perf_counter):
        """Serve arrivals (objects with .t .vol .w .h .iso .cam, sorted by t, in
        seconds from the start) in real time.  Returns (results, stats)."""
        pending = deque(enumerate(arrivals))
        waiting = deque()
        active = []            # dicts: idx, req, render, est, last_done, result
        results = [None] * len(arrivals)
        lat = []
        max_active = 0
        passes = 0
        t0 = clock()
        members_changed = False
        while pending or waiting or active:
            now = clock() - t0
            while pending and pending[0][1].t <= now:
                waiting.append(pending.popleft())
            # admission: cache memory, members, pixels
            used = sum(a["est"] for a in active)
            pixels = sum(a["req"].w * a["req"].h for a in active)
            while waiting and len(active) < self.max_requests:
                i, q = waiting[0]
                est = self.estimate(q)
                if active and (used + est > self.n_slots or pixels + q.w * q.h > self.max_pixels):
                    break
                waiting.popleft()
                r = spr.Render(self.vols[q.vol], q.cam, q.iso, q.w, q.h, spec_cap=self.spec_cap)
                res = Result(i, q.t, clock() - t0, 0.0, 0, 0)
                active.append({"idx": i, "req": q, "render": r, "est": est, "last_done": q.t, "result": res})
                used += est
                pixels += q.w * q.h
                members_changed = True
            if not active:
                if pending:
                    dt = pending[0][1].t - (clock() - t0)
                    if dt > 0:
                        time.sleep(min(dt, 0.01))
                continue
            if members_changed:
                self.batch.set([a["render"] for a in active])
                members_changed = False
            max_active = max(max_active, len(active))
            self.batch.pass_()
            states, active_blocks = self.batch.state()
            done_t = clock() - t0
            passes += 1
            # estimates: the pass's active blocks shared out over its requests by
            # their active rays at the start of the pass (w*h before the first)
            start_rays = [a.get("rays", a["req"].w * a["req"].h) for a in active]
            tot = sum(start_rays) or 1
            per_vol = {}
            for a, n0 in zip(active, start_rays):
                v = a["req"].vol
                per_vol[v] = max(per_vol.get(v, 0.0), active_blocks * n0 / tot)
            for v, e in per_vol.items():
                self.per_request_blocks[v] = max(1.0, e)
            for a, s in zip(active, states):
                a["rays"] = s["n_active"]
                a["est"] = int(self.per_request_blocks[a["req"].vol])
            still = []
            for a, s in zip(active, states):
                lt = done_t - a["last_done"]
                a["result"].latencies.append(lt)
                lat.append(lt)
                a["last_done"] = done_t
                if s["n_active"] == 0:
                    res = a["result"]
                    res.finished = done_t
                    info = a["render"].info()
                    res.passes = info["passes"]
                    res.rays_entered = info["rays_entered"]
                    if keep_results:
                        res.hits = a["render"].hits()
                        res.image = a["render"].image()
                    results[a["idx"]] = res
                    members_changed = True
                else:
                    still.append(a)
            if members_changed:
                # finished members leave before their renders are freed
                self.batch.set([a["render"] for a in still])
                members_changed = False
                for a in active:
                    if a not in still:
                        a["render"].free()
            active = still
        span = clock() - t0
        lat_a = np.array(lat) if lat else np.zeros(1)
        rays = sum(r.rays_entered for r in results if r is not None)
        stats = {"requests": len(arrivals), "passes": passes, "makespan_s": span,
                 "rays_per_s": rays / span if span > 0 else 0.0,
                 "pass_latency_ms_p50": float(np.percentile(lat_a, 50) * 1e3),
                 "pass_latency_ms_p99": float(np.percentile(lat_a, 99) * 1e3),
                 "max_concurrent": max_active,
                 "request_latency_ms_p50": float(np.percentile([r.finished - r.arrival for r in results if r], 50) * 1e3)
                 if any(results) else 0.0}
        return results, stats

    def close(self):
        self.batch.free()
