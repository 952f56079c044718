"""Seeded workload recipes built from volgen's fields: the batched pool and
request mix, and the serving arrival stream.  Inputs only: nothing here
renders or decodes.

Batched (B): a pool of 8 volumes - Gaussian blobs and Fourier fields at
128^3, 256^3, 512^3 and 1024^3 (blob widths scaled by n/64) - each stored as
float32 or as u8 levels (quantised to 0..255 over the field's range, then
compressed as float32 values), at 2, 4 or 8 bits/value (in turn along the
pool, so every rate appears); 64 requests (seeds
1000+i), each picking a pool volume, an image size from {256^2, 512^2,
640x360, 1280x720, 1920x1080}, an isovalue uniform in [p10, p90] of that
volume's values, and a seeded orbit camera.

Serving (S): Poisson arrivals at rate lam over a time span; each request is an
orbit step (70%) or an isovalue change (30%) on one of the resident volumes,
at 1280x720 or 1920x1080 (50/50).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import Camera, blobs, encode, fourier, orbit_camera, percentile_value, quantize_u8, splitmix_stream

POOL_KINDS = [("blobs", 128), ("blobs", 256), ("blobs", 512), ("blobs", 1024),
              ("fourier", 128), ("fourier", 256), ("fourier", 512), ("fourier", 1024)]
IMAGE_SIZES = [(256, 256), (512, 512), (640, 360), (1280, 720), (1920, 1080)]


@dataclass
class PoolVolume:
    name: str
    kind: str
    dims: tuple
    dtype: str           # "f32" or "u8"
    rate: int
    stream: np.ndarray = field(repr=False)
    p10: float = 0.0
    p90: float = 0.0


@dataclass
class Request:
    vol: int             # index into the pool
    w: int
    h: int
    iso: float
    cam: Camera
    seed: int


def _u(g) -> float:
    return (next(g) >> 11) * (1.0 / 9007199254740992.0)


def make_pool(sizes=(128, 256, 512, 1024), seed: int = 11) -> list[PoolVolume]:
    """The batched pool (subset of sizes for smaller runs); deterministic per seed."""
    g = splitmix_stream(seed)
    pool = []
    for i, (kind, n) in enumerate(POOL_KINDS):
        dtype = "u8" if next(g) & 1 else "f32"
        next(g)                      # (the draw that used to pick the rate; kept so dtypes stay put)
        rate = (2, 4, 8)[i % 3]      # every rate of the mix, 2 bits/value included, at every pool size subset
        if n not in sizes:
            continue
        fseed = 100 + i
        if kind == "blobs":
            f = blobs(n, n, n, seed=fseed)
        else:
            f = fourier(n, n, n, seed=fseed, nmode=64, kmax=24, period=float(n))
        if dtype == "u8":
            f = quantize_u8(f, float(f.min()), float(f.max()))
        p10 = percentile_value(f, 0.1)
        p90 = percentile_value(f, 0.9)
        s = encode(f, rate)
        del f
        pool.append(PoolVolume(f"{kind}{n}_{dtype}_r{rate}", kind, (n, n, n), dtype, rate, s, p10, p90))
    return pool


def make_requests(pool: list[PoolVolume], count: int = 64, seed0: int = 1000,
                  sizes=IMAGE_SIZES) -> list[Request]:
    reqs = []
    for i in range(count):
        g = splitmix_stream(seed0 + i)
        v = next(g) % len(pool)
        w, h = sizes[next(g) % len(sizes)]
        pv = pool[v]
        iso = pv.p10 + (pv.p90 - pv.p10) * _u(g)
        nx, ny, nz = pv.dims
        cam = orbit_camera(nx, ny, nz, seed=seed0 + i)
        reqs.append(Request(v, w, h, float(iso), cam, seed0 + i))
    return reqs


@dataclass
class Arrival:
    t: float             # seconds from the start
    vol: int
    w: int
    h: int
    iso: float
    cam: Camera
    kind: str            # "orbit" or "iso"


def serving_arrivals(vols, isos, lam: float = 200.0, span_s: float = 30.0, seed: int = 7) -> list[Arrival]:
    """Poisson arrivals over [0, span_s): vols = list of dims, isos = per-volume
    (p_lo, p_hi) isovalue range.  Each volume keeps an orbit position and an
    isovalue; an orbit request advances the camera one of 10 orbit steps, an
    isovalue request draws a new isovalue in the range."""
    g = splitmix_stream(seed)
    t = 0.0
    state = []
    for k, (lo, hi) in enumerate(isos):
        state.append({"step": 0, "iso": lo + 0.5 * (hi - lo)})
    out = []
    while True:
        t += -math.log(1.0 - _u(g)) / lam
        if t >= span_s:
            break
        v = next(g) % len(vols)
        orbit = _u(g) < 0.7
        w, h = (1280, 720) if _u(g) < 0.5 else (1920, 1080)
        st = state[v]
        if orbit:
            st["step"] = (st["step"] + 1) % 10
        else:
            lo, hi = isos[v]
            st["iso"] = lo + (hi - lo) * _u(g)
        nx, ny, nz = vols[v]
        cam = orbit_camera(nx, ny, nz, seed=20 + v, k=st["step"], npos=10)
        out.append(Arrival(t, v, w, h, float(st["iso"]), cam, "orbit" if orbit else "iso"))
    return out
