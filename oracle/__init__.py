"""CPU oracle for speculative progressive isosurface raycasting (arXiv 2309.10212).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links or
runs anything here, and this package shares no code with it.

The arithmetic lives in ``oracle.c`` (plain C, fp64, OpenMP over pixels); this
module compiles it with gcc (no FMA contraction, no fast-math) and wraps it
with ctypes.  Each wrapper names the paper section it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None
NONE = 0xFFFFFFFF


class _Cam(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("center", ctypes.c_double * 3),
                ("up", ctypes.c_double * 3), ("vfov_deg", ctypes.c_double)]


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc -O2 -fopenmp -ffp-contract=off."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i = ctypes.c_int
        lib.orc_decode_block.argtypes = [P, i, P]
        lib.orc_decode_blocks.argtypes = [P, ctypes.c_size_t, i, i, i, i, P, ctypes.c_size_t, P]
        lib.orc_decode_volume.argtypes = [P, ctypes.c_size_t, i, i, i, i, P]
        lib.orc_grids.argtypes = [P, i, i, i, P, P, P]
        lib.orc_render.argtypes = [P, i, i, i, ctypes.POINTER(_Cam), ctypes.c_float, i, i, P,
                                   ctypes.c_size_t, P, P, P, P, P]
        lib.orc_cell_walk.argtypes = [i, i, i, ctypes.POINTER(_Cam), i, i, i, i, P, P, ctypes.c_long, P]
        lib.orc_cell_walk.restype = ctypes.c_long
        lib.orc_ray.argtypes = [i, i, i, ctypes.POINTER(_Cam), i, i, i, i, P]
        lib.orc_nspec.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        lib.orc_nspec.restype = ctypes.c_uint32
        lib.orc_schedule.argtypes = [P, i, i, i, ctypes.POINTER(_Cam), ctypes.c_float, i, i,
                                     ctypes.c_uint32, ctypes.c_long, P]
        lib.orc_schedule.restype = ctypes.c_long
        lib.orc_schedule_lists.argtypes = [ctypes.c_uint64, ctypes.c_size_t, P, P, P, P, ctypes.c_long,
                                           ctypes.c_long, ctypes.c_long, ctypes.c_uint32, ctypes.c_long, P]
        lib.orc_schedule_lists.restype = ctypes.c_long
        lib.orc_schedule_policy.argtypes = [P, i, i, i, ctypes.POINTER(_Cam), ctypes.c_float, i, i,
                                            ctypes.c_uint32, ctypes.c_uint32, ctypes.c_long, P]
        lib.orc_schedule_policy.restype = ctypes.c_long
        lib.orc_schedule_lists_policy.argtypes = [ctypes.c_uint64, ctypes.c_size_t, P, P, P, P, P, P, ctypes.c_long,
                                                  ctypes.c_long, ctypes.c_long, ctypes.c_uint32, ctypes.c_uint32,
                                                  ctypes.c_long, P]
        lib.orc_schedule_lists_policy.restype = ctypes.c_long
        lib.orc_pixel_candidates.argtypes = [P, i, i, i, ctypes.POINTER(_Cam), ctypes.c_float, i, i, i, i, P, P,
                                             ctypes.c_long, P, P]
        lib.orc_pixel_candidates.restype = ctypes.c_long
        lib.orc_ray_weight.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.orc_ray_weight.restype = ctypes.c_uint32
        lib.orc_nspec_ray.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32,
                                      ctypes.c_uint32]
        lib.orc_nspec_ray.restype = ctypes.c_uint32
        lib.orc_render_stream.argtypes = [P, ctypes.c_size_t, i, i, i, i, ctypes.POINTER(_Cam), ctypes.c_float,
                                          i, i, P, ctypes.c_size_t, P, P, P, P, P]
        lib.orc_block_ranges_stream.argtypes = [P, ctypes.c_size_t, i, i, i, i, P]
        lib.orc_grids_from_blocks.argtypes = [P, i, i, i, P, P]
        lib.orc_blocks_containing.argtypes = [P, ctypes.c_size_t, ctypes.c_float]
        lib.orc_blocks_containing.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _p(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _cam(cam) -> _Cam:
    c = _Cam()
    c.eye[:] = [float(v) for v in cam.eye]
    c.center[:] = [float(v) for v in cam.center]
    c.up[:] = [float(v) for v in cam.up]
    c.vfov_deg = float(cam.vfov_deg)
    return c


def _ok(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle.{what} failed with status {rc}")


def _dims(vol: np.ndarray):
    nz, ny, nx = vol.shape
    return nx, ny, nz


# ---------------------------------------------------------------- codec -----

def decode_block(rec: np.ndarray, rate: int) -> np.ndarray:
    """One block record -> 64 floats (fixed-rate block decompression, Sec. 3.5)."""
    r = np.ascontiguousarray(np.frombuffer(np.asarray(rec, np.uint8).tobytes(), np.uint32))
    out = np.empty(64, np.float32)
    _ok(_load().orc_decode_block(_p(r), rate, _p(out)), "decode_block")
    return out


def decode_blocks(stream: np.ndarray, dims, rate: int, ids) -> np.ndarray:
    nx, ny, nz = dims
    s = np.ascontiguousarray(stream, np.uint8)
    ids = np.ascontiguousarray(ids, np.uint32)
    out = np.empty((len(ids), 64), np.float32)
    _ok(_load().orc_decode_blocks(_p(s), s.nbytes, nx, ny, nz, rate, _p(ids), len(ids), _p(out)),
        "decode_blocks")
    return out


def decode_volume(stream: np.ndarray, dims, rate: int) -> np.ndarray:
    """Whole-volume decompression -> (nz, ny, nx) float32."""
    nx, ny, nz = dims
    s = np.ascontiguousarray(stream, np.uint8)
    out = np.empty((nz, ny, nx), np.float32)
    _ok(_load().orc_decode_volume(_p(s), s.nbytes, nx, ny, nz, rate, _p(out)), "decode_volume")
    return out


# ---------------------------------------------------------------- grids -----

def grids(vol: np.ndarray):
    """(block, fine, coarse) ranges as (N, 2) float32 arrays (Sec. 3.1)."""
    nx, ny, nz = _dims(vol)
    nbx, nby, nbz = (nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4
    ncx, ncy, ncz = (nbx + 3) // 4, (nby + 3) // 4, (nbz + 3) // 4
    v = np.ascontiguousarray(vol, np.float32)
    blk = np.empty((nbx * nby * nbz, 2), np.float32)
    fin = np.empty_like(blk)
    crs = np.empty((ncx * ncy * ncz, 2), np.float32)
    _ok(_load().orc_grids(_p(v), nx, ny, nz, _p(blk), _p(fin), _p(crs)), "grids")
    return blk, fin, crs


# -------------------------------------------------------------- render ------

def render(vol: np.ndarray, cam, iso: float, w: int, h: int, pixels=None):
    """First-hit isosurface per pixel by marching every dual cell (Sec. 3.3-3.7).

    Returns dict of arrays t (f64, inf = no hit), block, cell, rgba (u32) and
    entered (bool: the ray entered the volume)."""
    nx, ny, nz = _dims(vol)
    v = np.ascontiguousarray(vol, np.float32)
    if pixels is None:
        n = w * h
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, np.uint32)
        n = len(pix)
    t = np.empty(n, np.float64)
    b = np.empty(n, np.uint32)
    c = np.empty(n, np.uint32)
    rgba = np.empty(n, np.uint32)
    ent = np.empty(n, np.uint8)
    cc = _cam(cam)
    _ok(_load().orc_render(_p(v), nx, ny, nz, ctypes.byref(cc), ctypes.c_float(iso), w, h,
                           _p(pix) if pix is not None else None, n, _p(t), _p(b), _p(c), _p(rgba), _p(ent)),
        "render")
    return {"t": t, "block": b, "cell": c, "rgba": rgba, "entered": ent.astype(bool)}


def render_stream(stream: np.ndarray, dims, rate: int, cam, iso: float, w: int, h: int, pixels=None):
    """render() for a volume given as its compressed stream: the same march, with
    each corner read from its block decoded on demand (volumes too large to
    decode whole; sampled pixels)."""
    nx, ny, nz = dims
    s = np.ascontiguousarray(stream, np.uint8)
    if pixels is None:
        n = w * h
        pix = None
    else:
        pix = np.ascontiguousarray(pixels, np.uint32)
        n = len(pix)
    t = np.empty(n, np.float64)
    b = np.empty(n, np.uint32)
    c = np.empty(n, np.uint32)
    rgba = np.empty(n, np.uint32)
    ent = np.empty(n, np.uint8)
    cc = _cam(cam)
    _ok(_load().orc_render_stream(_p(s), s.nbytes, nx, ny, nz, rate, ctypes.byref(cc), ctypes.c_float(iso), w, h,
                                  _p(pix) if pix is not None else None, n, _p(t), _p(b), _p(c), _p(rgba), _p(ent)),
        "render_stream")
    return {"t": t, "block": b, "cell": c, "rgba": rgba, "entered": ent.astype(bool)}


def block_ranges_stream(stream: np.ndarray, dims, rate: int) -> np.ndarray:
    """Per-block (min, max) over the samples inside the volume, decoding one
    block at a time from the stream (the block ranges of grids())."""
    nx, ny, nz = dims
    s = np.ascontiguousarray(stream, np.uint8)
    nb = ((nx + 3) // 4) * ((ny + 3) // 4) * ((nz + 3) // 4)
    out = np.empty((nb, 2), np.float32)
    _ok(_load().orc_block_ranges_stream(_p(s), s.nbytes, nx, ny, nz, rate, _p(out)), "block_ranges_stream")
    return out


def grids_from_blocks(block: np.ndarray, dims):
    """(fine, coarse) ranges from block ranges, as grids() builds them."""
    nx, ny, nz = dims
    blk = np.ascontiguousarray(block, np.float32)
    nbx, nby, nbz = (nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4
    nc = ((nbx + 3) // 4) * ((nby + 3) // 4) * ((nbz + 3) // 4)
    fine = np.empty((nbx * nby * nbz, 2), np.float32)
    coarse = np.empty((nc, 2), np.float32)
    _ok(_load().orc_grids_from_blocks(_p(blk), nx, ny, nz, _p(fine), _p(coarse)), "grids_from_blocks")
    return fine, coarse


def cell_walk(dims, cam, w: int, h: int, px: int, py: int, cap: int = 1 << 16):
    """Ordered dual cells (x,y,z) and [t0,t1] along one pixel's ray; None on a miss."""
    nx, ny, nz = dims
    cells = np.empty((cap, 3), np.int32)
    t01 = np.empty((cap, 2), np.float64)
    te = np.empty(2, np.float64)
    cc = _cam(cam)
    n = _load().orc_cell_walk(nx, ny, nz, ctypes.byref(cc), w, h, px, py, _p(cells), _p(t01), cap, _p(te))
    if n == -1:
        return None
    if n < 0:
        raise RuntimeError("oracle.cell_walk: invalid camera")
    if n > cap:
        raise RuntimeError("oracle.cell_walk: cap too small")
    return cells[:n].copy(), t01[:n].copy(), (float(te[0]), float(te[1]))


def ray(dims, cam, w: int, h: int, px: int, py: int):
    """(direction, t_enter, t_exit, entered) of one pixel's ray (Sec. 3.2)."""
    nx, ny, nz = dims
    out = np.empty(6, np.float64)
    cc = _cam(cam)
    _ok(_load().orc_ray(nx, ny, nz, ctypes.byref(cc), w, h, px, py, _p(out)), "ray")
    return out[:3].copy(), float(out[3]), float(out[4]), bool(out[5])


def nspec(slots: int, n_act: int, cap: int = 64) -> int:
    """N_spec = floor(w*h / N_act), at least 1, at most cap (Sec. 4)."""
    return int(_load().orc_nspec(slots, n_act, cap))


SCHED_FIELDS = ("n_active", "n_spec", "pairs", "visible", "active_blocks", "terminated", "slots", "wsum")
POLICY_UNIFORM, POLICY_PER_RAY = 0, 1


def ray_weight(t: float, t_exit: float) -> int:
    """Weight of a ray whose remaining walk starts at t (per-ray speculation)."""
    return int(_load().orc_ray_weight(ctypes.c_double(t), ctypes.c_double(t_exit)))


def pixel_candidates(vol: np.ndarray, cam, iso: float, w: int, h: int, px: int, py: int, cap: int = 1 << 16):
    """(candidate blocks, weight after each, weight before the first, first-hit index) of one pixel."""
    nx, ny, nz = _dims(vol)
    v = np.ascontiguousarray(vol, np.float32)
    lst = np.zeros(cap, np.uint32)
    wl = np.zeros(cap, np.uint32)
    hit = np.zeros(1, np.int64)
    w0 = np.zeros(1, np.uint32)
    cc = _cam(cam)
    n = _load().orc_pixel_candidates(_p(v), nx, ny, nz, ctypes.byref(cc), ctypes.c_float(iso), w, h, px, py,
                                     _p(lst), _p(wl), cap, _p(hit), _p(w0))
    if n < 0:
        raise RuntimeError(f"oracle.pixel_candidates failed with status {n}")
    return lst[:n].copy(), wl[:n].copy(), int(w0[0]), int(hit[0])


def nspec_ray(slots: int, n_act: int, wsum: int, w: int, cap: int = 64) -> int:
    """Per-ray count min(cap, 1 + floor((slots - n_act) * w / wsum))."""
    return int(_load().orc_nspec_ray(slots, n_act, wsum, w, cap))


def schedule(vol: np.ndarray, cam, iso: float, w: int, h: int, spec_cap: int, max_pass: int = 100000,
             policy: int = POLICY_UNIFORM):
    """Per-pass counters of the progressive speculative passes (Sec. 3, Sec. 4;
    policy 1: per-ray speculation counts)."""
    nx, ny, nz = _dims(vol)
    v = np.ascontiguousarray(vol, np.float32)
    st = np.zeros((max_pass, 8), np.uint64)
    cc = _cam(cam)
    n = _load().orc_schedule_policy(_p(v), nx, ny, nz, ctypes.byref(cc), ctypes.c_float(iso), w, h, spec_cap,
                                    policy, max_pass, _p(st))
    if n < 0:
        raise RuntimeError(f"oracle.schedule failed with status {n}")
    return [dict(zip(SCHED_FIELDS, (int(x) for x in row))) for row in st[:n]]


def schedule_lists(slots: int, lists, hit_idx, entered, nb_dims, spec_cap: int,
                   max_pass: int = 100000, policy: int = POLICY_UNIFORM, w0=None, wk=None):
    """Pass schedule (Sec. 3, Sec. 4) from explicit per-ray candidate-block lists.

    lists[i]: ordered candidate block ids of ray i; hit_idx[i]: index in it of
    the block holding the first hit, or -1; entered[i]: ray entered the volume.
    policy 1 (per-ray counts) takes each ray's weight before its first
    candidate (w0[i]) and after each candidate k (wk[i][k])."""
    n = len(lists)
    off = np.zeros(n + 1, np.uint64)
    for i, l in enumerate(lists):
        off[i + 1] = off[i] + len(l)
    flat = np.ascontiguousarray(np.concatenate([np.asarray(l, np.uint32) for l in lists])
                                if n and off[-1] else np.zeros(1, np.uint32), np.uint32)
    hit = np.ascontiguousarray(hit_idx, np.int64)
    ent = np.ascontiguousarray(entered, np.uint8)
    st = np.zeros((max_pass, 8), np.uint64)
    nbx, nby, nbz = nb_dims
    if policy == POLICY_PER_RAY:
        w0a = np.ascontiguousarray(w0, np.uint32)
        wka = np.ascontiguousarray(np.concatenate([np.asarray(x, np.uint32) for x in wk])
                                   if n and off[-1] else np.zeros(1, np.uint32), np.uint32)
        pw0, pwk = _p(w0a), _p(wka)
    else:
        pw0 = pwk = None
    r = _load().orc_schedule_lists_policy(slots, n, _p(off), _p(flat), _p(hit), _p(ent), pw0, pwk, nbx, nby, nbz,
                                          spec_cap, policy, max_pass, _p(st))
    if r < 0:
        raise RuntimeError(f"oracle.schedule_lists failed with status {r}")
    return [dict(zip(SCHED_FIELDS, (int(x) for x in row))) for row in st[:r]]


def blocks_containing(fine: np.ndarray, iso: float) -> int:
    f = np.ascontiguousarray(fine, np.float32)
    return int(_load().orc_blocks_containing(_p(f), f.shape[0], ctypes.c_float(iso)))
