"""Seeded synthetic inputs: scalar fields, the offline block encoder, cameras.

Everything here produces inputs for the renderer and for the oracle.  It holds
none of the rendering method's arithmetic (no decoder, no traversal, no
intersection); see ``volgen.c`` for the compressed-record format it writes.

The C part is compiled on first use (or by :func:`build`) into
``volgen/libvolgen.so`` with gcc + OpenMP.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "volgen.c")
_LIB = os.path.join(_HERE, "libvolgen.so")
_lib = None

F32, U8 = 0, 1


def build(force: bool = True) -> str:
    """Compile libvolgen.so (gcc, OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.vg_blobs.argtypes = [ctypes.c_int] * 3 + [ctypes.c_uint64, ctypes.c_int, P]
        lib.vg_fourier.argtypes = [ctypes.c_int] * 3 + [ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                                        ctypes.c_double, P]
        lib.vg_analytic.argtypes = [ctypes.c_int] * 4 + [P, P]
        lib.vg_quantize_u8.argtypes = [P, ctypes.c_size_t, ctypes.c_float, ctypes.c_float]
        lib.vg_kth_value.argtypes = [P, ctypes.c_size_t, ctypes.c_size_t, P]
        lib.vg_encode.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P]
        lib.vg_encode_block.argtypes = [P, ctypes.c_int, P]
        lib.vg_rm_field.argtypes = [ctypes.c_int] * 3 + [ctypes.c_uint64, ctypes.c_double, P]
        lib.vg_rm_encode.argtypes = [ctypes.c_int] * 3 + [ctypes.c_uint64, ctypes.c_double, ctypes.c_int, P]
        lib.vg_splitmix64.argtypes = [ctypes.POINTER(ctypes.c_uint64)]
        lib.vg_splitmix64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"volgen.{what} failed with status {rc}")


# ------------------------------------------------------------------ fields --

def blobs(nx: int, ny: int, nz: int, seed: int, nblob: int = 8) -> np.ndarray:
    out = np.empty((nz, ny, nx), np.float32)
    _check(_load().vg_blobs(nx, ny, nz, seed, nblob, _ptr(out)), "blobs")
    return out


def fourier(nx: int, ny: int, nz: int, seed: int, nmode: int = 64, kmax: int = 24,
            period: float | None = None) -> np.ndarray:
    out = np.empty((nz, ny, nx), np.float32)
    per = float(period if period is not None else max(nx, ny, nz))
    _check(_load().vg_fourier(nx, ny, nz, seed, nmode, kmax, per, _ptr(out)), "fourier")
    return out


def analytic(nx: int, ny: int, nz: int, kind: str, params) -> np.ndarray:
    k = {"plane": 0, "product": 1, "sphere": 2}[kind]
    p = np.zeros(4, np.float64)
    p[: len(params)] = params
    out = np.empty((nz, ny, nx), np.float32)
    _check(_load().vg_analytic(nx, ny, nz, k, _ptr(p), _ptr(out)), "analytic")
    return out


def rm_field(nx: int, ny: int, nz: int, seed: int = 3, hsum: float = 120.0) -> np.ndarray:
    """RM-like mixing-layer field, values 0..255 as float32 (small sizes)."""
    out = np.empty((nz, ny, nx), np.float32)
    _check(_load().vg_rm_field(nx, ny, nz, seed, hsum, _ptr(out)), "rm_field")
    return out


def rm_encode(nx: int, ny: int, nz: int, rate: int, seed: int = 3, hsum: float = 120.0) -> np.ndarray:
    """Generate and compress the RM-like field block by block (no full buffer)."""
    out = np.zeros(stream_bytes(nx, ny, nz, rate), np.uint8)
    _check(_load().vg_rm_encode(nx, ny, nz, seed, hsum, rate, _ptr(out)), "rm_encode")
    return out


def quantize_u8(vol: np.ndarray, lo: float, hi: float) -> np.ndarray:
    v = np.ascontiguousarray(vol, np.float32).copy()
    _check(_load().vg_quantize_u8(_ptr(v), v.size, lo, hi), "quantize_u8")
    return v


def kth_value(vol: np.ndarray, k: int) -> float:
    v = np.ascontiguousarray(vol, np.float32)
    out = np.zeros(1, np.float32)
    _check(_load().vg_kth_value(_ptr(v), v.size, int(k), _ptr(out)), "kth_value")
    return float(out[0])


def percentile_value(vol: np.ndarray, frac: float) -> float:
    """Exact order statistic at index floor(frac*(N-1)) of the field values."""
    n = vol.size
    return kth_value(vol, int(math.floor(frac * (n - 1))))


# ----------------------------------------------------------------- encoder --

def n_blocks(nx: int, ny: int, nz: int) -> int:
    return ((nx + 3) // 4) * ((ny + 3) // 4) * ((nz + 3) // 4)


def stream_bytes(nx: int, ny: int, nz: int, rate: int) -> int:
    return n_blocks(nx, ny, nz) * 8 * rate


def encode(vol: np.ndarray, rate: int) -> np.ndarray:
    """Compress a (nz, ny, nx) float32 field; returns the stream as uint8."""
    v = np.ascontiguousarray(vol, np.float32)
    nz, ny, nx = v.shape
    out = np.zeros(stream_bytes(nx, ny, nz, rate), np.uint8)
    _check(_load().vg_encode(_ptr(v), nx, ny, nz, rate, _ptr(out)), "encode")
    return out


def encode_block(v64, rate: int) -> np.ndarray:
    v = np.ascontiguousarray(np.asarray(v64, np.float32).reshape(64))
    out = np.zeros(8 * rate, np.uint8)
    _check(_load().vg_encode_block(_ptr(v), rate, _ptr(out)), "encode_block")
    return out


# ------------------------------------------------------------------ camera --

@dataclass
class Camera:
    eye: tuple
    center: tuple
    up: tuple
    vfov_deg: float = 45.0


def splitmix_stream(seed: int):
    st = ctypes.c_uint64(seed)
    lib = _load()
    while True:
        yield lib.vg_splitmix64(ctypes.byref(st))


def _unit(gen) -> float:
    return (next(gen) >> 11) * (1.0 / 9007199254740992.0)


def orbit_camera(nx: int, ny: int, nz: int, seed: int, k: int = 0, npos: int = 1,
                 vfov_deg: float = 45.0, dist_scale: float = 2.0) -> Camera:
    """Seeded orbit camera looking at the volume centre, up = +z.

    Azimuth phi0 + 2 pi k / npos with phi0 ~ U[0, 2 pi), elevation
    U[-60, 60] degrees, distance dist_scale x the half-diagonal of the
    sample domain [0, n-1]^3."""
    g = splitmix_stream(seed)
    phi0 = 2.0 * math.pi * _unit(g)
    elev = math.radians(-60.0 + 120.0 * _unit(g))
    az = phi0 + 2.0 * math.pi * k / max(npos, 1)
    c = ((nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0)
    half_diag = 0.5 * math.sqrt((nx - 1) ** 2 + (ny - 1) ** 2 + (nz - 1) ** 2)
    d = dist_scale * half_diag
    eye = (c[0] + d * math.cos(elev) * math.cos(az),
           c[1] + d * math.cos(elev) * math.sin(az),
           c[2] + d * math.sin(elev))
    return Camera(eye=eye, center=c, up=(0.0, 0.0, 1.0), vfov_deg=vfov_deg)


def uniform(seed: int, n: int):
    """n uniform doubles in [0,1) from SplitMix64 (host-side sampling helper)."""
    g = splitmix_stream(seed)
    return [_unit(g) for _ in range(n)]
