"""ctypes binding of libspr (include/spr.h): argument marshalling only.

Every step of the rendering path runs in the HIP kernels of libspr.so; this
module converts arguments, owns handles, and plugs torch's caching allocator
and current stream into the library.  If the shared library is missing the
import fails: there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspr.so")

SPR_OK = 0
ERRORS = {-1: "SPR_E_INVALID", -2: "SPR_E_OOM", -3: "SPR_E_HIP", -4: "SPR_E_CORRUPT", -5: "SPR_E_CAPACITY",
          -6: "SPR_E_STATE", -7: "SPR_E_UNIMPLEMENTED"}
NONE = 0xFFFFFFFF
DTYPE_F32, DTYPE_U8 = 0, 1
CODEC_VERSION = 1
NOALLOC_MAX_BLOCKS = 16384   # SPR_NOALLOC_MAX_BLOCKS
MAX_EXTENT = 524288          # SPR_MAX_EXTENT: samples per volume axis, and bound on each eye coordinate
SPEC_UNIFORM, SPEC_PER_RAY = 0, 1


class SprError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {ERRORS.get(status, status)}: {msg}")
        self.status = status


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class _Allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class _Config(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("stream", ctypes.c_void_p), ("cache_bytes", ctypes.c_size_t),
                ("spec_cap", ctypes.c_uint32), ("flags", ctypes.c_uint32), ("alloc", _Allocator)]


class _VolumeDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_uint32), ("ny", ctypes.c_uint32), ("nz", ctypes.c_uint32),
                ("rate_bits", ctypes.c_uint32), ("src_dtype", ctypes.c_uint32), ("codec_version", ctypes.c_uint32)]


class _Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("center", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("vfov_deg", ctypes.c_double)]


class PassStats(ctypes.Structure):
    _fields_ = [("pass_", ctypes.c_uint32), ("n_active", ctypes.c_uint32), ("n_spec", ctypes.c_uint32),
                ("pairs", ctypes.c_uint32), ("visible_blocks", ctypes.c_uint32), ("active_blocks", ctypes.c_uint32),
                ("blocks_decoded", ctypes.c_uint32), ("deferred_pairs", ctypes.c_uint32),
                ("terminated", ctypes.c_uint32), ("slots", ctypes.c_uint32), ("utilization", ctypes.c_double),
                ("ms", ctypes.c_float), ("pad", ctypes.c_float)]

    def as_dict(self):
        return {"pass": self.pass_, "n_active": self.n_active, "n_spec": self.n_spec, "pairs": self.pairs,
                "visible": self.visible_blocks, "active_blocks": self.active_blocks,
                "blocks_decoded": self.blocks_decoded, "deferred": self.deferred_pairs,
                "terminated": self.terminated, "slots": self.slots, "utilization": self.utilization, "ms": self.ms}


class Counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_uint64) for n in ("passes", "blocks_decoded", "visible_blocks", "active_blocks",
                                               "pairs", "evicted", "overflow", "rays", "pair_slots",
                                               "served_pairs", "max_active_blocks", "walk_guard", "coarse_steps", "coarse_masks")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class RenderInfo(ctypes.Structure):
    _fields_ = [("w", ctypes.c_uint32), ("h", ctypes.c_uint32), ("rays_entered", ctypes.c_uint32),
                ("n_active", ctypes.c_uint32), ("n_spec", ctypes.c_uint32), ("passes", ctypes.c_uint32),
                ("pairs", ctypes.c_uint64), ("bcmc_blocks", ctypes.c_uint64), ("iso_coarse_cells", ctypes.c_uint64),
                ("masks_built", ctypes.c_uint32)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


MEM_KINDS = ("compressed", "grids", "rays", "cache", "scratch")


class MemSplit(ctypes.Structure):
    _fields_ = [("current", ctypes.c_size_t * 5), ("at_peak", ctypes.c_size_t * 5), ("kind_peak", ctypes.c_size_t * 5),
                ("total", ctypes.c_size_t), ("peak", ctypes.c_size_t)]

    def as_dict(self):
        return {"current": dict(zip(MEM_KINDS, self.current)), "at_peak": dict(zip(MEM_KINDS, self.at_peak)),
                "kind_peak": dict(zip(MEM_KINDS, self.kind_peak)), "total": self.total, "peak": self.peak}


class Tuning(ctypes.Structure):
    _fields_ = [("pairs_per_wg", ctypes.c_uint32), ("slot_tile", ctypes.c_uint32)]


class MemberState(ctypes.Structure):
    _fields_ = [("n_active", ctypes.c_uint32), ("passes", ctypes.c_uint32), ("last_pairs", ctypes.c_uint32),
                ("n_spec", ctypes.c_uint32)]


class KernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("total_ms", ctypes.c_double), ("launches", ctypes.c_uint64)]


HIT_DTYPE = np.dtype([("t", np.float64), ("block", np.uint32), ("cell", np.uint32)])

# (name, restype, argtypes) of every exported call, in header order
_P = ctypes.c_void_p
_U32 = ctypes.c_uint32
_ST = ctypes.c_int32
SIGNATURES = [
    ("spr_ctx_create", _ST, [ctypes.POINTER(_Config), ctypes.POINTER(_P)]),
    ("spr_ctx_destroy", _ST, [_P]),
    ("spr_mem_stats", _ST, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
    ("spr_mem_split_get", _ST, [_P, ctypes.POINTER(MemSplit), ctypes.c_int]),
    ("spr_ctx_counters", _ST, [_P, ctypes.POINTER(Counters)]),
    ("spr_ctx_profile", _ST, [_P, ctypes.c_int, ctypes.c_int]),
    ("spr_ctx_kernel_times", _ST, [_P, ctypes.POINTER(KernelTime), _U32, ctypes.POINTER(_U32)]),
    ("spr_ctx_set_tuning", _ST, [_P, ctypes.POINTER(Tuning)]),
    ("spr_ctx_get_tuning", _ST, [_P, ctypes.POINTER(Tuning)]),
    ("spr_volume_load", _ST, [_P, _P, ctypes.c_size_t, ctypes.POINTER(_VolumeDesc), ctypes.POINTER(_P)]),
    ("spr_volume_free", _ST, [_P]),
    ("spr_volume_build_grids", _ST, [_P]),
    ("spr_volume_ranges", _ST, [_P, _P, ctypes.c_size_t, _P, ctypes.c_size_t]),
    ("spr_debug_decode_blocks", _ST, [_P, _P, _U32, _P]),
    ("spr_debug_decode_blocks_noalloc", _ST, [_P, _P, _U32, _P]),
    ("spr_debug_fp64_ops", _ST, [_P, _P, _P, ctypes.c_size_t, _P, _P]),
    ("spr_render_begin", _ST, [_P, ctypes.POINTER(_Camera), ctypes.c_float, _U32, _U32, ctypes.POINTER(_P)]),
    ("spr_render_set_spec_cap", _ST, [_P, _U32]),
    ("spr_render_set_spec_policy", _ST, [_P, _U32]),
    ("spr_render_pass", _ST, [_P, ctypes.POINTER(PassStats)]),
    ("spr_render_done", _ST, [_P, ctypes.POINTER(ctypes.c_int)]),
    ("spr_render_run", _ST, [_P, _U32, ctypes.POINTER(_U32)]),
    ("spr_render_get_info", _ST, [_P, ctypes.POINTER(RenderInfo)]),
    ("spr_read_image", _ST, [_P, _P, ctypes.c_size_t]),
    ("spr_read_hits", _ST, [_P, _P, ctypes.c_size_t]),
    ("spr_render_device_ptrs", _ST, [_P, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    ("spr_render_free", _ST, [_P]),
    ("spr_batch_create", _ST, [_P, _U32, ctypes.POINTER(_P), ctypes.POINTER(_P)]),
    ("spr_batch_create_empty", _ST, [_P, _U32, ctypes.c_uint64, ctypes.POINTER(_P)]),
    ("spr_batch_set", _ST, [_P, _U32, ctypes.POINTER(_P)]),
    ("spr_batch_pass", _ST, [_P, ctypes.POINTER(_U32)]),
    ("spr_batch_run", _ST, [_P, _U32, _U32, ctypes.POINTER(_U32)]),
    ("spr_batch_state", _ST, [_P, ctypes.POINTER(MemberState), _U32, ctypes.POINTER(_U32)]),
    ("spr_batch_free", _ST, [_P]),
    ("spr_last_error", ctypes.c_char_p, []),
    ("spr_version", ctypes.c_char_p, []),
]

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libspr.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"libspr.so not built at {path}; run __graft_entry__.build()")
        lib = ctypes.CDLL(path)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _chk(st: int, where: str):
    if st != SPR_OK:
        raise SprError(st, where, load_library().spr_last_error().decode())


def _ptr(a: np.ndarray):
    return ctypes.c_void_p(a.ctypes.data)


@dataclass
class Camera:
    eye: tuple
    center: tuple
    up: tuple
    vfov_deg: float = 45.0


def _cam(c) -> _Camera:
    out = _Camera()
    out.eye[:] = [float(v) for v in c.eye]
    out.center[:] = [float(v) for v in c.center]
    out.up[:] = [float(v) for v in c.up]
    out.vfov_deg = float(c.vfov_deg)
    return out


class Context:
    """A device, a stream, a decoded-block cache (spr_ctx)."""

    def __init__(self, device: int = 0, cache_bytes: int = 512 * 10**6, spec_cap: int = 64, stream=None,
                 torch_allocator: bool = True, alloc_hooks=None):
        """alloc_hooks: optional (alloc(nbytes) -> int pointer or None, free(ptr, nbytes)) used
        instead of torch's caching allocator (tests count or fail allocations with it)."""
        import torch
        lib = load_library()
        self._torch = torch
        self.device = device
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        cfg = _Config()
        cfg.device = device
        cfg.stream = ctypes.c_void_p(stream.cuda_stream)
        cfg.cache_bytes = int(cache_bytes)
        cfg.spec_cap = int(spec_cap)
        cfg.flags = 0
        self._keep = []
        if alloc_hooks is not None:
            ha, hf = alloc_hooks

            def _alloc(nbytes, user):
                try:
                    return ha(int(nbytes))
                except Exception:
                    return None

            def _free(p, nbytes, user):
                hf(p, int(nbytes))

            fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
            self._keep += [fa, ff]
            cfg.alloc = _Allocator(fa, ff, None)
        elif torch_allocator:
            def _alloc(nbytes, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
                except Exception:
                    return None

            def _free(p, nbytes, user):
                torch.cuda.caching_allocator_delete(p)

            fa, ff = _ALLOC_FN(_alloc), _FREE_FN(_free)
            self._keep += [fa, ff]
            cfg.alloc = _Allocator(fa, ff, None)
        h = ctypes.c_void_p()
        _chk(lib.spr_ctx_create(ctypes.byref(cfg), ctypes.byref(h)), "spr_ctx_create")
        self.h = h
        self.cache_bytes = int(cache_bytes)

    def mem_stats(self):
        cur, peak = ctypes.c_size_t(), ctypes.c_size_t()
        _chk(load_library().spr_mem_stats(self.h, ctypes.byref(cur), ctypes.byref(peak)), "spr_mem_stats")
        return cur.value, peak.value

    def mem_split(self, reset_peak: bool = False):
        m = MemSplit()
        _chk(load_library().spr_mem_split_get(self.h, ctypes.byref(m), int(reset_peak)), "spr_mem_split_get")
        return m.as_dict()

    def counters(self):
        c = Counters()
        _chk(load_library().spr_ctx_counters(self.h, ctypes.byref(c)), "spr_ctx_counters")
        return c.as_dict()

    def profile(self, enable: bool, reset: bool = False):
        _chk(load_library().spr_ctx_profile(self.h, int(enable), int(reset)), "spr_ctx_profile")

    def set_tuning(self, pairs_per_wg: int, slot_tile: int):
        t = Tuning(pairs_per_wg, slot_tile)
        _chk(load_library().spr_ctx_set_tuning(self.h, ctypes.byref(t)), "spr_ctx_set_tuning")

    def tuning(self):
        t = Tuning()
        _chk(load_library().spr_ctx_get_tuning(self.h, ctypes.byref(t)), "spr_ctx_get_tuning")
        return {"pairs_per_wg": t.pairs_per_wg, "slot_tile": t.slot_tile}

    def kernel_times(self):
        arr = (KernelTime * 64)()
        n = ctypes.c_uint32()
        _chk(load_library().spr_ctx_kernel_times(self.h, arr, 64, ctypes.byref(n)), "spr_ctx_kernel_times")
        return {arr[i].name.decode(): (arr[i].total_ms, arr[i].launches) for i in range(n.value)}

    def fp64_ops(self, x: np.ndarray, y: np.ndarray):
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        sq = np.empty_like(x)
        dv = np.empty_like(x)
        _chk(load_library().spr_debug_fp64_ops(self.h, _ptr(x), _ptr(y), x.size, _ptr(sq), _ptr(dv)),
             "spr_debug_fp64_ops")
        return sq, dv

    def load_volume(self, stream: np.ndarray, dims, rate: int, src_dtype: int = DTYPE_F32,
                    codec_version: int = CODEC_VERSION) -> "Volume":
        return Volume(self, stream, dims, rate, src_dtype, codec_version)

    def close(self):
        if self.h:
            _chk(load_library().spr_ctx_destroy(self.h), "spr_ctx_destroy")
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Volume:
    """A compressed volume resident on the device with its macrocell grids."""

    def __init__(self, ctx: Context, stream: np.ndarray, dims, rate: int, src_dtype: int, codec_version: int):
        self.ctx = ctx
        self.dims = tuple(int(v) for v in dims)
        self.rate = rate
        s = np.ascontiguousarray(stream, np.uint8)
        d = _VolumeDesc(self.dims[0], self.dims[1], self.dims[2], rate, src_dtype, codec_version)
        h = ctypes.c_void_p()
        _chk(load_library().spr_volume_load(ctx.h, _ptr(s), s.nbytes, ctypes.byref(d), ctypes.byref(h)),
             "spr_volume_load")
        self.h = h
        nx, ny, nz = self.dims
        self.nb = ((nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4)
        self.nc = tuple((b + 3) // 4 for b in self.nb)
        self.nblocks = self.nb[0] * self.nb[1] * self.nb[2]

    def build_grids(self):
        _chk(load_library().spr_volume_build_grids(self.h), "spr_volume_build_grids")

    def ranges(self):
        fine = np.empty((self.nblocks, 2), np.float32)
        nc = self.nc[0] * self.nc[1] * self.nc[2]
        coarse = np.empty((nc, 2), np.float32)
        _chk(load_library().spr_volume_ranges(self.h, _ptr(fine), self.nblocks, _ptr(coarse), nc),
             "spr_volume_ranges")
        return fine, coarse

    def decode_blocks(self, ids) -> np.ndarray:
        ids = np.ascontiguousarray(ids, np.uint32)
        out = np.empty((len(ids), 64), np.float32)
        _chk(load_library().spr_debug_decode_blocks(self.h, _ptr(ids), len(ids), _ptr(out)),
             "spr_debug_decode_blocks")
        return out

    def decode_blocks_noalloc(self, ids) -> np.ndarray:
        """decode_blocks through the allocation-free entry point (at most
        NOALLOC_MAX_BLOCKS ids)."""
        ids = np.ascontiguousarray(ids, np.uint32)
        out = np.empty((len(ids), 64), np.float32)
        _chk(load_library().spr_debug_decode_blocks_noalloc(self.h, _ptr(ids), len(ids), _ptr(out)),
             "spr_debug_decode_blocks_noalloc")
        return out

    def free(self):
        if self.h:
            _chk(load_library().spr_volume_free(self.h), "spr_volume_free")
            self.h = None


class Render:
    """One camera/isovalue request rendered progressively (spr_render)."""

    def __init__(self, vol: Volume, cam, iso: float, w: int, h: int, spec_cap: int | None = None,
                 policy: int = 0):
        self.vol = vol
        self.w, self.h = int(w), int(h)
        c = _cam(cam)
        hh = ctypes.c_void_p()
        _chk(load_library().spr_render_begin(vol.h, ctypes.byref(c), ctypes.c_float(iso), self.w, self.h,
                                             ctypes.byref(hh)), "spr_render_begin")
        self.h_ = hh
        if spec_cap is not None:
            self.set_spec_cap(spec_cap)
        if policy:
            self.set_spec_policy(policy)

    def set_spec_policy(self, policy: int):
        """SPEC_UNIFORM (Sec. 4's single count) or SPEC_PER_RAY (per-ray counts)."""
        _chk(load_library().spr_render_set_spec_policy(self.h_, int(policy)), "spr_render_set_spec_policy")

    def set_spec_cap(self, cap: int):
        _chk(load_library().spr_render_set_spec_cap(self.h_, int(cap)), "spr_render_set_spec_cap")

    def pass_(self, stats: bool = False):
        if stats:
            s = PassStats()
            _chk(load_library().spr_render_pass(self.h_, ctypes.byref(s)), "spr_render_pass")
            return s.as_dict()
        _chk(load_library().spr_render_pass(self.h_, None), "spr_render_pass")
        return None

    def done(self) -> bool:
        d = ctypes.c_int()
        _chk(load_library().spr_render_done(self.h_, ctypes.byref(d)), "spr_render_done")
        return bool(d.value)

    def run(self, max_passes: int = 100000) -> int:
        n = ctypes.c_uint32()
        _chk(load_library().spr_render_run(self.h_, max_passes, ctypes.byref(n)), "spr_render_run")
        return n.value

    def info(self):
        i = RenderInfo()
        _chk(load_library().spr_render_get_info(self.h_, ctypes.byref(i)), "spr_render_get_info")
        return i.as_dict()

    def image(self) -> np.ndarray:
        out = np.empty((self.h, self.w, 4), np.uint8)
        _chk(load_library().spr_read_image(self.h_, _ptr(out), out.nbytes), "spr_read_image")
        return out

    def hits(self) -> np.ndarray:
        out = np.empty(self.w * self.h, HIT_DTYPE)
        _chk(load_library().spr_read_hits(self.h_, _ptr(out), out.size), "spr_read_hits")
        return out

    def device_ptrs(self):
        a, b = ctypes.c_void_p(), ctypes.c_void_p()
        _chk(load_library().spr_render_device_ptrs(self.h_, ctypes.byref(a), ctypes.byref(b)),
             "spr_render_device_ptrs")
        return a.value, b.value

    def free(self):
        if self.h_:
            _chk(load_library().spr_render_free(self.h_), "spr_render_free")
            self.h_ = None


class Batch:
    """Many renders advanced together, one captured pass per call (spr_batch).

    Batch(ctx, renders) fixes capacity to the given renders; Batch(ctx,
    max_requests=..., max_pixels=...) creates an empty batch whose members
    change with set() (continuous batching)."""

    def __init__(self, ctx: Context, renders=None, max_requests: int = 0, max_pixels: int = 0):
        self.ctx = ctx
        h = ctypes.c_void_p()
        if renders is not None:
            self.renders = list(renders)
            arr = (ctypes.c_void_p * len(self.renders))(*[r.h_ for r in self.renders])
            _chk(load_library().spr_batch_create(ctx.h, len(self.renders), arr, ctypes.byref(h)),
                 "spr_batch_create")
        else:
            self.renders = []
            _chk(load_library().spr_batch_create_empty(ctx.h, max_requests, max_pixels, ctypes.byref(h)),
                 "spr_batch_create_empty")
        self.h = h

    def set(self, renders):
        rs = list(renders)
        arr = (ctypes.c_void_p * max(len(rs), 1))(*[r.h_ for r in rs])
        _chk(load_library().spr_batch_set(self.h, len(rs), arr), "spr_batch_set")
        self.renders = rs

    def pass_(self) -> int:
        n = ctypes.c_uint32()
        _chk(load_library().spr_batch_pass(self.h, ctypes.byref(n)), "spr_batch_pass")
        return n.value

    def run(self, max_passes: int = 100000, poll_every: int = 1) -> int:
        n = ctypes.c_uint32()
        _chk(load_library().spr_batch_run(self.h, max_passes, poll_every, ctypes.byref(n)), "spr_batch_run")
        return n.value

    def state(self):
        """([per-member dicts], active blocks of the last pass)."""
        n = len(self.renders)
        arr = (MemberState * max(n, 1))()
        ab = ctypes.c_uint32()
        _chk(load_library().spr_batch_state(self.h, arr, n, ctypes.byref(ab)), "spr_batch_state")
        return [{f: getattr(arr[i], f) for f, _ in MemberState._fields_} for i in range(n)], ab.value

    def free(self):
        if self.h:
            _chk(load_library().spr_batch_free(self.h), "spr_batch_free")
            self.h = None


def version() -> str:
    return load_library().spr_version().decode()
