"""The C-ABI library loads and exports every call that include/spr.h declares
(CPU only: no compute calls)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spr.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:spr_status|const char \*)\s*(spr_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["spr_ctx_create", "spr_volume_load", "spr_render_begin", "spr_render_pass", "spr_read_image",
                 "spr_read_hits", "spr_batch_create", "spr_batch_pass", "spr_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2309_10212_amd import spr
    lib = spr.load_library()
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers exactly the declared calls
    assert sorted(n for n, _, _ in spr.SIGNATURES) == declared()
    assert b"gfx950" in lib.spr_version()


def test_error_paths_without_gpu():
    from paper_2309_10212_amd import spr
    lib = spr.load_library()
    assert lib.spr_ctx_create(None, None) == -1
    assert b"null" in lib.spr_last_error()
    assert lib.spr_render_pass(None, None) == -1
    assert lib.spr_volume_free(None) == -1
    assert lib.spr_batch_free(None) == -1


def test_config_is_validated_before_any_device_call():
    from paper_2309_10212_amd import spr
    lib = spr.load_library()
    out = ctypes.c_void_p()
    cfg = spr._Config()
    cfg.device, cfg.cache_bytes, cfg.flags = 0, 1 << 20, 1
    assert lib.spr_ctx_create(ctypes.byref(cfg), ctypes.byref(out)) == -1
    assert b"flags" in lib.spr_last_error()
    cfg.flags, cfg.spec_cap = 0, 4097   # beyond the documented 1..4096
    assert lib.spr_ctx_create(ctypes.byref(cfg), ctypes.byref(out)) == -1
    assert b"spec cap" in lib.spr_last_error()
    assert not out.value


def test_struct_layouts_match_header():
    from paper_2309_10212_amd import spr
    assert ctypes.sizeof(spr.PassStats) == 56
    assert spr.HIT_DTYPE.itemsize == 16
    assert ctypes.sizeof(spr._Camera) == 80
    assert ctypes.sizeof(spr._VolumeDesc) == 24
