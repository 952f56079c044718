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


def test_struct_layouts_match_header():
    from paper_2309_10212_amd import spr
    assert ctypes.sizeof(spr.PassStats) == 56
    assert spr.HIT_DTYPE.itemsize == 16
    assert ctypes.sizeof(spr._Camera) == 80
    assert ctypes.sizeof(spr._VolumeDesc) == 24
