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


def test_struct_layouts_match_c_compiler(tmp_path):
    """Every ctypes mirror has the size and field offsets gcc gives the
    header's struct (a C program built from include/spr.h prints them)."""
    import subprocess
    from paper_2309_10212_amd import spr
    pairs = [("spr_allocator", spr._Allocator), ("spr_config", spr._Config), ("spr_volume_desc", spr._VolumeDesc),
             ("spr_camera", spr._Camera), ("spr_pass_stats", spr.PassStats), ("spr_counters", spr.Counters),
             ("spr_render_info", spr.RenderInfo), ("spr_mem_split", spr.MemSplit), ("spr_tuning", spr.Tuning),
             ("spr_member_state", spr.MemberState), ("spr_kernel_time", spr.KernelTime)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spr.h"', 'int main(void) {']
    for cname, cls in pairs:
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            cf = {"pass_": "pass"}.get(fname, fname)
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {cf}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run(["gcc", "-std=c11", "-I", inc, "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.splitlines())
    for cname, cls in pairs:
        assert int(got[cname]) == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(cls, fname).offset, (cname, fname)
