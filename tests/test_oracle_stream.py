"""Pins of the oracle's streamed paths (for volumes too large to decode whole):
the march that decodes blocks on demand, the block ranges computed one
record at a time and the grids built from them must equal the whole-volume
oracle (itself pinned by the analytic and brute-force tests) bitwise.  Also
pins the streamed RM-like generator against encoding its materialised field.
"""
import numpy as np
import pytest

import oracle
import volgen


def _cases():
    yield "blobs64_r8", volgen.blobs(64, 64, 64, seed=1), 8
    yield "fourier_ragged_r4", volgen.fourier(37, 29, 23, seed=5, nmode=16, kmax=6, period=64.0), 4
    yield "fourier_ragged_r2", volgen.fourier(30, 41, 19, seed=6, nmode=16, kmax=6, period=64.0), 2
    yield "sphere_raw", volgen.analytic(24, 24, 24, "sphere", (11.5, 11.5, 11.5)), 32


@pytest.mark.parametrize("name,vol,rate", list(_cases()), ids=[c[0] for c in _cases()])
def test_streamed_render_equals_whole_volume_render(name, vol, rate):
    nz, ny, nx = vol.shape
    s = volgen.encode(vol, rate)
    dec = oracle.decode_volume(s, (nx, ny, nz), rate)
    iso = float(np.percentile(dec, 55))
    for k in range(3):
        cam = volgen.orbit_camera(nx, ny, nz, seed=11 + k, k=k, npos=3)
        a = oracle.render(dec, cam, iso, 48, 36)
        b = oracle.render_stream(s, (nx, ny, nz), rate, cam, iso, 48, 36)
        assert np.array_equal(a["t"].view(np.uint64), b["t"].view(np.uint64)), name
        for key in ("block", "cell", "rgba", "entered"):
            assert np.array_equal(a[key], b[key]), (name, key)
        assert np.isfinite(a["t"]).sum() > 0, name


def test_streamed_render_pixel_subset():
    vol = volgen.blobs(40, 40, 40, seed=3)
    s = volgen.encode(vol, 4)
    dec = oracle.decode_volume(s, (40, 40, 40), 4)
    cam = volgen.orbit_camera(40, 40, 40, seed=3)
    full = oracle.render(dec, cam, 0.5, 64, 64)
    pix = np.random.default_rng(0).choice(64 * 64, 300, replace=False).astype(np.uint32)
    sub = oracle.render_stream(s, (40, 40, 40), 4, cam, 0.5, 64, 64, pixels=pix)
    assert np.array_equal(sub["t"].view(np.uint64), full["t"][pix].view(np.uint64))
    assert np.array_equal(sub["block"], full["block"][pix])


@pytest.mark.parametrize("name,vol,rate", list(_cases()), ids=[c[0] for c in _cases()])
def test_streamed_ranges_and_grids_equal_whole_volume(name, vol, rate):
    nz, ny, nx = vol.shape
    s = volgen.encode(vol, rate)
    dec = oracle.decode_volume(s, (nx, ny, nz), rate)
    blk, fine, coarse = oracle.grids(dec)
    sblk = oracle.block_ranges_stream(s, (nx, ny, nz), rate)
    assert np.array_equal(sblk.view(np.uint32), blk.view(np.uint32)), name
    sf, sc = oracle.grids_from_blocks(sblk, (nx, ny, nz))
    assert np.array_equal(sf.view(np.uint32), fine.view(np.uint32)), name
    assert np.array_equal(sc.view(np.uint32), coarse.view(np.uint32)), name


@pytest.mark.parametrize("dims", [(64, 48, 40), (37, 29, 31)])
def test_rm_streamed_encoder_equals_encoding_the_field(dims):
    nx, ny, nz = dims
    field = volgen.rm_field(nx, ny, nz, seed=3)
    for rate in (2, 4):
        a = volgen.rm_encode(nx, ny, nz, rate, seed=3)
        b = volgen.encode(field, rate)
        assert np.array_equal(a, b), (dims, rate)
    # values are the 0..255 mixing-layer levels, with both fluids present
    assert field.min() == 0.0 and field.max() == 255.0
    assert np.all(field == np.round(field))
