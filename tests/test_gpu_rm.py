"""GPU parity on the RM-like mixing-layer volume at full size: 2048x2048x1920
values 0..255 (as float32) compressed at 2 bits/value (2,013,265,920 bytes,
125,829,120 blocks), rendered at 1280x720 with speculation cap 64 and a
2*10^9-byte cache, at isovalues 64, 128 and 192.

The volume cannot be decoded whole on the host (32 GB), so the oracle's
streamed paths are used: every block decoded by the device decoder is
compared bitwise with the oracle's decode, in chunks; block ranges one record
at a time (the fine and coarse grids must match bitwise); and, on every 8th
row and column of the image plus a seeded sample of hit pixels, the
per-pixel march reading blocks decoded on demand (hit block and cell exact,
t within 1e-4, RGBA within 1 LSB).  Properties that hold at any size are
checked on every pass: at most w*h pairs, no cache overflow, no step-guard
exit."""
import time

import numpy as np
import pytest

import oracle
import volgen

pytestmark = pytest.mark.gpu

NX, NY, NZ, RATE, W, H = 2048, 2048, 1920, 2, 1280, 720
DIMS = (NX, NY, NZ)


@pytest.fixture(scope="module")
def rm():
    t0 = time.time()
    s = volgen.rm_encode(NX, NY, NZ, RATE, seed=3)
    print(f"RM-like stream: {s.nbytes} bytes in {time.time() - t0:.1f} s", flush=True)
    assert s.nbytes == 2_013_265_920
    cams = [volgen.orbit_camera(NX, NY, NZ, seed=3, k=k, npos=10) for k in range(10)]
    from paper_2309_10212_amd import spr
    ctx = spr.Context(device=0, cache_bytes=2 * 10**9, spec_cap=64)
    t0 = time.time()
    vol = ctx.load_volume(s, DIMS, RATE)
    print(f"loaded in {time.time() - t0:.1f} s", flush=True)
    yield s, cams, ctx, vol
    vol.free()
    ctx.close()


def test_rm_fullsize_grids(rm):
    s, _, _, vol = rm
    fine, coarse = vol.ranges()
    t0 = time.time()
    blk = oracle.block_ranges_stream(s, DIMS, RATE)
    rf, rc = oracle.grids_from_blocks(blk, DIMS)
    del blk
    print(f"oracle grids in {time.time() - t0:.1f} s", flush=True)
    assert np.array_equal(coarse.view(np.uint32), rc.view(np.uint32))
    assert np.array_equal(fine.view(np.uint32), rf.view(np.uint32))
    # both fluids are present (decoded values may overshoot 0..255 at 2 bits/value)
    assert coarse[:, 0].min() <= 0.0 and coarse[:, 1].max() >= 255.0


def test_rm_every_block_decodes_bitexact(rm):
    s, _, _, vol = rm
    nb = vol.nblocks
    assert nb == 125_829_120
    chunk = 1 << 21
    t0 = time.time()
    for b0 in range(0, nb, chunk):
        ids = np.arange(b0, min(nb, b0 + chunk), dtype=np.uint32)
        got = vol.decode_blocks(ids)
        ref = oracle.decode_blocks(s, DIMS, RATE, ids)
        if not np.array_equal(got.view(np.uint32), ref.view(np.uint32)):
            bad = np.nonzero((got.view(np.uint32) != ref.view(np.uint32)).any(axis=1))[0]
            raise AssertionError(f"blocks {ids[bad[:8]]} differ ({bad.size} in chunk at {b0})")
        del got, ref
    print(f"{nb} blocks decoded and compared in {time.time() - t0:.1f} s", flush=True)


def _subset():
    ys, xs = np.meshgrid(np.arange(0, H, 8), np.arange(0, W, 8), indexing="ij")
    return (ys * W + xs).astype(np.uint32).ravel()


@pytest.mark.parametrize("iso", [64.0, 128.0, 192.0])
def test_rm_fullsize_render_sampled(rm, iso):
    from paper_2309_10212_amd import spr
    s, cams, ctx, vol = rm
    k = {64.0: 0, 128.0: 3, 192.0: 7}[iso]
    r = spr.Render(vol, cams[k], iso, W, H, spec_cap=64)
    c0 = ctx.counters()
    passes = 0
    t0 = time.time()
    while not r.done():
        st = r.pass_(stats=True)
        passes += 1
        assert st["pairs"] <= W * H
        assert passes < 500
    c1 = ctx.counters()
    assert c1["overflow"] == c0["overflow"]
    hits, img = r.hits(), r.image().reshape(-1, 4).astype(np.int32)
    info = r.info()
    print(f"iso {iso}: {passes} passes in {time.time() - t0:.2f} s, {info['rays_entered']} rays entered, "
          f"{int(np.isfinite(hits['t']).sum())} hits, {c1['blocks_decoded'] - c0['blocks_decoded']} blocks decoded",
          flush=True)
    assert c1["walk_guard"] == c0["walk_guard"]
    rng = np.random.default_rng(int(iso))
    fin = np.nonzero(np.isfinite(hits["t"]))[0]
    # every 8th row and column, plus a seeded sample of hit pixels
    pix = np.unique(np.concatenate([_subset(), rng.choice(fin, min(512, fin.size), replace=False)
                                    if fin.size else np.zeros(0, np.int64)]).astype(np.int64))
    pix = pix.astype(np.uint32)
    t0 = time.time()
    ref = oracle.render_stream(s, DIMS, RATE, cams[k], iso, W, H, pixels=pix)
    print(f"oracle: {pix.size} pixels in {time.time() - t0:.1f} s", flush=True)
    g = hits[pix]
    fin_ref = np.isfinite(ref["t"])
    assert np.array_equal(np.isfinite(g["t"]), fin_ref)
    assert np.array_equal(g["block"], ref["block"])
    assert np.array_equal(g["cell"], ref["cell"])
    if fin_ref.any():
        assert float(np.abs(g["t"][fin_ref] - ref["t"][fin_ref]).max()) <= 1e-4
    o = ref["rgba"].view(np.uint8).reshape(-1, 4).astype(np.int32)
    assert np.abs(img[pix] - o).max() <= 1
    assert int(ref["entered"].sum()) > 0
    r.free()
