"""GPU tests of the engine behind the C ABI: memory accounting by kind,
error paths through the product library (short stream, failing allocator),
the hand-built codec record decoded on the device, the step-guard counter,
and renders whose rays pass exactly through block corners and along block
edges (exact ties of the cell walk, Sec. 3.3 / 3.7)."""
import json
import os

import numpy as np
import pytest

import oracle
import volgen

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


class CountingAllocator:
    """torch's caching allocator behind counters; fails every allocation
    after `fail_after` successful ones when set."""

    def __init__(self, fail_after=None):
        import torch
        self.torch = torch
        self.live = {}
        self.allocs = self.frees = 0
        self.fail_after = fail_after

    def alloc(self, nbytes):
        if self.fail_after is not None and self.allocs >= self.fail_after:
            return None
        p = self.torch.cuda.caching_allocator_alloc(nbytes, 0, self.torch.cuda.current_stream(0))
        self.live[p] = nbytes
        self.allocs += 1
        return p

    def free(self, p, nbytes):
        assert self.live.pop(p) == nbytes
        self.frees += 1
        self.torch.cuda.caching_allocator_delete(p)


def _tiny():
    n = 64
    f = volgen.blobs(n, n, n, 1)
    s = volgen.encode(f, 8)
    return s, (n, n, n)


def test_memory_by_kind_returns_to_zero_and_allocations_balance():
    from paper_2309_10212_amd import spr
    ca = CountingAllocator()
    ctx = spr.Context(device=0, cache_bytes=64 << 20, alloc_hooks=(ca.alloc, ca.free))
    m0 = ctx.mem_split()
    assert m0["current"]["cache"] >= (64 << 20) and m0["current"]["compressed"] == 0
    s, dims = _tiny()
    vol = ctx.load_volume(s, dims, 8)
    m1 = ctx.mem_split()
    assert m1["current"]["compressed"] >= s.nbytes
    nb = 16 ** 3
    # per-block state: fine ranges (8 B) plus map, pair counter, visible index (4 B each); per
    # coarse cell of 4^3 blocks its range (8 B) and claim word (8 B)
    assert nb * 20 + (nb // 64) * 16 <= m1["current"]["grids"] <= nb * 20 + 64 * 1024
    cam = volgen.orbit_camera(*dims, seed=1)
    rs = [spr.Render(vol, cam, 0.5, 96, 64, spec_cap=c) for c in (1, 16)]
    rs[0].run()
    b = spr.Batch(ctx, rs[1:])
    b.run()
    m2 = ctx.mem_split()
    assert m2["current"]["rays"] > 0 and m2["current"]["scratch"] > 0
    assert sum(m2["current"].values()) == m2["total"]
    assert sum(m2["at_peak"].values()) == m2["peak"]
    b.free()
    for r in rs:
        r.free()
    vol.free()
    m3 = ctx.mem_split()
    for k in ("compressed", "grids", "rays"):
        assert m3["current"][k] == 0, (k, m3)
    assert ctx.counters()["walk_guard"] == 0
    ctx.close()
    assert ca.allocs == ca.frees and not ca.live, (ca.allocs, ca.frees, len(ca.live))


def test_short_stream_is_corrupt_and_bad_version_invalid():
    from paper_2309_10212_amd import spr
    ctx = spr.Context(device=0, cache_bytes=1 << 20)
    s, dims = _tiny()
    with pytest.raises(spr.SprError) as e:
        ctx.load_volume(s[:-1], dims, 8)
    assert e.value.status == -4
    with pytest.raises(spr.SprError) as e:
        ctx.load_volume(np.concatenate([s, s[:8]]), dims, 8)
    assert e.value.status == -4
    with pytest.raises(spr.SprError) as e:
        ctx.load_volume(s, dims, 8, codec_version=2)
    assert e.value.status == -1
    assert ctx.mem_split()["current"]["compressed"] == 0
    ctx.close()


def test_extent_and_eye_limits_are_invalid():
    """Volumes longer than MAX_EXTENT samples on an axis and eyes farther than
    MAX_EXTENT on a coordinate are rejected (the traversal's block estimate is
    exact within these limits); the limits themselves are accepted."""
    from paper_2309_10212_amd import spr
    ctx = spr.Context(device=0, cache_bytes=1 << 20)
    s, dims = _tiny()
    with pytest.raises(spr.SprError) as e:
        ctx.load_volume(s, (spr.MAX_EXTENT + 1, 2, 2), 8)
    assert e.value.status == -1
    vol = ctx.load_volume(s, dims, 8)
    c = dims[0] / 2.0
    for eye, ok in [((spr.MAX_EXTENT + 1.0, c, c), False), ((c, c, -spr.MAX_EXTENT - 0.5), False),
                    ((float(spr.MAX_EXTENT), c, c), True)]:
        cam = volgen.Camera(eye=eye, center=(c, c, c), up=(0.0, 0.0, 1.0) if eye[2] == c else (0.0, 1.0, 0.0),
                            vfov_deg=0.01)
        if ok:
            r = spr.Render(vol, cam, 0.5, 8, 8)
            r.run()
            r.free()
        else:
            with pytest.raises(spr.SprError) as e:
                spr.Render(vol, cam, 0.5, 8, 8)
            assert e.value.status == -1
    vol.free()
    ctx.close()


@pytest.mark.parametrize("fail_after", [0, 1, 3, 6])
def test_failing_allocator_gives_oom_and_leaks_nothing(fail_after):
    from paper_2309_10212_amd import spr
    ca = CountingAllocator()
    ctx = spr.Context(device=0, cache_bytes=1 << 20, alloc_hooks=(ca.alloc, ca.free))
    before = ctx.mem_split()["total"]
    n0 = ca.allocs
    ca.fail_after = n0 + fail_after     # the volume's fail_after-th allocation fails
    s, dims = _tiny()
    with pytest.raises(spr.SprError) as e:
        ctx.load_volume(s, dims, 8)
    assert e.value.status == -2
    assert ctx.mem_split()["total"] == before
    ca.fail_after = None
    vol = ctx.load_volume(s, dims, 8)        # the context still works
    cam = volgen.orbit_camera(*dims, seed=1)
    ca.fail_after = ca.allocs + 2
    with pytest.raises(spr.SprError) as e:
        spr.Render(vol, cam, 0.5, 64, 64)
    assert e.value.status == -2
    ca.fail_after = None
    # the failed set-up left no masks for its isovalue: the next render builds them
    r = spr.Render(vol, cam, 0.5, 64, 64)
    assert r.info()["masks_built"] == 1
    r.run()
    r.free()
    vol.free()
    ctx.close()
    assert ca.allocs == ca.frees and not ca.live


def test_hand_built_record_decodes_on_the_device():
    """The record of tests/golden/codec_wrap_record.json (its inverse transform
    wraps in 32 bits; expected samples derived by hand) as a one-block volume."""
    from paper_2309_10212_amd import spr
    with open(os.path.join(HERE, "golden", "codec_wrap_record.json")) as fh:
        g = json.load(fh)
    rec = np.array([int(w, 16) for w in g["record_words_hex"]], np.uint32)
    ctx = spr.Context(device=0, cache_bytes=1 << 20)
    vol = ctx.load_volume(rec.view(np.uint8), (4, 4, 4), g["rate_bits"])
    got = vol.decode_blocks(np.array([0], np.uint32))[0]
    assert np.array_equal(got, np.array(g["expected_values"], np.float32))
    vol.free()
    ctx.close()


def _tie_cameras(n):
    """Eyes on lattice points looking along exact diagonals (the centre pixel
    of an odd-sized image looks exactly along the view direction, so its ray
    crosses x, y and z planes at identical parameters and passes through
    block corners), and eyes on block edges and faces looking along an axis
    (the ray runs along the shared edge of four blocks or the face of two)."""
    m = n - 1
    far = 4 * ((m + 8) // 4 + 1)      # a multiple of 4 beyond the top face: block corners stay on the diagonal
    cams = []
    for sx, sy, sz in ((1, 1, 1), (-1, 1, 1), (1, -1, 1), (1, 1, -1)):
        eye = tuple(float(-8 if s > 0 else far) for s in (sx, sy, sz))
        cen = tuple(e + s * 40.0 for e, s in zip(eye, (sx, sy, sz)))
        up = (0.0, 1.0, 0.0) if (sx, sy) == (1, 1) and sz == 1 else (0.0, 0.0, 1.0)
        cams.append(volgen.Camera(eye=eye, center=cen, up=up, vfov_deg=40.0))
    for x, y in ((4.0, 8.0), (16.0, 16.0), (0.0, 12.0), (float(m), 20.0), (4.0, 9.5)):
        cams.append(volgen.Camera(eye=(x, y, -10.0), center=(x, y, 40.0), up=(0.0, 1.0, 0.0), vfov_deg=35.0))
    cams.append(volgen.Camera(eye=(12.0, -10.0, 8.0), center=(12.0, 40.0, 8.0), up=(0.0, 0.0, 1.0), vfov_deg=35.0))
    return cams


@pytest.mark.parametrize("rate,cap", [(8, 1), (8, 64), (32, 16)])
def test_exact_block_ties_match_the_oracle(rate, cap):
    from paper_2309_10212_amd import spr
    from test_gpu_parity import _cmp_hits
    n = 48
    f = volgen.blobs(n, n, n, 5)
    s = volgen.encode(f, rate)
    dec = oracle.decode_volume(s, (n, n, n), rate)
    iso = float(volgen.percentile_value(dec, 0.8))
    ctx = spr.Context(device=0, cache_bytes=64 << 20)
    vol = ctx.load_volume(s, (n, n, n), rate)
    w = h = 33
    centre_hits = 0
    for k, cam in enumerate(_tie_cameras(n)):
        r = spr.Render(vol, cam, iso, w, h, spec_cap=cap)
        r.run()
        ref = oracle.render(dec, cam, iso, w, h)
        _cmp_hits(r.hits(), r.image(), ref, f"tie camera {k} rate {rate} cap {cap}")
        centre_hits += bool(np.isfinite(ref["t"][(h // 2) * w + w // 2]))
        r.free()
    assert centre_hits >= 3, centre_hits
    assert ctx.counters()["walk_guard"] == 0
    vol.free()
    ctx.close()
