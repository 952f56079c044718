"""GPU parity at the benchmark's full size, in the benchmark's launch
configuration: the 512^3 Fourier field at 4 bits/value, 1280x720, the 60th-
percentile isovalue, cache 512*10^6 bytes.  Every pixel is compared with the
oracle (hit block and cell exact, t within 1e-4, RGBA within 1 LSB), the
per-pass counters against the oracle's pass schedule, the macrocell grids
bitwise, and every decoded block bitwise.  A small cache
(deferral and LRU sweeps at scale) must give the same image."""
import numpy as np
import pytest

import oracle
import volgen

pytestmark = pytest.mark.gpu

N, RATE, W, H = 512, 4, 1280, 720


@pytest.fixture(scope="module")
def fourier():
    f = volgen.fourier(N, N, N, seed=2, nmode=64, kmax=24, period=float(N))
    iso = volgen.percentile_value(f, 0.6)
    s = volgen.encode(f, RATE)
    del f
    dec = oracle.decode_volume(s, (N, N, N), RATE)
    cams = [volgen.orbit_camera(N, N, N, seed=2, k=k, npos=10) for k in range(10)]
    return s, dec, iso, cams


def _cmp(hits, img, ref, label):
    fin = np.isfinite(ref["t"])
    assert np.array_equal(np.isfinite(hits["t"]), fin), label
    bad = np.nonzero(hits["block"] != ref["block"])[0]
    assert bad.size == 0, (label, bad[:8])
    bad = np.nonzero(hits["cell"] != ref["cell"])[0]
    assert bad.size == 0, (label, bad[:8])
    dt = float(np.abs(hits["t"][fin] - ref["t"][fin]).max())
    assert dt <= 1e-4, (label, dt)
    g = img.reshape(-1, 4).astype(np.int32)
    o = ref["rgba"].view(np.uint8).reshape(-1, 4).astype(np.int32)
    assert np.abs(g - o).max() <= 1, label
    return dt


def test_fullsize_grids_decode_and_render(fourier):
    from paper_2309_10212_amd import spr
    s, dec, iso, cams = fourier
    ctx = spr.Context(device=0, cache_bytes=512 * 10**6, spec_cap=16)
    vol = ctx.load_volume(s, (N, N, N), RATE)
    fine, coarse = vol.ranges()
    _, rf, rc = oracle.grids(dec)
    assert np.array_equal(fine, rf) and np.array_equal(coarse, rc)
    # every block through the device decoder, bitwise against the oracle's decode
    for b0 in range(0, vol.nblocks, 1 << 20):
        ids = np.arange(b0, min(vol.nblocks, b0 + (1 << 20)), dtype=np.uint32)
        assert np.array_equal(vol.decode_blocks(ids).view(np.uint32),
                              oracle.decode_blocks(s, (N, N, N), RATE, ids).view(np.uint32)), b0
    for k, cap, pol in ((0, 16, 0), (5, 1, 0), (7, 64, 0), (3, 64, 1)):
        r = spr.Render(vol, cams[k], iso, W, H, spec_cap=cap, policy=pol)
        got = []
        while not r.done():
            got.append(r.pass_(stats=True))
            assert len(got) < 500
        sched = oracle.schedule(dec, cams[k], iso, W, H, cap, policy=pol)
        assert len(got) == len(sched), (k, cap, len(got), len(sched))
        keys = ("n_active", "slots", "pairs", "visible", "active_blocks", "terminated") if pol else \
            ("n_active", "n_spec", "slots", "pairs", "visible", "active_blocks", "terminated")
        for p, (g, o) in enumerate(zip(got, sched)):
            for key in keys:
                assert g[key] == o[key], (k, cap, pol, p, key, g, o)
        dt = _cmp(r.hits(), r.image(), oracle.render(dec, cams[k], iso, W, H), f"view {k} cap {cap}")
        assert r.info()["bcmc_blocks"] == oracle.blocks_containing(rf, iso)
        print(f"view {k} cap {cap} policy {pol}: {len(got)} passes, max |dt| {dt:.3g}", flush=True)
        r.free()
    vol.free()
    ctx.close()


def test_fullsize_small_cache_defers_and_evicts(fourier):
    from paper_2309_10212_amd import spr
    s, dec, iso, cams = fourier
    ctx = spr.Context(device=0, cache_bytes=256 * 60000, spec_cap=16)
    vol = ctx.load_volume(s, (N, N, N), RATE)
    for k in (2, 3):
        r = spr.Render(vol, cams[k], iso, W, H)
        deferred = 0
        passes = 0
        while not r.done():
            st = r.pass_(stats=True)
            deferred += st["deferred"]
            passes += 1
            assert st["active_blocks"] <= 60000
            assert passes < 2000
        _cmp(r.hits(), r.image(), oracle.render(dec, cams[k], iso, W, H), f"small cache view {k}")
        assert deferred > 0
        r.free()
    c = ctx.counters()
    assert c["evicted"] > 0 and c["overflow"] == 0
    vol.free()
    ctx.close()
