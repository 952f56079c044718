"""GPU parity: the HIP path through the C ABI against the CPU oracle, element
by element on the same seeded inputs.

Bar: decoded values, macrocell ranges, hit block and cell indices and the
per-pass integer counters bit-exact; hit parameter t within 1e-4 voxels;
RGBA8 within 1 LSB per channel.
"""
import numpy as np
import pytest

import oracle
import volgen

pytestmark = pytest.mark.gpu

T_TOL = 1e-4


@pytest.fixture(scope="module", params=[(256, 32), (256, 0)], ids=["staged", "direct"])
def ctx(request):
    """A context with each block-raytrace variant: dual grids staged in LDS
    per tile, or every pair reading its corners from the cache slots."""
    from paper_2309_10212_amd import spr
    c = spr.Context(device=0, cache_bytes=256 << 20)
    c.set_tuning(*request.param)
    yield c
    c.close()


@pytest.fixture(autouse=True)
def _no_step_guard_exit(request):
    """Every walk ends by leaving the domain or its block, or by finding its
    blocks, never by the step guard (a counter the library keeps)."""
    yield
    if "ctx" in request.fixturenames:
        assert request.getfixturevalue("ctx").counters()["walk_guard"] == 0


def _cmp_hits(hits, img, ref, label=""):
    fin = np.isfinite(ref["t"])
    gfin = np.isfinite(hits["t"])
    bad = np.nonzero(fin != gfin)[0]
    assert bad.size == 0, f"{label}: hit/miss differs at {bad[:10]} (gpu t {hits['t'][bad[:5]]}, ref {ref['t'][bad[:5]]})"
    bb = np.nonzero(hits["block"] != ref["block"])[0]
    assert bb.size == 0, f"{label}: block differs at {bb[:10]}: {hits['block'][bb[:5]]} vs {ref['block'][bb[:5]]}"
    cb = np.nonzero(hits["cell"] != ref["cell"])[0]
    assert cb.size == 0, f"{label}: cell differs at {cb[:10]}"
    if fin.any():
        dt = np.abs(hits["t"][fin] - ref["t"][fin]).max()
        assert dt <= T_TOL, f"{label}: max |dt| = {dt}"
    g = img.reshape(-1, 4).astype(np.int32)
    o = ref["rgba"].view(np.uint8).reshape(-1, 4).astype(np.int32)
    d = np.abs(g - o).max() if g.size else 0
    assert d <= 1, f"{label}: rgba differs by {d}"


def test_fp64_sqrt_and_division_correctly_rounded(ctx):
    rng = np.random.default_rng(0)
    n = 1 << 20
    x = np.exp(rng.uniform(-700, 700, n)) * rng.choice([1.0, 1.0, 1.0, -1.0], n)
    y = np.exp(rng.uniform(-700, 700, n)) * rng.choice([1.0, -1.0], n)
    x[:8] = [0.0, -0.0, 1.0, 2.0, 5e-324, 1.7976931348623157e308, 0.5, 3.0]
    y[:8] = [1.0, 3.0, 3.0, 7.0, 2.0, 0.5, 1e-300, 1e300]
    sq, dv = ctx.fp64_ops(np.abs(x), y)
    assert np.array_equal(sq.view(np.uint64), np.sqrt(np.abs(x)).view(np.uint64))
    assert np.array_equal(dv.view(np.uint64), (np.abs(x) / y).view(np.uint64))


@pytest.mark.parametrize("dims,rate,kind", [((64, 64, 64), 8, "blobs"), ((37, 29, 23), 2, "fourier"),
                                            ((32, 32, 32), 4, "fourier"), ((16, 12, 9), 16, "blobs"),
                                            ((20, 20, 20), 32, "blobs"), ((8, 8, 8), 1, "blobs")])
def test_decode_bitexact(ctx, dims, rate, kind):
    nx, ny, nz = dims
    f = volgen.blobs(nx, ny, nz, 3) if kind == "blobs" else volgen.fourier(nx, ny, nz, 5, nmode=16, kmax=6)
    s = volgen.encode(f, rate)
    vol = ctx.load_volume(s, dims, rate)
    ids = np.arange(vol.nblocks, dtype=np.uint32)
    got = vol.decode_blocks(ids)
    ref = oracle.decode_blocks(s, dims, rate, ids)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    vol.free()


def _arbitrary_records(rate, rng):
    """Records that no encoder writes but the decoder must take as they come:
    random bits at several densities, and all ones / all zeros / periodic
    bits with the exponent field varied.  They reach the decoder's edge
    paths: every plane empty, all 64 coefficients significant before a plane
    with refinement bits, scans that run out of candidates or of record."""
    nbits = 64 * rate
    recs = []
    for p1 in (0.005, 0.05, 0.3, 0.8, 0.995):
        bits = (rng.random((128, nbits)) < p1).astype(np.uint8)
        recs.append(bits)
    for pat in ("ones", "zeros", "p3", "p7", "p61"):
        b = np.zeros((64, nbits), np.uint8)
        for i in range(64):
            if pat == "ones":
                b[i, :] = 1
            elif pat != "zeros":
                per = int(pat[1:])
                b[i, (np.arange(nbits) + i) % per == 0] = 1
            b[i, 1:9] = (np.arange(8) < (i % 9)).astype(np.uint8)
        recs.append(b)
    bits = np.concatenate(recs)
    bits[:, 0] = 1   # every record nonzero
    return np.packbits(bits, axis=1, bitorder="little").reshape(-1)


@pytest.mark.parametrize("rate", list(range(1, 17)))
def test_decode_bitexact_arbitrary_records(ctx, rate):
    s = _arbitrary_records(rate, np.random.default_rng(100 + rate))
    nb = s.size // (8 * rate)
    dims = (4 * nb, 4, 4)
    vol = ctx.load_volume(s, dims, rate)
    ids = np.arange(nb, dtype=np.uint32)
    got = vol.decode_blocks(ids)
    ref = oracle.decode_blocks(s, dims, rate, ids)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    vol.free()


@pytest.mark.parametrize("dims,rate", [((64, 64, 64), 8), ((37, 29, 23), 2), ((17, 21, 65), 4)])
def test_grids_bitexact(ctx, dims, rate):
    nx, ny, nz = dims
    s = volgen.encode(volgen.fourier(nx, ny, nz, 7, nmode=16, kmax=6), rate)
    vol = ctx.load_volume(s, dims, rate)
    fine, coarse = vol.ranges()
    dec = oracle.decode_volume(s, dims, rate)
    _, rfine, rcoarse = oracle.grids(dec)
    assert np.array_equal(fine, rfine)
    assert np.array_equal(coarse, rcoarse)
    vol.free()


def _tiny():
    n = 64
    f = volgen.blobs(n, n, n, 1)
    s = volgen.encode(f, 8)
    dec = oracle.decode_volume(s, (n, n, n), 8)
    cam = volgen.orbit_camera(n, n, n, seed=1)
    return s, dec, cam


@pytest.mark.parametrize("cap", [1, 64])
def test_tiny_render_and_pass_counters(ctx, cap):
    from paper_2309_10212_amd import spr
    s, dec, cam = _tiny()
    n, w, h, iso = 64, 256, 256, 0.5
    vol = ctx.load_volume(s, (n, n, n), 8)
    r = spr.Render(vol, cam, iso, w, h, spec_cap=cap)
    sched = oracle.schedule(dec, cam, iso, w, h, cap)
    got = []
    while not r.done():
        got.append(r.pass_(stats=True))
        assert len(got) <= len(sched) + 2
    ref = oracle.render(dec, cam, iso, w, h)
    _cmp_hits(r.hits(), r.image(), ref, f"tiny cap={cap}")
    assert len(got) == len(sched)
    for p, (g, o) in enumerate(zip(got, sched)):
        for k in ("n_active", "n_spec", "pairs", "visible", "active_blocks", "terminated"):
            assert g[k] == o[k], (p, k, g, o)
    # the BCMC-proxy count: blocks whose fine range contains the isovalue
    _, fine, coarse = oracle.grids(dec)
    assert r.info()["bcmc_blocks"] == oracle.blocks_containing(fine, iso)
    # the coarse cells whose range contains the isovalue (their fine ranges are read for the masks)
    assert r.info()["iso_coarse_cells"] == oracle.blocks_containing(coarse, iso)
    r.free()
    vol.free()


@pytest.mark.parametrize("cap", [1, 64])
def test_sparse_volume_empty_space_jumps(ctx, cap):
    """Two small blobs in a 256^3 volume: most coarse cells are far from any
    candidate block, so the traversal jumps over empty space.  Every pixel and
    every per-pass counter must equal the oracle (which marches every cell)."""
    from paper_2309_10212_amd import spr
    n = 256
    f = volgen.blobs(n, n, n, seed=21, nblob=2)
    s = volgen.encode(f, 8)
    dec = oracle.decode_volume(s, (n, n, n), 8)
    vol = ctx.load_volume(s, (n, n, n), 8)
    for k in range(2):
        cam = volgen.orbit_camera(n, n, n, seed=21 + k)
        iso = 0.3
        r = spr.Render(vol, cam, iso, 160, 120, spec_cap=cap)
        got = []
        while not r.done():
            got.append(r.pass_(stats=True))
            assert len(got) < 400
        sched = oracle.schedule(dec, cam, iso, 160, 120, cap)
        assert len(got) == len(sched), (k, len(got), len(sched))
        for p, (g, o) in enumerate(zip(got, sched)):
            for key in ("n_active", "n_spec", "pairs", "visible", "active_blocks", "terminated"):
                assert g[key] == o[key], (k, p, key, g, o)
        _cmp_hits(r.hits(), r.image(), oracle.render(dec, cam, iso, 160, 120), f"sparse view {k} cap {cap}")
        r.free()
    vol.free()


def test_far_eye_at_the_extent_limit(ctx):
    """Eyes at the coordinate limit: ray parameters near 10^6 samples, where the
    traversal's fp32 block estimates carry their largest error."""
    from paper_2309_10212_amd import spr
    n = 64
    s = volgen.encode(volgen.blobs(n, n, n, 5), 8)
    dec = oracle.decode_volume(s, (n, n, n), 8)
    vol = ctx.load_volume(s, (n, n, n), 8)
    lim = float(spr.MAX_EXTENT)
    for eye in [(lim, 0.61 * lim, -0.37 * lim), (-lim, -lim, lim)]:
        cam = volgen.Camera(eye=eye, center=(31.3, 29.7, 33.1), up=(0.0, 0.0, 1.0), vfov_deg=0.006)
        r = spr.Render(vol, cam, 0.5, 48, 40, spec_cap=8)
        r.run()
        ref = oracle.render(dec, cam, 0.5, 48, 40)
        assert np.isfinite(ref["t"]).sum() > 100
        _cmp_hits(r.hits(), r.image(), ref, f"far eye {eye}")
        r.free()
    vol.free()


@pytest.mark.parametrize("cap", [1, 64])
def test_exact_block_level_ties(ctx, cap):
    """Rays through block corners and along block edges and faces: the centre
    pixel of an odd image looks exactly along the view direction, here
    (1,1,1)/sqrt3 from an integer eye (three planes crossed at one parameter at
    every block corner), (1,0,0) on the planes y = 8, z = 12 (two parallel axes
    on block planes) and (1,1,0)/sqrt2 (x and y planes crossed together).  The
    image and every pass counter equal the oracle's."""
    from paper_2309_10212_amd import spr
    n = 48
    s = volgen.encode(volgen.blobs(n, n, n, 4), 8)
    dec = oracle.decode_volume(s, (n, n, n), 8)
    vol = ctx.load_volume(s, (n, n, n), 8)
    cams = [volgen.Camera(eye=(-8.0, -8.0, -8.0), center=(40.0, 40.0, 40.0), up=(0.0, 0.0, 1.0), vfov_deg=40.0),
            volgen.Camera(eye=(-5.0, 8.0, 12.0), center=(30.0, 8.0, 12.0), up=(0.0, 1.0, 0.0), vfov_deg=40.0),
            volgen.Camera(eye=(-8.0, -8.0, 20.0), center=(40.0, 40.0, 20.0), up=(0.0, 0.0, 1.0), vfov_deg=40.0)]
    for ci, cam in enumerate(cams):
        d, _, _, _ = oracle.ray((n, n, n), cam, 33, 33, 16, 16)
        assert (d[0] == d[1] == d[2]) if ci == 0 else (d[1] == d[2] == 0.0 if ci == 1 else (d[0] == d[1] and d[2] == 0.0))
        r = spr.Render(vol, cam, 0.5, 33, 33, spec_cap=cap)
        sched = oracle.schedule(dec, cam, 0.5, 33, 33, cap)
        got = []
        while not r.done():
            got.append(r.pass_(stats=True))
            assert len(got) <= len(sched) + 2
        _cmp_hits(r.hits(), r.image(), oracle.render(dec, cam, 0.5, 33, 33), f"tie camera {ci} cap {cap}")
        assert len(got) == len(sched)
        for p, (g, o) in enumerate(zip(got, sched)):
            for k in ("n_active", "n_spec", "pairs", "visible", "active_blocks", "terminated"):
                assert g[k] == o[k], (ci, p, k, g, o)
        r.free()
    vol.free()


def test_ragged_volume_inside_camera_and_edges(ctx):
    from paper_2309_10212_amd import spr
    dims = (37, 29, 23)
    f = volgen.fourier(*dims, seed=9, nmode=16, kmax=5)
    s = volgen.encode(f, 4)
    dec = oracle.decode_volume(s, dims, 4)
    iso = volgen.percentile_value(dec, 0.5)
    vol = ctx.load_volume(s, dims, 4)
    cams = [volgen.orbit_camera(*dims, seed=3), volgen.Camera(eye=(18.0, 14.0, 11.0), center=(36.0, 0.0, 22.0),
                                                                up=(0.0, 0.0, 1.0), vfov_deg=70.0),
            volgen.Camera(eye=(-5.0, 14.0, 11.0), center=(18.0, 14.0, 11.0), up=(0.0, 1.0, 0.0), vfov_deg=30.0)]
    for ci, cam in enumerate(cams):
        for (w, h, cap) in [(61, 47, 64), (1, 1, 4), (33, 17, 1)]:
            r = spr.Render(vol, cam, iso, w, h, spec_cap=cap)
            r.run()
            ref = oracle.render(dec, cam, iso, w, h)
            _cmp_hits(r.hits(), r.image(), ref, f"cam{ci} {w}x{h} cap{cap}")
            r.free()
    vol.free()


def test_empty_renders(ctx):
    from paper_2309_10212_amd import spr
    s, dec, cam = _tiny()
    vol = ctx.load_volume(s, (64, 64, 64), 8)
    away = volgen.Camera(eye=(-100.0, -100.0, -100.0), center=(-200.0, -150.0, -100.0), up=(0.0, 0.0, 1.0))
    r = spr.Render(vol, away, 0.5, 32, 32)
    assert r.done() and r.run() == 0
    assert not np.isfinite(r.hits()["t"]).any() and not r.image().any()
    r.free()
    r = spr.Render(vol, cam, 1e6, 32, 32)      # isovalue above every sample: no candidate blocks
    passes = r.run()
    assert passes == 1 and not np.isfinite(r.hits()["t"]).any()
    r.free()
    vol.free()


def test_speculation_and_cache_size_do_not_change_the_image(ctx):
    from paper_2309_10212_amd import spr
    s, dec, cam = _tiny()
    vol = ctx.load_volume(s, (64, 64, 64), 8)
    outs = []
    for cap in (1, 3, 64):
        r = spr.Render(vol, cam, 0.5, 128, 96, spec_cap=cap)
        r.run()
        outs.append((r.hits(), r.image()))
        r.free()
    vol.free()
    small = spr.Context(device=0, cache_bytes=256 * 40)    # 40 slots: 5 blocks served per pass
    vol2 = small.load_volume(s, (64, 64, 64), 8)
    r = spr.Render(vol2, cam, 0.5, 128, 96, spec_cap=8)
    deferred = 0
    passes = 0
    while not r.done():
        st = r.pass_(stats=True)
        deferred += st["deferred"]
        passes += 1
        assert st["active_blocks"] <= 40
        assert passes < 5000, "no progress under deferral"
    outs.append((r.hits(), r.image()))
    assert deferred > 0
    r.free()
    vol2.free()
    small.close()
    h0, i0 = outs[0]
    for h1, i1 in outs[1:]:
        assert np.array_equal(h0.view(np.uint8), h1.view(np.uint8))
        assert np.array_equal(i0, i1)


def test_cache_too_small_for_one_block_is_rejected():
    from paper_2309_10212_amd import spr
    with pytest.raises(spr.SprError) as e:
        spr.Context(device=0, cache_bytes=256 * 7)
    assert e.value.status == -5


def test_kept_isovalue_mask_sets(ctx):
    """A volume keeps the isovalue masks of up to four isovalues: a render at
    a kept isovalue reads them and their counts, one at a new isovalue takes
    the least recently used set that no live render reads, and while every
    set is read a render builds its own.  Every image equals the oracle's and
    the counts equal the oracle's, whichever path served the masks."""
    from paper_2309_10212_amd import spr
    s, dec, cam = _tiny()
    n, w, h = 64, 96, 80
    vol = ctx.load_volume(s, (n, n, n), 8)
    _, fine, coarse = oracle.grids(dec)
    refs = {}

    def begin(iso, built):
        r = spr.Render(vol, cam, iso, w, h, spec_cap=16)
        info = r.info()
        assert info["masks_built"] == built, (iso, built, info)
        assert info["bcmc_blocks"] == oracle.blocks_containing(fine, iso), iso
        assert info["iso_coarse_cells"] == oracle.blocks_containing(coarse, iso), iso
        return r

    def finish(r, iso, label):
        r.run()
        if iso not in refs:
            refs[iso] = oracle.render(dec, cam, iso, w, h)
        _cmp_hits(r.hits(), r.image(), refs[iso], label)
        r.free()

    # one render at a time: (isovalue, expected masks_built)
    seq = [(0.5, 1), (0.5, 0), (0.3, 1), (0.7, 1), (0.2, 1), (0.5, 0),
           (0.6, 1),            # replaces 0.3, the least recently used set
           (0.3, 1), (0.2, 0), (0.5, 0), (0.6, 0)]   # 0.3 replaces 0.7
    for k, (iso, built) in enumerate(seq):
        finish(begin(iso, built), iso, f"sequential {k} iso {iso}")
    # kept now: 0.5, 0.6, 0.3, 0.2; while renders read all four, new
    # isovalues build private masks and kept ones are still shared
    live = [(iso, begin(iso, 0)) for iso in (0.5, 0.6, 0.3, 0.2)]
    live += [(0.4, begin(0.4, 1)), (0.7, begin(0.7, 1)), (0.5, begin(0.5, 0))]
    for k, (iso, r) in enumerate(live):
        finish(r, iso, f"live {k} iso {iso}")
    finish(begin(0.4, 1), 0.4, "after the live renders")
    # rebuilding the grids drops every kept set
    vol.build_grids()
    finish(begin(0.5, 1), 0.5, "after a grid rebuild")
    finish(begin(0.5, 0), 0.5, "kept again")
    vol.free()


@pytest.mark.parametrize("w,h", [(8, 8), (6, 5)])
def test_small_image_many_misses(ctx, w, h):
    """A small image on a freshly loaded 64^3 Fourier field: the first pass
    misses more blocks (324 and 136) than half of the decode grid's lanes
    (256 and 128 for these images), so the decoding workgroups take several
    blocks per lane while the others list the neighbourhoods.  Every pixel
    and per-pass counter against the oracle."""
    from paper_2309_10212_amd import spr
    n = 64
    f = volgen.fourier(n, n, n, seed=5, nmode=64, kmax=16, period=float(n))
    iso = float(np.percentile(f, 50))
    s = volgen.encode(f, 8)
    dec = oracle.decode_volume(s, (n, n, n), 8)
    cam = volgen.orbit_camera(n, n, n, seed=1)
    vol = ctx.load_volume(s, (n, n, n), 8)
    r = spr.Render(vol, cam, iso, w, h, spec_cap=64)
    got = []
    while not r.done():
        got.append(r.pass_(stats=True))
        assert len(got) < 50
    sched = oracle.schedule(dec, cam, iso, w, h, 64)
    assert len(got) == len(sched)
    assert got[0]["blocks_decoded"] == sched[0]["active_blocks"] > 64 * (((8 * w * h + 63) // 64 + 1) // 2)
    for p, (g, o) in enumerate(zip(got, sched)):
        for k in ("n_active", "n_spec", "pairs", "visible", "active_blocks", "terminated"):
            assert g[k] == o[k], (p, k, g, o)
    _cmp_hits(r.hits(), r.image(), oracle.render(dec, cam, iso, w, h), f"fourier {w}x{h}")
    r.free()
    vol.free()


def test_two_runs_bitwise_identical(ctx):
    from paper_2309_10212_amd import spr
    s, dec, cam = _tiny()
    vol = ctx.load_volume(s, (64, 64, 64), 8)
    res = []
    for _ in range(2):
        r = spr.Render(vol, cam, 0.5, 200, 150, spec_cap=16)
        r.run()
        res.append((r.hits().tobytes(), r.image().tobytes()))
        r.free()
    assert res[0] == res[1]
    vol.free()


def test_batch_equals_alone(ctx):
    from paper_2309_10212_amd import spr
    vols, reqs = [], []
    specs = [((64, 64, 64), 8, "blobs", 1), ((48, 40, 36), 4, "fourier", 2), ((32, 32, 32), 2, "fourier", 3)]
    for dims, rate, kind, seed in specs:
        f = volgen.blobs(*dims, seed) if kind == "blobs" else volgen.fourier(*dims, seed, nmode=16, kmax=6)
        s = volgen.encode(f, rate)
        v = ctx.load_volume(s, dims, rate)
        dec = oracle.decode_volume(s, dims, rate)
        vols.append((v, dec))
    sizes = [(64, 48), (100, 75), (17, 33), (128, 128), (40, 40)]
    for i in range(7):
        vi = i % len(vols)
        v, dec = vols[vi]
        cam = volgen.orbit_camera(*v.dims, seed=100 + i)
        iso = volgen.percentile_value(dec, 0.3 + 0.08 * i)
        w, h = sizes[i % len(sizes)]
        cap = [64, 1, 8, 16][i % 4]
        reqs.append((v, dec, cam, iso, w, h, cap))
    alone = []
    for v, dec, cam, iso, w, h, cap in reqs:
        r = spr.Render(v, cam, iso, w, h, spec_cap=cap)
        r.run()
        alone.append((r.hits(), r.image()))
        r.free()
    rs = [spr.Render(v, cam, iso, w, h, spec_cap=cap) for v, dec, cam, iso, w, h, cap in reqs]
    b = spr.Batch(ctx, rs)
    b.run(poll_every=2)
    for k, r in enumerate(rs):
        h1, i1 = r.hits(), r.image()
        assert np.array_equal(alone[k][0].view(np.uint8), h1.view(np.uint8)), k
        assert np.array_equal(alone[k][1], i1), k
        v, dec, cam, iso, w, h, cap = reqs[k]
        _cmp_hits(h1, i1, oracle.render(dec, cam, iso, w, h), f"batch req {k}")
    b.free()
    for r in rs:
        r.free()
    for v, _ in vols:
        v.free()


@pytest.mark.parametrize("cap", [16, 64])
def test_per_ray_speculation_counters_and_image(ctx, cap):
    """Per-ray speculation counts: every per-pass counter (active rays, slots
    handed out, pairs, visible and active blocks, terminated rays) equals the
    oracle's per-ray schedule, and the image equals the oracle's (and so the
    single-count image)."""
    from paper_2309_10212_amd import spr
    s, dec, cam = _tiny()
    n, w, h, iso = 64, 256, 256, 0.5
    vol = ctx.load_volume(s, (n, n, n), 8)
    r = spr.Render(vol, cam, iso, w, h, spec_cap=cap, policy=spr.SPEC_PER_RAY)
    sched = oracle.schedule(dec, cam, iso, w, h, cap, policy=oracle.POLICY_PER_RAY)
    got = []
    while not r.done():
        got.append(r.pass_(stats=True))
        assert len(got) <= len(sched) + 2
    assert len(got) == len(sched), (len(got), len(sched))
    for p, (g, o) in enumerate(zip(got, sched)):
        for k in ("n_active", "slots", "pairs", "visible", "active_blocks", "terminated"):
            assert g[k] == o[k], (p, k, g, o)
    _cmp_hits(r.hits(), r.image(), oracle.render(dec, cam, iso, w, h), f"per-ray cap={cap}")
    r.free()
    # a batch mixing both policies equals the renders alone
    rs = [spr.Render(vol, cam, iso, 128, 96, spec_cap=cap, policy=pol) for pol in (spr.SPEC_PER_RAY, spr.SPEC_UNIFORM)]
    b = spr.Batch(ctx, rs)
    b.run()
    outs = [(x.hits(), x.image()) for x in rs]
    b.free()
    for x in rs:
        x.free()
    for pol, (hb, ib) in zip((spr.SPEC_PER_RAY, spr.SPEC_UNIFORM), outs):
        ra = spr.Render(vol, cam, iso, 128, 96, spec_cap=cap, policy=pol)
        ra.run()
        assert np.array_equal(ra.hits().view(np.uint8), hb.view(np.uint8)) and np.array_equal(ra.image(), ib)
        ra.free()
    vol.free()


def test_per_ray_speculation_sparse_volume(ctx):
    from paper_2309_10212_amd import spr
    n = 256
    f = volgen.blobs(n, n, n, seed=21, nblob=2)
    s = volgen.encode(f, 8)
    dec = oracle.decode_volume(s, (n, n, n), 8)
    vol = ctx.load_volume(s, (n, n, n), 8)
    cam = volgen.orbit_camera(n, n, n, seed=22)
    r = spr.Render(vol, cam, 0.3, 160, 120, spec_cap=8, policy=spr.SPEC_PER_RAY)   # cap <= 16: segmented walks
    got = []
    while not r.done():
        got.append(r.pass_(stats=True))
        assert len(got) < 400
    sched = oracle.schedule(dec, cam, 0.3, 160, 120, 8, policy=oracle.POLICY_PER_RAY)
    assert len(got) == len(sched)
    for p, (g, o) in enumerate(zip(got, sched)):
        for key in ("n_active", "slots", "pairs", "visible", "active_blocks", "terminated"):
            assert g[key] == o[key], (p, key, g, o)
    _cmp_hits(r.hits(), r.image(), oracle.render(dec, cam, 0.3, 160, 120), "sparse per-ray")
    r.free()
    vol.free()
