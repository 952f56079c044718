"""GPU parity of the batched form (the B workload, on a reduced pool): requests
with mixed volumes (blobs and Fourier fields, float32 and u8 levels, 2, 4 and
8 bits/value) and mixed image sizes, run as one graph-replayed batch under the
tuning the autotuner picks, must equal each request rendered alone under other
launch tuning and speculation caps (hit block, cell and t bitwise, image
bitwise), and a sample of each request's pixels must equal the oracle."""
import numpy as np
import pytest

import oracle
from volgen import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    from paper_2309_10212_amd import spr
    pool = workloads.make_pool(sizes=(128, 256))
    reqs = workloads.make_requests(pool, count=12, sizes=[(256, 256), (640, 360), (512, 512)])
    ctx = spr.Context(device=0, cache_bytes=512 * 10**6, spec_cap=16)
    vols = [ctx.load_volume(p.stream, p.dims, p.rate) for p in pool]
    yield pool, reqs, ctx, vols
    for v in vols:
        v.free()
    ctx.close()


def test_pool_and_requests_are_mixed(setup):
    pool, reqs, _, _ = setup
    assert len(pool) == 4
    assert {p.dtype for p in pool} >= {"f32"} and len({p.rate for p in pool}) >= 2
    assert len({(q.w, q.h) for q in reqs}) >= 2 and len({q.vol for q in reqs}) >= 3


def test_batched_equals_alone_and_oracle(setup):
    from paper_2309_10212_amd import autotune, spr
    pool, reqs, ctx, vols = setup
    best, table = autotune.autotune(ctx, vols, reqs, caps=(4, 64), tiles=((256, 0), (256, 32)), sample=4)
    assert len(table) == 4 and best in table
    print(f"autotuned: cap {best.spec_cap}, {best.pairs_per_wg} pairs/wg, slot tile {best.slot_tile}, "
          f"{best.rays_per_s / 1e6:.1f} Mrays/s", flush=True)
    _, rays, passes, batched = autotune.run_batch(ctx, vols, reqs, best.spec_cap)
    assert rays > 0 and passes > 0
    ctx.set_tuning(256, 0 if best.slot_tile else 16)   # the renders alone under another raytrace variant
    for i, (q, rb) in enumerate(zip(reqs, batched)):
        cap = 1 if i % 3 == 0 else 64
        ra = spr.Render(vols[q.vol], q.cam, q.iso, q.w, q.h, spec_cap=cap)
        ra.run()
        hb, ha = rb.hits(), ra.hits()
        assert np.array_equal(hb.view(np.uint8), ha.view(np.uint8)), i
        assert np.array_equal(rb.image(), ra.image()), i
        ra.free()
        pv = pool[q.vol]
        dec = oracle.decode_volume(pv.stream, pv.dims, pv.rate)
        pix = np.random.default_rng(i).choice(q.w * q.h, 1500, replace=False).astype(np.uint32)
        ref = oracle.render(dec, q.cam, q.iso, q.w, q.h, pixels=pix)
        g = hb[pix]
        fin = np.isfinite(ref["t"])
        assert np.array_equal(np.isfinite(g["t"]), fin), i
        assert np.array_equal(g["block"], ref["block"]), i
        assert np.array_equal(g["cell"], ref["cell"]), i
        if fin.any():
            assert float(np.abs(g["t"][fin] - ref["t"][fin]).max()) <= 1e-4, i
        img = rb.image().reshape(-1, 4).astype(np.int32)
        o = ref["rgba"].view(np.uint8).reshape(-1, 4).astype(np.int32)
        assert np.abs(img[pix] - o).max() <= 1, i
        rb.free()
    ctx.set_tuning(256, 0)


def test_tuning_rejects_unsupported_values(setup):
    from paper_2309_10212_amd import spr
    _, _, ctx, _ = setup
    with pytest.raises(spr.SprError):
        ctx.set_tuning(192, 32)
    with pytest.raises(spr.SprError):
        ctx.set_tuning(256, 8)
    assert ctx.tuning() == {"pairs_per_wg": 256, "slot_tile": 0}
