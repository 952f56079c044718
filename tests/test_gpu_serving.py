"""The serving loop (continuous batching with admission by cache memory) on a
short Poisson arrival stream over two resident volumes: requests overlap on
the device, every request completes, and each served result equals the same
request rendered alone (hit records and image bitwise); a sample also equals
the oracle."""
import dataclasses

import numpy as np
import pytest

import oracle
import volgen
from volgen import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def served():
    from paper_2309_10212_amd import serve, spr
    fields = [volgen.blobs(64, 64, 64, seed=1), volgen.fourier(128, 128, 128, seed=4, nmode=32, kmax=12, period=128.0)]
    rates = [8, 4]
    streams = [volgen.encode(f, r) for f, r in zip(fields, rates)]
    ranges = [(volgen.percentile_value(f, 0.2), volgen.percentile_value(f, 0.8)) for f in fields]
    dims = [f.shape[::-1] for f in fields]
    arr = workloads.serving_arrivals(dims, ranges, lam=400.0, span_s=0.25, seed=7)
    # small images keep the test short; the arrival times and camera/iso mix are the recipe's
    arr = [dataclasses.replace(a, w=256 if a.w == 1280 else 320, h=144 if a.w == 1280 else 180) for a in arr]
    ctx = spr.Context(device=0, cache_bytes=64 * 10**6, spec_cap=16)
    vols = [ctx.load_volume(s, d, r) for s, d, r in zip(streams, dims, rates)]
    srv = serve.Server(ctx, vols, cache_bytes=64 * 10**6, max_requests=16, max_pixels=16 * 320 * 180)
    results, stats = srv.run(arr, keep_results=True)
    print({k: (round(v, 3) if isinstance(v, float) else v) for k, v in stats.items()}, flush=True)
    yield arr, results, stats, ctx, vols, streams, dims, rates
    srv.close()
    for v in vols:
        v.free()
    ctx.close()


def test_every_request_completes_and_requests_overlap(served):
    arr, results, stats, *_ = served
    assert len(arr) > 50
    assert all(r is not None for r in results)
    assert stats["max_concurrent"] > 1
    assert stats["pass_latency_ms_p99"] >= stats["pass_latency_ms_p50"] > 0
    for r in results:
        assert r.finished >= r.admitted >= 0 and len(r.latencies) >= r.passes


def test_served_results_equal_alone_and_oracle(served):
    from paper_2309_10212_amd import spr
    arr, results, _, ctx, vols, streams, dims, rates = served
    decoded = [oracle.decode_volume(s, d, r) for s, d, r in zip(streams, dims, rates)]
    for i in range(0, len(arr), 4):
        a, res = arr[i], results[i]
        r = spr.Render(vols[a.vol], a.cam, a.iso, a.w, a.h, spec_cap=(1 if i % 8 == 0 else 64))
        r.run()
        assert np.array_equal(r.hits().view(np.uint8), res.hits.view(np.uint8)), i
        assert np.array_equal(r.image(), res.image), i
        r.free()
        if i % 16 == 0:
            pix = np.random.default_rng(i).choice(a.w * a.h, 800, replace=False).astype(np.uint32)
            ref = oracle.render(decoded[a.vol], a.cam, a.iso, a.w, a.h, pixels=pix)
            g = res.hits[pix]
            assert np.array_equal(g["block"], ref["block"]), i
            assert np.array_equal(g["cell"], ref["cell"]), i
            fin = np.isfinite(ref["t"])
            if fin.any():
                assert float(np.abs(g["t"][fin] - ref["t"][fin]).max()) <= 1e-4, i
