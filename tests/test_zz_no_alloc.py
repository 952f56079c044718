"""The allocation-free decode entry point (spr_debug_decode_blocks_noalloc)
through the C ABI: bitwise equal to spr_debug_decode_blocks (and so to the
oracle's decoder) on two calls in a row, the second with fewer blocks than
the first; no allocator call and no change of device memory during either;
sizes beyond its limit and ids outside the volume rejected."""
import numpy as np
import pytest

import oracle
import volgen

pytestmark = pytest.mark.gpu


class CountingAllocator:
    """torch's caching allocator behind counters."""

    def __init__(self):
        import torch
        self.torch = torch
        self.allocs = self.frees = 0

    def alloc(self, nbytes):
        self.allocs += 1
        return self.torch.cuda.caching_allocator_alloc(nbytes, 0, self.torch.cuda.current_stream(0))

    def free(self, p, nbytes):
        self.frees += 1
        self.torch.cuda.caching_allocator_delete(p)


@pytest.mark.parametrize("dims,rate,kind", [((40, 36, 44), 8, "blobs"), ((64, 64, 64), 4, "fourier"),
                                            ((24, 24, 24), 32, "blobs")])
def test_noalloc_decode_equals_the_allocating_decode(dims, rate, kind):
    from paper_2309_10212_amd import spr
    f = volgen.blobs(*dims, seed=5) if kind == "blobs" else volgen.fourier(*dims, seed=6)
    s = volgen.encode(f, rate)
    ca = CountingAllocator()
    ctx = spr.Context(device=0, cache_bytes=1 << 20, alloc_hooks=(ca.alloc, ca.free))
    vol = ctx.load_volume(s, dims, rate)
    nb = vol.nblocks
    rng = np.random.default_rng(11)
    # first call: the largest size the entry point takes (ids repeat), second: fewer blocks
    sizes = [spr.NOALLOC_MAX_BLOCKS, 37]
    for n in sizes:
        ids = rng.integers(0, nb, n).astype(np.uint32)
        ids[:min(n, nb)] = np.arange(min(n, nb), dtype=np.uint32)   # every block at least once when n >= nb
        ref = vol.decode_blocks(ids)
        a0, f0, cur0 = ca.allocs, ca.frees, ctx.mem_split()["total"]
        got = vol.decode_blocks_noalloc(ids)
        assert (ca.allocs, ca.frees, ctx.mem_split()["total"]) == (a0, f0, cur0), "the entry point allocated"
        assert got.shape == (n, 64)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), f"n={n}: differs from the allocating decode"
        orc = oracle.decode_blocks(s, dims, rate, ids)
        assert np.array_equal(got.view(np.uint32), orc.view(np.uint32)), f"n={n}: differs from the oracle"
    vol.free()
    ctx.close()


def test_noalloc_rejects_sizes_beyond_its_limit_and_bad_ids():
    from paper_2309_10212_amd import spr
    n = 32
    s = volgen.encode(volgen.blobs(n, n, n, seed=1), 8)
    ctx = spr.Context(device=0, cache_bytes=1 << 20)
    vol = ctx.load_volume(s, (n, n, n), 8)
    with pytest.raises(spr.SprError) as e:
        vol.decode_blocks_noalloc(np.zeros(spr.NOALLOC_MAX_BLOCKS + 1, np.uint32))
    assert e.value.status == -5
    with pytest.raises(spr.SprError) as e:
        vol.decode_blocks_noalloc(np.array([0, vol.nblocks], np.uint32))
    assert e.value.status == -1
    assert vol.decode_blocks_noalloc(np.zeros(0, np.uint32)).shape == (0, 64)
    # still usable after the rejected calls
    ids = np.arange(vol.nblocks, dtype=np.uint32)
    assert np.array_equal(vol.decode_blocks_noalloc(ids).view(np.uint32), vol.decode_blocks(ids).view(np.uint32))
    vol.free()
    ctx.close()
