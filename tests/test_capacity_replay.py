"""Host-side replay of the pass's index spaces and buffer capacities (no GPU).

For the pass schedules the oracle computes (per pass: active rays, the
speculation count, slots handed out, pairs, visible and active blocks), the
library's sizing rules are replayed in Python and every index the kernels can
form is checked against the buffer it addresses:

  - pair slots: each request's slot range (N_act * N_spec, or the per-ray
    counts' sum) within its w*h entries of pair_blk / tslot / pair_ray;
  - the active-ray space (64-aligned) within the request's padded pixels;
  - traversal lanes: the segment rule of the pass set-up kernel, the LDS
    candidate buffer (TR_BUF entries per lane) and, for segmented lanes with
    more slots than that, the rows of the column buffer (SEG_BIG_NS entries,
    SEG_BIG_LANES lanes);
  - the pass workspace: visible list within cap_P = w*h entries, active and
    miss lists within cap_K = 8 * cap_P.

The constants are read from the kernel sources, so the replay follows them.
The renders are cases of the GPU parity tests: the tiny blob volume at
speculation caps 1, 3 and 64 and with per-ray counts, and the sparse volume
with its empty-space jumps."""
import os
import re

import pytest

import oracle
import volgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2309_10212_amd", "csrc")


def _const(name):
    src = open(os.path.join(CSRC, "spr_kernels.hip")).read() + open(os.path.join(CSRC, "spr_internal.h")).read()
    m = re.search(r"constexpr\s+(?:uint32_t|int)\s+" + name + r"\s*=\s*(\d+)\s*;", src)
    assert m, name
    return int(m.group(1))


TR_BUF, SEG_TARGET = _const("TR_BUF"), _const("SEG_TARGET")
SEG_BIG_LANES, SEG_BIG_NS = _const("SEG_BIG_LANES"), _const("SEG_BIG_NS")


def round64(x):
    return (x + 63) // 64 * 64


def pow2_segments(budget, all_na):
    """The set-up kernel's rule: a power of two up to 16 with 2 * segs <= budget / all_na."""
    segs = 1
    if all_na > 0:
        want = budget // all_na
        while segs < 16 and 2 * segs <= want:
            segs *= 2
    return segs


def replay(sched, w, h, cap, policy):
    npix = w * h
    cap_P, cap_K = npix, 8 * npix
    for p, s in enumerate(sched):
        na, ns = s["n_active"], s["n_spec"]
        slots = s["slots"]
        # slots handed out lie inside the request's w*h pair entries
        if policy == oracle.POLICY_UNIFORM:
            assert slots == na * ns, (p, s)
        assert slots <= npix, (p, s)
        # active-ray space of the request
        assert round64(na) <= round64(npix)
        # traversal lanes
        most = cap if policy == oracle.POLICY_PER_RAY else ns
        seg_ok, big_ok = most <= TR_BUF, TR_BUF < most <= SEG_BIG_NS
        segs = pow2_segments(SEG_TARGET, na) if seg_ok else (pow2_segments(SEG_BIG_LANES, na) if big_ok else 1)
        if na == 0:
            segs = 1
        if segs > 1:
            # a segmented lane lists at most its ray's count: the LDS buffer, or the column buffer's rows
            assert most <= (TR_BUF if seg_ok else SEG_BIG_NS), (p, most)
            if big_ok:
                assert na * segs <= SEG_BIG_LANES, (p, na, segs)
        # pass workspace
        assert s["pairs"] <= slots
        assert s["visible"] <= s["pairs"] <= cap_P, (p, s)
        assert s["active_blocks"] <= 8 * s["visible"] <= cap_K, (p, s)


def _tiny():
    n = 64
    dec = oracle.decode_volume(volgen.encode(volgen.blobs(n, n, n, seed=1), 8), (n, n, n), 8)
    return dec, volgen.orbit_camera(n, n, n, seed=1)


@pytest.mark.parametrize("cap", [1, 3, 64])
def test_tiny_render_index_spaces(cap):
    dec, cam = _tiny()
    sched = oracle.schedule(dec, cam, 0.5, 256, 256, cap)
    assert len(sched) > 1
    replay(sched, 256, 256, cap, oracle.POLICY_UNIFORM)
    if cap == 64:
        # the last pass has few rays and more slots each than the LDS buffer holds: segmented
        # walks with the column buffer
        assert any(0 < s["n_active"] and s["n_spec"] > TR_BUF for s in sched)


@pytest.mark.parametrize("cap", [16, 64])
def test_tiny_render_per_ray_counts_index_spaces(cap):
    dec, cam = _tiny()
    sched = oracle.schedule(dec, cam, 0.5, 256, 256, cap, policy=oracle.POLICY_PER_RAY)
    replay(sched, 256, 256, cap, oracle.POLICY_PER_RAY)


def test_sparse_volume_segmented_walks_index_spaces():
    n = 128
    dec = oracle.decode_volume(volgen.encode(volgen.blobs(n, n, n, seed=21, nblob=2), 8), (n, n, n), 8)
    for k in range(2):
        cam = volgen.orbit_camera(n, n, n, seed=21 + k)
        for cap in (1, 64):
            sched = oracle.schedule(dec, cam, 0.3, 160, 120, cap)
            replay(sched, 160, 120, cap, oracle.POLICY_UNIFORM)


def test_replay_catches_an_oversized_pass():
    """The replay is not vacuous: a schedule whose slots exceed w*h fails."""
    bad = [{"n_active": 100, "n_spec": 3, "slots": 300, "pairs": 10, "visible": 5, "active_blocks": 9,
            "terminated": 0, "wsum": 0}]
    with pytest.raises(AssertionError):
        replay(bad, 16, 16, 64, oracle.POLICY_UNIFORM)
