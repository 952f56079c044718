"""Pins of the oracle's progressive pass schedule (Sec. 3 passes, Sec. 4
speculation): the worked example of the traversal/speculation figure, the
speculation-count definition, and consistency between the pass schedule and
the per-pixel march (speculation only adds ray-block tests; every ray that
entered terminates exactly once; hit rays terminate in the pass that
reaches their hit block)."""
import json
import os

import numpy as np
import pytest

import oracle
import volgen

GOLD = os.path.join(os.path.dirname(__file__), "golden", "traversal_speculation_example.json")


def test_nspec_definition():
    assert oracle.nspec(6, 4, 64) == 1      # first pass of the figure
    assert oracle.nspec(6, 2, 64) == 3      # second pass of the figure
    assert oracle.nspec(921600, 1, 64) == 64   # capped at 64
    assert oracle.nspec(100, 101, 64) == 1  # at least one block per ray
    assert oracle.nspec(10, 0, 64) == 0


def test_figure_worked_example():
    g = json.load(open(GOLD))
    rays = g["rays"]
    lists = [r["candidates"] for r in rays]
    hit = [r["hit_index"] for r in rays]
    ent = [r["entered"] for r in rays]
    spec = oracle.schedule_lists(g["slots"], lists, hit, ent, g["nb_dims"], spec_cap=64)
    e = g["expected_with_speculation"]
    assert len(spec) == e["passes"]
    assert [p["n_spec"] for p in spec] == e["n_spec"]
    assert [p["n_active"] for p in spec] == e["n_active"]
    assert [p["pairs"] for p in spec] == e["pairs"]
    assert spec[1]["pairs"] / g["slots"] == pytest.approx(e["utilization_pass2"])
    nos = oracle.schedule_lists(g["slots"], lists, hit, ent, g["nb_dims"], spec_cap=1)
    e = g["expected_without_speculation"]
    assert len(nos) == e["passes"]
    assert [p["n_spec"] for p in nos] == e["n_spec"]
    assert [p["n_active"] for p in nos] == e["n_active"]
    # pass one is identical with and without speculation
    assert spec[0] == nos[0]


def test_active_blocks_are_visible_plus_positive_neighbours():
    # one ray, one visible block in the middle of a 4^3 block grid -> 8 active;
    # a block on the +x/+y/+z corner of the grid has no + neighbours -> 1 active
    s = oracle.schedule_lists(1, [[21]], [0], [True], (4, 4, 4), 1)
    assert s[0]["visible"] == 1 and s[0]["active_blocks"] == 8
    s = oracle.schedule_lists(1, [[63]], [0], [True], (4, 4, 4), 1)
    assert s[0]["active_blocks"] == 1
    s = oracle.schedule_lists(1, [[15]], [0], [True], (4, 4, 4), 1)   # (3,3,0): only +z exists
    assert s[0]["active_blocks"] == 2


@pytest.mark.parametrize("cap", [1, 4, 64])
def test_schedule_consistent_with_march(cap):
    n = 32
    field = volgen.blobs(n, n, n, seed=1)
    vol = oracle.decode_volume(volgen.encode(field, 8), (n, n, n), 8)
    cam = volgen.orbit_camera(n, n, n, seed=1)
    w = h = 48
    iso = 0.5
    sched = oracle.schedule(vol, cam, iso, w, h, cap)
    r = oracle.render(vol, cam, iso, w, h)
    entered = sum(oracle.ray((n, n, n), cam, w, h, p % w, p // w)[3] for p in range(w * h))
    assert sched[0]["n_active"] == entered
    assert sum(p["terminated"] for p in sched) == entered
    for a, b in zip(sched, sched[1:]):
        assert b["n_active"] == a["n_active"] - a["terminated"]
    for p in sched:
        assert p["n_spec"] == oracle.nspec(w * h, p["n_active"], cap)
        assert p["pairs"] <= w * h
        assert p["visible"] <= p["pairs"] and p["active_blocks"] <= 8 * p["visible"]
    assert np.isfinite(r["t"]).sum() > 0


def test_speculation_reduces_passes_and_keeps_pair_budget():
    n = 32
    field = volgen.fourier(n, n, n, seed=2, nmode=16, kmax=6)
    vol = oracle.decode_volume(volgen.encode(field, 4), (n, n, n), 4)
    iso = volgen.percentile_value(vol, 0.6)
    cam = volgen.orbit_camera(n, n, n, seed=2)
    s1 = oracle.schedule(vol, cam, iso, 40, 30, 1)
    s16 = oracle.schedule(vol, cam, iso, 40, 30, 16)
    assert len(s16) < len(s1)
    assert sum(p["terminated"] for p in s1) == sum(p["terminated"] for p in s16)
    assert sum(p["pairs"] for p in s16) >= sum(p["pairs"] for p in s1)


# --------------------------------------------------- per-ray speculation ----
# The per-ray count (the paper's conclusion names a per-ray speculation count
# as future work): n_i = min(cap, 1 + floor((B - N) w_i / W)), weights from
# each ray's remaining path.  Pinned by a worked example, by the reduction to
# Sec. 4's count when all weights are equal, by the slot budget, and by the
# weights against the ray geometry computed here.

GOLD_PR = os.path.join(os.path.dirname(__file__), "golden", "per_ray_speculation_example.json")


def test_per_ray_worked_example():
    g = json.load(open(GOLD_PR))
    rays = g["rays"]
    s = oracle.schedule_lists(g["slots"], [r["candidates"] for r in rays], [r["hit_index"] for r in rays],
                              [True] * len(rays), g["nb_dims"], g["cap"], policy=oracle.POLICY_PER_RAY,
                              w0=[r["w0"] for r in rays], wk=[r["wk"] for r in rays])
    e = g["expected"]
    assert len(s) == e["passes"]
    for key in ("n_active", "wsum", "slots", "n_spec", "pairs", "terminated"):
        assert [p[key] for p in s] == e[key], key
    # every candidate block is distinct here, so the visible blocks are the pairs
    assert [p["visible"] for p in s] == e["pairs"]


def test_per_ray_count_definition():
    assert oracle.nspec_ray(12, 4, 14, 7, 64) == 5
    assert oracle.nspec_ray(12, 4, 14, 1, 64) == 1
    assert oracle.nspec_ray(921600, 10, 10, 1, 64) == 64          # capped
    assert oracle.nspec_ray(100, 100, 500, 499, 64) == 1         # no slot beyond one each
    # equal weights give Sec. 4's count
    for B, N in ((921600, 3), (65536, 65536), (1000, 7), (6, 4)):
        for w in (1, 5, 113):
            assert oracle.nspec_ray(B, N, N * w, w, 64) == oracle.nspec(B, N, 64)
    assert oracle.ray_weight(10.0, 10.0) == 1 and oracle.ray_weight(11.0, 10.0) == 1
    assert oracle.ray_weight(0.0, 3.999) == 1 and oracle.ray_weight(0.0, 4.0) == 2
    assert oracle.ray_weight(1.5, 10.0) == 3


def test_per_ray_equal_weights_reduce_to_uniform():
    rng = np.random.default_rng(3)
    lists, hits = [], []
    for i in range(40):
        n = int(rng.integers(0, 30))
        lists.append(list(rng.integers(0, 512, n)))
        hits.append(int(rng.integers(-1, n)) if n else -1)
    ent = [True] * 40
    uni = oracle.schedule_lists(64, lists, hits, ent, (8, 8, 8), 64)
    pr = oracle.schedule_lists(64, lists, hits, ent, (8, 8, 8), 64, policy=oracle.POLICY_PER_RAY,
                               w0=[9] * 40, wk=[[9] * len(l) for l in lists])
    assert len(pr) == len(uni)
    for a, b in zip(uni, pr):
        for key in ("n_active", "n_spec", "pairs", "visible", "active_blocks", "terminated", "slots"):
            assert a[key] == b[key], key


@pytest.mark.parametrize("cap", [4, 64])
def test_per_ray_schedule_invariants(cap):
    n = 32
    field = volgen.blobs(n, n, n, seed=1)
    vol = oracle.decode_volume(volgen.encode(field, 8), (n, n, n), 8)
    cam = volgen.orbit_camera(n, n, n, seed=1)
    w = h = 48
    uni = oracle.schedule(vol, cam, 0.5, w, h, cap)
    pr = oracle.schedule(vol, cam, 0.5, w, h, cap, policy=oracle.POLICY_PER_RAY)
    assert pr[0]["n_active"] == uni[0]["n_active"]
    assert sum(p["terminated"] for p in pr) == uni[0]["n_active"]
    for a, b in zip(pr, pr[1:]):
        assert b["n_active"] == a["n_active"] - a["terminated"]
    for p in pr:
        assert p["n_active"] <= p["slots"] <= w * h           # at least one slot each, within the budget
        assert p["pairs"] <= p["slots"] and p["n_spec"] <= cap
    # every ray's candidates are served in order either way, so the candidate pairs add up the same
    # until each ray terminates: the per-ray schedule serves at most what a ray has
    assert sum(p["pairs"] for p in pr) <= sum(p["pairs"] for p in uni) + w * h * len(pr)


def test_per_ray_weights_from_the_ray_geometry():
    """The weight after a candidate block is 1 + floor((t_exit - t) / 4), t the
    parameter where the ray leaves that block: computed here from the ray and
    the block's exit planes (block planes at 4m, the last one of an axis at the
    domain face n-1)."""
    n = 40
    field = volgen.fourier(n, n, n, seed=5, nmode=12, kmax=4)
    vol = oracle.decode_volume(volgen.encode(field, 8), (n, n, n), 8)
    iso = float(np.quantile(vol, 0.5))
    cam = volgen.orbit_camera(n, n, n, seed=5)
    w, h = 24, 20
    nb = (n + 3) // 4
    tb = (n - 1 + 3) // 4
    checked = 0
    for p in range(0, w * h, 7):
        d, te, tx, ent = oracle.ray((n, n, n), cam, w, h, p % w, p // w)
        lst, wl, w0, hit = oracle.pixel_candidates(vol, cam, iso, w, h, p % w, p // w)
        if not ent:
            assert len(lst) == 0
            continue
        assert w0 == oracle.ray_weight(te, tx) == (1 + int(np.floor((tx - te) * 0.25)) if te < tx else 1)
        eye = np.array(cam.eye)
        for b, wk in zip(lst, wl):
            bc = (int(b) % nb, (int(b) // nb) % nb, int(b) // (nb * nb))
            t_out = np.inf
            for a in range(3):
                if d[a] == 0:
                    continue
                m = bc[a] + 1 if d[a] > 0 else bc[a]
                pos = n - 1 if m >= tb else 4 * m
                t_out = min(t_out, (pos - eye[a]) * (1.0 / d[a]))
            want = 1 if not t_out < tx else 1 + int(np.floor((tx - t_out) * 0.25))
            assert wk == want, (p, b, wk, want)
            checked += 1
    assert checked > 50
