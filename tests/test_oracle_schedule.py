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
