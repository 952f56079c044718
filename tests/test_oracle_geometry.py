"""Pins of the oracle's camera rays, slab test and dual-cell walk
(Sec. 3.2 initial rays, Sec. 3.3 Amanatides-Woo traversal).

The walk is pinned against a DDA-free brute force: every dual cell's box is
intersected with the ray in exact rational arithmetic (on the same fp64
origin and direction), the cells with a positive-length intersection are
sorted by entry parameter, and the sequence must equal the walk's.  Rays
through grid edges (ties) use the reading that tied planes are crossed
together, so the zero-length corner cells are not visited; the exact
enumeration drops them too.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
import volgen


def _exact_cells(dims, eye, d):
    """Cells with a positive-length exact intersection, sorted by entry t."""
    nx, ny, nz = dims
    o = [Fraction(v) for v in eye]
    dd = [Fraction(v) for v in d]
    n = (nx, ny, nz)

    def slab(a, lo, hi):
        if dd[a] == 0:
            return (None, None) if lo <= o[a] <= hi else (1, 0)
        t1 = (lo - o[a]) / dd[a]
        t2 = (hi - o[a]) / dd[a]
        return (min(t1, t2), max(t1, t2))

    # whole domain
    te, tx = Fraction(0), None
    for a in range(3):
        lo_, hi_ = slab(a, 0, n[a] - 1)
        if lo_ is None:
            continue
        if lo_ == 1 and hi_ == 0:
            return []
        te = max(te, lo_)
        tx = hi_ if tx is None else min(tx, hi_)
    if tx is None or te > tx:
        return []
    out = []
    per_axis = []
    for a in range(3):
        rng = []
        for m in range(n[a] - 1):
            lo_, hi_ = slab(a, m, m + 1)
            if lo_ == 1 and hi_ == 0:
                continue
            rng.append((m, lo_, hi_))
        per_axis.append(rng)
    for (i, xl, xh) in per_axis[0]:
        for (j, yl, yh) in per_axis[1]:
            for (k, zl, zh) in per_axis[2]:
                t0, t1 = te, tx
                for lo_, hi_ in ((xl, xh), (yl, yh), (zl, zh)):
                    if lo_ is not None:
                        t0 = max(t0, lo_)
                        t1 = min(t1, hi_)
                if t1 > t0:
                    out.append((t0, (i, j, k)))
    out.sort()
    return [c for _, c in out]


def _random_cams(seed, n, dims):
    rng = np.random.default_rng(seed)
    nx, ny, nz = dims
    cams = []
    for _ in range(n):
        c = volgen.Camera(eye=tuple(rng.uniform(-8, 20, 3)),
                          center=tuple(rng.uniform(0, 1, 3) * (np.array(dims) - 1)),
                          up=(0.0, 0.0, 1.0), vfov_deg=float(rng.uniform(20, 80)))
        cams.append(c)
    return cams


@pytest.mark.parametrize("dims", [(8, 8, 8), (11, 7, 9), (2, 5, 3)])
def test_cell_walk_equals_exact_box_enumeration(dims):
    checked = [0]
    for cam in _random_cams(sum(dims) * 7 + dims[0], 12, dims):
        for px, py in [(x, y) for x in range(8) for y in range(6)]:
            got = oracle.cell_walk(dims, cam, 8, 6, px, py)
            d, te, tx, entered = oracle.ray(dims, cam, 8, 6, px, py)
            ref = _exact_cells(dims, cam.eye, d)
            if got is None:
                assert ref == [] and not entered
                continue
            cells, t01, _ = got
            seq = [tuple(int(v) for v in c) for c in cells]
            # a ray grazing an edge can have only zero-length exact cells
            if ref or len(seq) > 1:
                assert seq == ref, (cam, px, py)
                checked[0] += 1
    assert checked[0] > 40


def test_cell_walk_through_edges_takes_diagonal_steps():
    # eye on integer coordinates, direction exactly (1,1,0)/sqrt2 in fp64:
    # x and y planes are crossed at identical parameters.
    dims = (8, 8, 8)
    cam = volgen.Camera(eye=(-2.0, -2.0, 3.5), center=(5.0, 5.0, 3.5), up=(0.0, 0.0, 1.0), vfov_deg=30.0)
    # centre pixel of an odd image looks exactly along fwd
    cells, t01, _ = oracle.cell_walk(dims, cam, 9, 9, 4, 4)
    d, _, _, _ = oracle.ray(dims, cam, 9, 9, 4, 4)
    assert d[0] == d[1] and d[2] == 0.0
    seq = [tuple(int(v) for v in c) for c in cells]
    assert seq == [(i, i, 3) for i in range(7)]
    assert seq == _exact_cells(dims, cam.eye, d)


def test_cell_intervals_match_exact_values():
    dims = (9, 9, 9)
    cam = volgen.Camera(eye=(-4.3, 2.2, 14.1), center=(4.0, 4.0, 4.0), up=(0.0, 0.0, 1.0), vfov_deg=40.0)
    cells, t01, (te, tx) = oracle.cell_walk(dims, cam, 5, 5, 2, 1)
    d, te2, tx2, _ = oracle.ray(dims, cam, 5, 5, 2, 1)
    assert (te, tx) == (te2, tx2)
    o = [Fraction(v) for v in cam.eye]
    dd = [Fraction(v) for v in d]
    for (i, j, k), (t0, t1) in zip(cells, t01):
        lo, hi = Fraction(te), Fraction(tx)
        for a, m in enumerate((i, j, k)):
            if dd[a] != 0:
                ta, tb = (m - o[a]) / dd[a], (m + 1 - o[a]) / dd[a]
                lo, hi = max(lo, min(ta, tb)), min(hi, max(ta, tb))
        assert abs(float(lo) - t0) <= 1e-12 * max(1.0, abs(t0))
        assert abs(float(hi) - t1) <= 1e-12 * max(1.0, abs(t1))
        assert t0 <= t1
    # consecutive intervals share their boundary parameter
    for a, b in zip(t01[:-1], t01[1:]):
        assert a[1] == b[0]


def test_camera_basis_closed_form():
    # odd square image: centre pixel = forward; middle-row edge pixels are at
    # +-atan((1 - 1/w) tan(fov/2)) from it; top row points along +up.
    dims = (16, 16, 16)
    cam = volgen.Camera(eye=(7.5, -30.0, 7.5), center=(7.5, 7.5, 7.5), up=(0.0, 0.0, 1.0), vfov_deg=45.0)
    w = h = 1001
    dc, _, _, _ = oracle.ray(dims, cam, w, h, 500, 500)
    assert np.allclose(dc, [0.0, 1.0, 0.0], atol=1e-15)
    dl, _, _, _ = oracle.ray(dims, cam, w, h, 0, 500)
    dr, _, _, _ = oracle.ray(dims, cam, w, h, w - 1, 500)
    half = math.atan((1.0 - 1.0 / w) * math.tan(math.radians(22.5)))
    assert math.isclose(math.acos(float(np.dot(dl, dc))), half, rel_tol=1e-12)
    assert math.isclose(math.acos(float(np.dot(dr, dc))), half, rel_tol=1e-12)
    assert dl[0] < 0 < dr[0]       # right = fwd x up = +x here
    dt, _, _, _ = oracle.ray(dims, cam, w, h, 500, 0)
    assert dt[2] > 0
    for d in (dc, dl, dr, dt):
        assert abs(float(np.dot(d, d)) - 1.0) < 4e-16


def test_slab_entry_exit_axis_aligned():
    dims = (16, 12, 10)
    cam = volgen.Camera(eye=(7.25, 5.5, -10.0), center=(7.25, 5.5, 4.0), up=(0.0, 1.0, 0.0), vfov_deg=45.0)
    d, te, tx, ent = oracle.ray(dims, cam, 3, 3, 1, 1)
    assert ent and list(d) == [0.0, 0.0, 1.0]
    assert te == 10.0 and tx == 19.0
    cells, _, _ = oracle.cell_walk(dims, cam, 3, 3, 1, 1)
    assert [tuple(int(v) for v in c) for c in cells] == [(7, 5, k) for k in range(9)]


def test_miss_and_inside_origin():
    dims = (8, 8, 8)
    away = volgen.Camera(eye=(-10.0, -10.0, -10.0), center=(-20.0, -20.0, -20.0), up=(0.0, 0.0, 1.0))
    assert oracle.cell_walk(dims, away, 4, 4, 1, 1) is None
    inside = volgen.Camera(eye=(3.5, 3.5, 3.5), center=(10.0, 3.5, 3.5), up=(0.0, 0.0, 1.0))
    cells, t01, (te, tx) = oracle.cell_walk(dims, inside, 1, 1, 0, 0)
    assert te == 0.0 and tx == 3.5
    assert [tuple(int(v) for v in c) for c in cells] == [(3, 3, 3), (4, 3, 3), (5, 3, 3), (6, 3, 3)]
