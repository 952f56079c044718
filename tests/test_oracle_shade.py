"""Pins of the oracle's hit shading (Sec. 3.7 colours the hit; the headlight
Lambertian model is this build's reading: base (0.90, 0.75, 0.40) times
0.15 + 0.85 |n.d|, n the normalised gradient of the trilinear interpolant at
the hit, RGBA8 with r in the low byte, alpha 255) and of the BCMC block count.

The expected colours come from closed forms of the interpolant's gradient,
computed here from the ray and the hit parameter, not from the oracle's
shading code:
  - plane a.x + d: the interpolant is the plane itself, so the gradient is
    the constant (a, b, c);
  - product (x-a)(y-b)(z-c): multilinear, reproduced exactly, so the gradient
    at the hit point p is ((y-b)(z-c), (x-a)(z-c), (x-a)(y-b)) and varies
    across the cell (a swapped component or a wrong interpolation weight in
    the gradient changes it);
  - sphere |p-c|^2 with integer c: on each axis the interpolant of the
    quadratic is linear inside a cell, so the gradient is exactly
    2 (cell midpoint - c), constant over the cell.
All three fields are stored raw (rate 32), so the samples are the field's
values exactly.  The hit parameters are pinned separately (test_oracle_hits).
"""
import numpy as np
import pytest

import oracle
import volgen

BASE = np.array([0.90, 0.75, 0.40])


def _raw(vol):
    s = volgen.encode(vol, 32)
    nz, ny, nx = vol.shape
    return oracle.decode_volume(s, (nx, ny, nz), 32)


def _cam(eye, center):
    return volgen.Camera(eye=eye, center=center, up=(0.0, 0.0, 1.0), vfov_deg=50.0)


def _colour(grad, d):
    g = np.asarray(grad, np.float64)
    nd = abs(float(g @ d)) / float(np.sqrt(g @ g))
    k = 0.15 + 0.85 * nd
    ch = np.clip(np.floor(255.0 * (BASE * k) + 0.5), 0, 255).astype(np.uint32)
    return int(ch[0] | (ch[1] << 8) | (ch[2] << 16) | (0xFF << 24))


def _check(r, dims, cam, w, h, grad_at):
    exact = close = 0
    for p in range(w * h):
        t = r["t"][p]
        if not np.isfinite(t):
            assert r["rgba"][p] == 0, p          # background is 0
            continue
        d, te, tx, ent = oracle.ray(dims, cam, w, h, p % w, p // w)
        hp = np.array(cam.eye) + t * d
        want = _colour(grad_at(hp, r["block"][p], r["cell"][p]), d)
        got = int(r["rgba"][p])
        assert got >> 24 == 0xFF, p
        diff = max(abs(((got >> s) & 255) - ((want >> s) & 255)) for s in (0, 8, 16))
        assert diff <= 1, (p, hex(got), hex(want))
        exact += diff == 0
        close += 1
    return exact, close


@pytest.mark.parametrize("coef,iso", [((1.0, 0.5, 0.25, -3.0), 13.5), ((-0.5, 1.0, 0.0, 8.0), 12.25),
                                      ((0.25, -0.75, 1.5, 2.0), 9.0)])
def test_plane_colour_closed_form(coef, iso):
    n = 20
    vol = _raw(volgen.analytic(n, n, n, "plane", coef))
    cam = _cam((-14.0, -9.0, 31.0), (9.5, 9.5, 9.5))
    w = h = 24
    r = oracle.render(vol, cam, iso, w, h)
    exact, hits = _check(r, (n, n, n), cam, w, h, lambda p, b, c: coef[:3])
    assert hits > 30 and exact >= 0.95 * hits, (exact, hits)


@pytest.mark.parametrize("abc,iso", [((6.0, 7.0, 5.0), 20.5), ((9.0, 4.0, 8.0), -13.0)])
def test_product_colour_follows_exact_gradient(abc, iso):
    n = 14
    a, b, c = abc
    vol = _raw(volgen.analytic(n, n, n, "product", abc))
    cam = _cam((-10.5, 23.0, 19.25), (6.5, 6.5, 6.5))
    w, h = 20, 16
    r = oracle.render(vol, cam, iso, w, h)

    def grad(p, blk, cell):
        x, y, z = p
        return ((y - b) * (z - c), (x - a) * (z - c), (x - a) * (y - b))

    exact, hits = _check(r, (n, n, n), cam, w, h, grad)
    assert hits > 20 and exact >= 0.95 * hits, (exact, hits)


def test_sphere_colour_uses_cell_midpoint_normal():
    n = 24
    cen = (11.0, 12.0, 11.0)
    iso = 64.0
    vol = _raw(volgen.analytic(n, n, n, "sphere", cen))
    cam = _cam((40.0, -20.0, 30.0), cen)
    w = h = 32
    r = oracle.render(vol, cam, iso, w, h)
    nb = (n + 3) // 4

    def grad(p, blk, cell):
        bx, by, bz = blk % nb, (blk // nb) % nb, blk // (nb * nb)
        i = 4 * bx + (cell & 3)
        j = 4 * by + ((cell >> 2) & 3)
        k = 4 * bz + (cell >> 4)
        # the hit lies in (or on the boundary of) its cell
        assert i - 1e-9 <= p[0] <= i + 1 + 1e-9 and j - 1e-9 <= p[1] <= j + 1 + 1e-9 and k - 1e-9 <= p[2] <= k + 1 + 1e-9
        return (2 * (i + 0.5 - cen[0]), 2 * (j + 0.5 - cen[1]), 2 * (k + 0.5 - cen[2]))

    exact, hits = _check(r, (n, n, n), cam, w, h, grad)
    assert hits > 80 and exact >= 0.95 * hits, (exact, hits)


@pytest.mark.parametrize("dims,seed,q", [((16, 16, 16), 3, 0.6), ((13, 10, 9), 4, 0.3), ((24, 20, 16), 5, 0.9)])
def test_blocks_containing_brute_force(dims, seed, q):
    """The BCMC count (blocks a decompress-everything-that-may-hold-the-surface
    renderer decodes, Sec. 5 comparison): blocks whose 2x2x2 block
    neighbourhood of samples spans the isovalue, counted by brute force over
    the samples."""
    nx, ny, nz = dims
    vol = volgen.blobs(nx, ny, nz, seed)
    iso = float(np.quantile(vol, q))
    blk, fin, crs = oracle.grids(vol)
    nbx, nby, nbz = (nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4
    want = 0
    for bz in range(nbz):
        for by in range(nby):
            for bx in range(nbx):
                sub = vol[4 * bz:4 * bz + 8, 4 * by:4 * by + 8, 4 * bx:4 * bx + 8]
                want += bool(sub.min() <= np.float32(iso) <= sub.max())
    assert oracle.blocks_containing(fin, np.float32(iso)) == want
    assert 0 < want < nbx * nby * nbz
