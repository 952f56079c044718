"""Pins of the oracle's first-hit isosurface march (Sec. 3.7: Amanatides-Woo
through the dual cells, Marmitt-style ray-voxel intersection) and of its
macrocell ranges (Sec. 3.1).

All analytic fields are stored in raw mode (rate 32), so the samples the
oracle interpolates are exactly the field's values:
  - planes: trilinear interpolation reproduces a linear field exactly, so the
    hit is t = (iso - d - a.eye) / (a.dir) in exact arithmetic;
  - f = (x-a)(y-b)(z-c): multilinear, reproduced exactly; along a ray it is a
    true cubic whose first root in [t_enter, t_exit] comes from mpmath at
    60 digits;
  - spheres f = |p-c|^2: the interpolant exceeds f by at most 3/4, so the hit
    lies between the ray's entries into the spheres of radius sqrt(iso-3/4)
    and sqrt(iso).
On random smooth fields an independent march (dense point sampling of the
trilinear interpolant evaluated directly from the 8 corner samples) checks
that each oracle hit lies on the surface and that no crossing comes earlier.
"""
import math

import mpmath
import numpy as np
import pytest

import oracle
import volgen

mpmath.mp.dps = 60


def _raw(vol):
    s = volgen.encode(vol, 32)
    nz, ny, nx = vol.shape
    return oracle.decode_volume(s, (nx, ny, nz), 32)


def _cam(eye, center):
    return volgen.Camera(eye=eye, center=center, up=(0.0, 0.0, 1.0), vfov_deg=50.0)


@pytest.mark.parametrize("coef,iso", [((1.0, 0.5, 0.25, -3.0), 13.5), ((-0.5, 1.0, 0.0, 8.0), 12.25),
                                      ((0.0, 0.0, 1.0, 0.0), 9.5)])
def test_plane_hits_closed_form(coef, iso):
    n = 20
    vol = _raw(volgen.analytic(n, n, n, "plane", coef))
    cam = _cam((-14.0, -9.0, 31.0), (9.5, 9.5, 9.5))
    w = h = 24
    r = oracle.render(vol, cam, iso, w, h)
    a = np.array(coef[:3])
    checked = 0
    for p in range(w * h):
        d, te, tx, ent = oracle.ray((n, n, n), cam, w, h, p % w, p // w)
        eye = np.array(cam.eye)
        den = float(a @ d)
        t_true = (iso - coef[3] - float(a @ eye)) / den if den != 0 else math.inf
        inside = ent and te <= t_true <= tx
        if not inside:
            assert not np.isfinite(r["t"][p]), p
            continue
        assert abs(r["t"][p] - t_true) <= 1e-9 * max(1.0, t_true), (p, r["t"][p], t_true)
        hp = eye + t_true * d
        frac = hp - np.floor(hp)
        if np.all((frac > 1e-7) & (frac < 1 - 1e-7)):
            c = np.minimum(np.floor(hp).astype(int), n - 2)
            assert r["block"][p] == (c[0] >> 2) + 5 * ((c[1] >> 2) + 5 * (c[2] >> 2))
            assert r["cell"][p] == (c[0] & 3) + 4 * (c[1] & 3) + 16 * (c[2] & 3)
        checked += 1
    assert checked > 30


def _first_root_product(eye, d, abc, iso, te, tx):
    ex, ey, ez = (mpmath.mpf(v) for v in eye)
    dx, dy, dz = (mpmath.mpf(v) for v in d)
    a, b, c = (mpmath.mpf(v) for v in abc)
    px, qx = ex - a, dx
    py, qy = ey - b, dy
    pz, qz = ez - c, dz
    # (px + qx t)(py + qy t)(pz + qz t) - iso
    c3 = qx * qy * qz
    c2 = px * qy * qz + qx * py * qz + qx * qy * pz
    c1 = px * py * qz + px * qy * pz + qx * py * pz
    c0 = px * py * pz - mpmath.mpf(iso)
    roots = mpmath.polyroots([c3, c2, c1, c0], maxsteps=200, extraprec=200)
    real = sorted(float(mpmath.re(z)) for z in roots if abs(mpmath.im(z)) < mpmath.mpf(10) ** -40)
    for t in real:
        if te <= t <= tx:
            return t
    return math.inf


@pytest.mark.parametrize("abc,iso", [((6.0, 7.0, 5.0), 20.5), ((9.0, 4.0, 8.0), -13.0), ((5.0, 5.0, 5.0), 0.0)])
def test_product_field_cubic_roots(abc, iso):
    n = 14
    vol = _raw(volgen.analytic(n, n, n, "product", abc))
    cam = _cam((-10.5, 23.0, 19.25), (6.5, 6.5, 6.5))
    w, h = 20, 16
    r = oracle.render(vol, cam, iso, w, h)
    checked = 0
    for p in range(w * h):
        d, te, tx, ent = oracle.ray((n, n, n), cam, w, h, p % w, p // w)
        if not ent:
            assert not np.isfinite(r["t"][p])
            continue
        t_true = _first_root_product(cam.eye, d, abc, iso, te, tx)
        if not np.isfinite(t_true):
            assert not np.isfinite(r["t"][p]), p
            continue
        assert abs(r["t"][p] - t_true) <= 1e-8, (p, r["t"][p], t_true)
        checked += 1
    assert checked > 20


def _sphere_entry(eye, d, c, rad2):
    oc = np.array(eye) - np.array(c)
    b = float(oc @ d)
    disc = b * b - (float(oc @ oc) - rad2)
    if disc < 0:
        return None
    return -b - math.sqrt(disc)


def test_sphere_hits_within_interpolation_bound():
    n = 24
    c = (11.5, 12.25, 11.0)
    iso = 64.0
    vol = _raw(volgen.analytic(n, n, n, "sphere", c))
    cam = _cam((40.0, -20.0, 30.0), c)
    w = h = 32
    r = oracle.render(vol, cam, iso, w, h)
    checked = 0
    for p in range(w * h):
        d, te, tx, ent = oracle.ray((n, n, n), cam, w, h, p % w, p // w)
        outer = _sphere_entry(cam.eye, d, c, iso)
        inner = _sphere_entry(cam.eye, d, c, iso - 0.75)
        t = r["t"][p]
        if outer is None:
            assert not np.isfinite(t)
            continue
        if inner is not None:
            assert np.isfinite(t)
            assert outer - 1e-9 <= t <= inner + 1e-9, (p, t, outer, inner)
            checked += 1
        elif np.isfinite(t):
            assert t >= outer - 1e-9
    assert checked > 80


def _interp(vol, pts):
    """Trilinear interpolant at points (N,3), straight from the 8 corner samples."""
    pts = np.atleast_2d(pts)
    nz, ny, nx = vol.shape
    i = np.clip(np.floor(pts).astype(np.int64), 0, [nx - 2, ny - 2, nz - 2])
    f = pts - i
    u, v, w = f[:, 0], f[:, 1], f[:, 2]
    x, y, z = i[:, 0], i[:, 1], i[:, 2]
    V = vol.astype(np.float64)
    c = lambda dx, dy, dz: V[z + dz, y + dy, x + dx]
    return ((c(0, 0, 0) * (1 - u) + c(1, 0, 0) * u) * (1 - v) + (c(0, 1, 0) * (1 - u) + c(1, 1, 0) * u) * v) * (1 - w) \
        + ((c(0, 0, 1) * (1 - u) + c(1, 0, 1) * u) * (1 - v) + (c(0, 1, 1) * (1 - u) + c(1, 1, 1) * u) * v) * w


@pytest.mark.parametrize("kind,seed", [("blobs", 1), ("fourier", 2)])
def test_dense_march_agrees(kind, seed):
    n = 16
    field = volgen.blobs(n, n, n, seed) if kind == "blobs" else volgen.fourier(n, n, n, seed, nmode=12, kmax=3)
    vol = oracle.decode_volume(volgen.encode(field, 8), (n, n, n), 8)
    iso = volgen.percentile_value(vol, 0.7)
    cam = volgen.orbit_camera(n, n, n, seed=seed)
    w = h = 24
    r = oracle.render(vol, cam, iso, w, h)
    step = 1e-3
    hits = 0
    for p in range(w * h):
        d, te, tx, ent = oracle.ray((n, n, n), cam, w, h, p % w, p // w)
        t = r["t"][p]
        if not ent:
            assert not np.isfinite(t)
            continue
        eye = np.array(cam.eye)
        end = t if np.isfinite(t) else tx
        ts = np.arange(te, end - step, step)
        if len(ts) > 1:
            vals = _interp(vol, eye[None, :] + ts[:, None] * d[None, :]) - iso
            sgn = np.sign(vals)
            # no strict sign change before the oracle's hit (or along the whole ray)
            assert not np.any(sgn[:-1] * sgn[1:] < 0), (p, t)
        if np.isfinite(t):
            assert abs(_interp(vol, eye + t * d)[0] - iso) <= 1e-9 * max(1.0, abs(iso))
            hits += 1
    assert hits > 50


def test_grid_ranges_cover_every_dual_cell_and_are_tight():
    for dims, seed in (((16, 16, 16), 3), ((13, 10, 9), 4)):
        nx, ny, nz = dims
        vol = volgen.blobs(nx, ny, nz, seed)
        blk, fin, crs = oracle.grids(vol)
        nbx, nby, nbz = (nx + 3) // 4, (ny + 3) // 4, (nz + 3) // 4
        ncx, ncy = (nbx + 3) // 4, (nby + 3) // 4
        # every dual cell's 8 corners lie inside its block's fine range
        for k in range(nz - 1):
            for j in range(ny - 1):
                for i in range(nx - 1):
                    b = (i >> 2) + nbx * ((j >> 2) + nby * (k >> 2))
                    c = vol[k:k + 2, j:j + 2, i:i + 2]
                    assert fin[b, 0] <= c.min() and c.max() <= fin[b, 1]
        # tightness: each bound is attained by a sample of the 2x2x2 block neighbourhood
        for b in range(nbx * nby * nbz):
            bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
            sub = vol[4 * bz:4 * bz + 8, 4 * by:4 * by + 8, 4 * bx:4 * bx + 8]
            assert fin[b, 0] == sub.min() and fin[b, 1] == sub.max()
            own = vol[4 * bz:4 * bz + 4, 4 * by:4 * by + 4, 4 * bx:4 * bx + 4]
            assert blk[b, 0] == own.min() and blk[b, 1] == own.max()
        # coarse cells: union of their fine cells, and contain every one of them
        for b in range(nbx * nby * nbz):
            bx, by, bz = b % nbx, (b // nbx) % nby, b // (nbx * nby)
            cc = (bx >> 2) + ncx * ((by >> 2) + ncy * (bz >> 2))
            assert crs[cc, 0] <= fin[b, 0] and fin[b, 1] <= crs[cc, 1]
        assert crs[:, 0].min() == fin[:, 0].min() and crs[:, 1].max() == fin[:, 1].max()
