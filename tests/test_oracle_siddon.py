"""Pins of the oracle's system matrix: brute-force intersection lengths on
tiny grids, closed-form chord lengths, axis-aligned special cases.

The brute force below is written independently of ``oracle.geometry``: it
clips the ray against every pixel square (Liang-Barsky), with the half-open
pixel rule for rays parallel to a grid line, instead of merging crossings.
"""

import math

import numpy as np
import pytest

import datagen
import oracle

EPS = 1e-9


def _trig(v, V, arc):
    th = v * arc / V
    c, s = math.cos(th), math.sin(th)
    if abs(c) < 1e-12:
        c, s = 0.0, math.copysign(1.0, s)
    if abs(s) < 1e-12:
        s, c = 0.0, math.copysign(1.0, c)
    return c, s


def _clip(ox, oy, dx, dy, x0, x1, y0, y1):
    """Length of the line ``o + t d`` inside ``[x0, x1) x [y0, y1)``."""
    lo, hi = -math.inf, math.inf
    for o, d, a, b in ((ox, dx, x0, x1), (oy, dy, y0, y1)):
        if d == 0.0:
            if not (a <= o < b):
                return 0.0
        else:
            t0, t1 = (a - o) / d, (b - o) / d
            if t0 > t1:
                t0, t1 = t1, t0
            lo, hi = max(lo, t0), min(hi, t1)
    return max(0.0, hi - lo)


def brute_row(geom, v, b):
    """Dense row of ``A`` for ray (v, b) by clipping against every pixel."""
    c, s = _trig(v, geom.n_views, geom.arc_rad)
    u = (b - (geom.n_bins - 1) / 2.0) * (geom.bin_mm / geom.pixel_mm)
    ox, oy = u * c + geom.nx / 2.0, u * s + geom.ny / 2.0
    dx, dy = -s, c
    row = np.zeros(geom.nx * geom.ny)
    for iy in range(geom.ny):
        for ix in range(geom.nx):
            ln = _clip(ox, oy, dx, dy, ix, ix + 1, iy, iy + 1)
            if ln >= EPS:
                row[iy * geom.nx + ix] = ln * geom.pixel_mm
    return row


def chord_in_square(geom, v, b):
    """Closed-form chord of the ray through the image square (half-open)."""
    c, s = _trig(v, geom.n_views, geom.arc_rad)
    u = (b - (geom.n_bins - 1) / 2.0) * (geom.bin_mm / geom.pixel_mm)
    ox, oy = u * c + geom.nx / 2.0, u * s + geom.ny / 2.0
    return _clip(ox, oy, -s, c, 0.0, geom.nx, 0.0, geom.ny) * geom.pixel_mm


def _tiny_geoms():
    rng = np.random.default_rng(7)
    out = []
    for nx in range(1, 9):
        for ny in (nx, max(1, nx - 1)):
            V = int(rng.integers(1, 9))
            B = int(rng.integers(1, 2 * max(nx, ny) + 3))
            bin_mm = float(rng.choice([1.0, 0.5, 0.7, 1.3]))
            out.append(datagen.Geometry(nx, ny, 1.0, V, B, bin_mm))
    # views that hit the axis-aligned and 45-degree cases, with even N / odd B
    out.append(datagen.Geometry(4, 4, 2.0, 4, 5, 2.0))
    out.append(datagen.Geometry(6, 6, 1.0, 8, 9, 1.0))
    out.append(datagen.Geometry(5, 3, 1.5, 6, 7, 1.5))
    return out


@pytest.mark.parametrize("geom", _tiny_geoms(), ids=lambda g: f"{g.nx}x{g.ny}v{g.n_views}b{g.n_bins}")
def test_siddon_matches_brute_force(geom):
    A = oracle.system_matrix(geom).toarray()
    for v in range(geom.n_views):
        for b in range(geom.n_bins):
            ref = brute_row(geom, v, b)
            np.testing.assert_allclose(A[v * geom.n_bins + b], ref, rtol=1e-12, atol=1e-12)


def test_siddon_random_rays_brute_force():
    """Random non-grid angles and offsets on an 8x8 grid."""
    rng = np.random.default_rng(11)
    for trial in range(20):
        V = int(rng.integers(3, 40))
        B = int(rng.integers(3, 20))
        geom = datagen.Geometry(8, 8, 1.0, V, B, float(rng.uniform(0.3, 1.2)),
                                float(rng.uniform(0.5, math.pi)))
        A = oracle.system_matrix(geom)
        for _ in range(10):
            v, b = int(rng.integers(V)), int(rng.integers(B))
            np.testing.assert_allclose(A[v * B + b].toarray().ravel(), brute_row(geom, v, b),
                                       rtol=1e-12, atol=1e-12)


def test_row_sums_are_chords():
    geom = datagen.Geometry(16, 12, 2.0, 13, 27, 1.7)
    A = oracle.system_matrix(geom)
    rs = np.asarray(A.sum(axis=1)).ravel()
    ref = np.array([chord_in_square(geom, v, b) for v in range(geom.n_views)
                    for b in range(geom.n_bins)])
    np.testing.assert_allclose(rs, ref, rtol=1e-12, atol=1e-12)


def test_vertical_view_gives_pixel_size_per_pixel():
    """theta = 0: each ray is a vertical line; with N even and B odd the rays
    lie on grid lines and (half-open pixels) belong to the column on their
    high side; the ray on the image's outer high edge contributes nothing."""
    geom = datagen.Geometry(4, 4, 3.0, 2, 5, 3.0)
    A = oracle.system_matrix(geom).toarray()
    for b in range(5):
        x = b - 2 + 2  # grid coordinate of the line
        row = A[b].reshape(4, 4)
        if x >= 4:
            assert row.sum() == 0.0
        else:
            expect = np.zeros((4, 4))
            expect[:, x] = 3.0
            np.testing.assert_array_equal(row, expect)


def test_horizontal_view_snaps():
    """theta = pi/2 must be exactly horizontal despite cos(pi/2) != 0 in FP."""
    geom = datagen.Geometry(4, 4, 1.0, 2, 5, 1.0)
    A = oracle.system_matrix(geom).toarray()
    for b in range(5):
        row = A[5 + b].reshape(4, 4)
        nz = np.nonzero(row.sum(axis=1))[0]
        assert len(nz) <= 1
        if len(nz):
            np.testing.assert_array_equal(row[nz[0]], np.ones(4))


def test_entries_in_ray_order_and_unique():
    geom = datagen.Geometry(32, 32, 1.0, 17, 45, 1.0)
    A = oracle.system_matrix(geom)
    for m in range(0, A.shape[0], 7):
        cols = A.indices[A.indptr[m]:A.indptr[m + 1]]
        assert len(set(cols.tolist())) == len(cols)
        # consecutive pixels along a ray are 4- or 8-connected
        iy, ix = cols // 32, cols % 32
        if len(cols) > 1:
            assert np.all(np.abs(np.diff(iy)) <= 1) and np.all(np.abs(np.diff(ix)) <= 1)


def test_attenuation_factor():
    geom = datagen.Geometry(10, 10, 2.0, 7, 15, 2.0)
    rng = np.random.default_rng(3)
    mu = rng.uniform(0.0, 0.05, geom.n_pixels)
    A0 = oracle.system_matrix(geom)
    A1 = oracle.system_matrix(geom, mu)
    lineint = A0 @ mu
    expect = A0.multiply(np.exp(-lineint)[:, None]).tocsr()
    np.testing.assert_allclose(A1.toarray(), expect.toarray(), rtol=1e-14, atol=0)


def test_small_config_shape():
    P = datagen.make_problem(**datagen.CONFIG_SMALL)
    A = oracle.system_matrix(P.geom, P.mu)
    assert A.shape == (60 * 95, 64 * 64)
    assert 250_000 < A.nnz < 400_000
    assert np.all(A.data > 0)
