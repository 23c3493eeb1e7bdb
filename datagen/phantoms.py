"""Seeded phantoms, attenuation maps and Poisson sinograms.

Scanner convention (2D parallel beam, shared *as a convention* by every
consumer of these inputs, and restated independently by each of them):

* view ``v`` has angle ``theta_v = v * arc / V`` (``arc`` = pi, i.e. 180 deg);
* radial bin ``b`` sits at ``s_b = (b - (B - 1) / 2) * bin_mm``;
* ray ``(v, b)`` is the line ``s_b (cos t, sin t) + u (-sin t, cos t)``;
* sinogram index ``m = v * B + b``; pixel ``(ix, iy)`` has flat index
  ``iy * nx + ix`` and covers ``[x0 + ix*dx, x0 + (ix+1)*dx)`` with
  ``x0 = -nx*dx/2`` (same in y).

The measured data are simulated from the *continuous* phantom: every line
integral is the exact chord length of the line through each ellipse (or
ellipse slice of an ellipsoid) times its intensity, attenuated by the exact
chord through the attenuating disc.  No pixel grid and no system matrix is
involved, so the data carry a realistic model mismatch and neither the oracle
nor the HIP path can reuse anything from here.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

# ---------------------------------------------------------------------------
# Workload descriptions (sizes of the scanner configurations the library is
# measured on).  Pixel sizes not fixed by the workload description use 2 mm.
# ---------------------------------------------------------------------------

CONFIG_SMALL = dict(nx=64, ny=64, pixel_mm=4.0, n_views=60, n_bins=95, bin_mm=4.0,
                    n_subsets=6, counts=1e5, attenuation=True, seed=0)
CONFIG_HEADLINE = dict(nx=256, ny=256, pixel_mm=2.0, n_views=252, n_bins=344, bin_mm=2.0,
                       n_subsets=21, counts=1e6, attenuation=False, seed=1)
CONFIG_MULTISLICE = dict(nx=285, ny=285, pixel_mm=2.5, n_views=344, n_bins=435, bin_mm=2.5,
                         n_subsets=21, counts=5e7, n_slices=127, seed=4)

MU_WATER_PER_MM = 0.0096  # attenuation coefficient of the attenuating disc (1/mm)


@dataclasses.dataclass(frozen=True)
class Geometry:
    nx: int
    ny: int
    pixel_mm: float
    n_views: int
    n_bins: int
    bin_mm: float
    arc_rad: float = math.pi

    @property
    def n_pixels(self) -> int:
        return self.nx * self.ny

    @property
    def n_rays(self) -> int:
        return self.n_views * self.n_bins


@dataclasses.dataclass
class Problem:
    """One reconstruction problem: geometry, data and the truth it came from."""

    geom: Geometry
    n_subsets: int
    g: np.ndarray          # (S, M) float32 Poisson counts, natural order m = v*B + b
    w: np.ndarray          # (S, M) float32 mean background (randoms + scatter)
    f_true: np.ndarray     # (S, N) float64 rasterised phantom (same units as the reconstruction)
    mu: Optional[np.ndarray]  # (N,) float32 attenuation map in 1/mm, or None
    ybar_true: np.ndarray  # (S, M) float64 noiseless mean data without background
    meta: dict

    @property
    def n_slices(self) -> int:
        return self.g.shape[0]


# ---------------------------------------------------------------------------
# Closed-form chord lengths
# ---------------------------------------------------------------------------

def _ray_lines(geom: Geometry):
    """Points and unit directions of every bin-centre line, shape (M,)."""
    v = np.arange(geom.n_views, dtype=np.float64)
    th = v * geom.arc_rad / geom.n_views
    s = (np.arange(geom.n_bins, dtype=np.float64) - (geom.n_bins - 1) / 2.0) * geom.bin_mm
    c, sn = np.cos(th)[:, None], np.sin(th)[:, None]
    px = (s[None, :] * c).ravel()
    py = (s[None, :] * sn).ravel()
    dx = np.broadcast_to(-sn, (geom.n_views, geom.n_bins)).ravel()
    dy = np.broadcast_to(c, (geom.n_views, geom.n_bins)).ravel()
    return px, py, dx, dy


def _ellipse_chords(px, py, dx, dy, cx, cy, a, b, phi):
    """Length of each line ``p + u d`` (|d| = 1) inside the ellipse."""
    cph, sph = math.cos(phi), math.sin(phi)
    qx, qy = px - cx, py - cy
    # rotate into the ellipse frame and scale to the unit circle
    Px = (cph * qx + sph * qy) / a
    Py = (-sph * qx + cph * qy) / b
    Dx = (cph * dx + sph * dy) / a
    Dy = (-sph * dx + cph * dy) / b
    dd = Dx * Dx + Dy * Dy
    pd = Px * Dx + Py * Dy
    pp = Px * Px + Py * Py
    disc = pd * pd - dd * (pp - 1.0)
    out = np.zeros_like(px)
    pos = disc > 0
    out[pos] = 2.0 * np.sqrt(disc[pos]) / dd[pos]
    return out


def _inside_ellipse(x, y, cx, cy, a, b, phi):
    cph, sph = math.cos(phi), math.sin(phi)
    qx, qy = x - cx, y - cy
    u = (cph * qx + sph * qy) / a
    v = (-sph * qx + cph * qy) / b
    return (u * u + v * v) <= 1.0


def _pixel_subsamples(geom: Geometry, ss: int = 4):
    """Sub-sample coordinates (ss x ss per pixel), shape (ny, nx, ss*ss)."""
    d = geom.pixel_mm
    x0 = -geom.nx * d / 2.0
    y0 = -geom.ny * d / 2.0
    sub = (np.arange(ss) + 0.5) / ss
    xs = x0 + (np.arange(geom.nx)[:, None] + sub[None, :]) * d   # (nx, ss)
    ys = y0 + (np.arange(geom.ny)[:, None] + sub[None, :]) * d   # (ny, ss)
    X = np.broadcast_to(xs[None, :, None, :], (geom.ny, geom.nx, ss, ss))
    Y = np.broadcast_to(ys[:, None, :, None], (geom.ny, geom.nx, ss, ss))
    return X.reshape(geom.ny, geom.nx, ss * ss), Y.reshape(geom.ny, geom.nx, ss * ss)


# ---------------------------------------------------------------------------
# Phantoms
# ---------------------------------------------------------------------------

def _draw_ellipses(rng: np.random.Generator, fov: float, radius: float, n: int):
    """Ellipses inside a disc of ``radius``: centres within 0.6*radius,
    semi-axes U[0.04, 0.2]*fov (shrunk to stay inside the disc), angle U[0, pi),
    intensity U[0.5, 4].  Returns a list of (cx, cy, a, b, phi, rho)."""
    out = []
    for _ in range(n):
        r = 0.6 * radius * math.sqrt(rng.uniform())
        ang = rng.uniform(0.0, 2.0 * math.pi)
        cx, cy = r * math.cos(ang), r * math.sin(ang)
        a = rng.uniform(0.04, 0.2) * fov
        b = rng.uniform(0.04, 0.2) * fov
        room = 0.95 * (radius - r)
        scale = min(1.0, room / max(a, b))
        a, b = a * scale, b * scale
        phi = rng.uniform(0.0, math.pi)
        rho = rng.uniform(0.5, 4.0)
        out.append((cx, cy, a, b, phi, rho))
    return out


def _phantom_2d(geom: Geometry, rng: np.random.Generator, n_ellipses: int):
    """Disc of intensity 1 plus additive ellipses (each adds rho - 1, so an
    isolated ellipse shows intensity rho).  Redraws until the phantom stays
    >= 0.25 everywhere inside the disc."""
    fov = min(geom.nx, geom.ny) * geom.pixel_mm
    radius = 0.45 * fov
    X, Y = _pixel_subsamples(geom)
    for _attempt in range(100):
        ells = _draw_ellipses(rng, fov, radius, n_ellipses)
        disc = (X * X + Y * Y) <= radius * radius
        val = disc.astype(np.float64)
        for (cx, cy, a, b, phi, rho) in ells:
            val += (rho - 1.0) * _inside_ellipse(X, Y, cx, cy, a, b, phi)
        if val[disc].min() >= 0.25:
            raster = val.mean(axis=2).reshape(-1)
            return radius, ells, raster
    raise RuntimeError("could not draw a non-negative ellipse phantom")


def _sinogram_2d(geom: Geometry, radius: float, ells, attenuation: bool):
    px, py, dx, dy = _ray_lines(geom)
    disc_chord = _ellipse_chords(px, py, dx, dy, 0.0, 0.0, radius, radius, 0.0)
    p = disc_chord.copy()
    for (cx, cy, a, b, phi, rho) in ells:
        p += (rho - 1.0) * _ellipse_chords(px, py, dx, dy, cx, cy, a, b, phi)
    if attenuation:
        p *= np.exp(-MU_WATER_PER_MM * disc_chord)
    return p


def _mu_map(geom: Geometry, radius: float) -> np.ndarray:
    X, Y = _pixel_subsamples(geom)
    frac = ((X * X + Y * Y) <= radius * radius).mean(axis=2).reshape(-1)
    return (MU_WATER_PER_MM * frac).astype(np.float32)


def make_problem(nx: int, ny: int, pixel_mm: float, n_views: int, n_bins: int, bin_mm: float,
                 n_subsets: int, counts: float, attenuation: bool = False, seed: int = 0,
                 bg_frac: float = 0.1, n_ellipses: int = 6, arc_rad: float = math.pi) -> Problem:
    """A seeded 2D problem.  Phantom seed ``1000+seed``, Poisson seed ``2000+seed``.

    The noiseless data are scaled so that their total (before background)
    equals ``counts``; the background is uniform at ``bg_frac`` of the mean
    noiseless bin value; ``g ~ Poisson(noiseless + background)``.
    """
    geom = Geometry(nx, ny, float(pixel_mm), n_views, n_bins, float(bin_mm), float(arc_rad))
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    radius, ells, raster = _phantom_2d(geom, rng, n_ellipses)
    p = _sinogram_2d(geom, radius, ells, attenuation)
    k = counts / p.sum()
    ybar = k * p
    f_true = k * raster
    bg = bg_frac * ybar.mean()
    w = np.full_like(ybar, bg)
    prng = np.random.Generator(np.random.PCG64(2000 + seed))
    g = prng.poisson(ybar + w).astype(np.float32)
    mu = _mu_map(geom, radius) if attenuation else None
    return Problem(geom=geom, n_subsets=n_subsets, g=g[None, :], w=w.astype(np.float32)[None, :],
                   f_true=f_true[None, :], mu=mu, ybar_true=ybar[None, :],
                   meta=dict(counts=counts, bg=bg, seed=seed, n_ellipses=n_ellipses,
                             attenuation=attenuation))


def make_multislice_problem(nx: int, ny: int, pixel_mm: float, n_views: int, n_bins: int,
                            bin_mm: float, n_subsets: int, counts: float, n_slices: int,
                            seed: int = 0, bg_frac: float = 0.1, n_ellipsoids: int = 8,
                            slice_mm: Optional[float] = None) -> Problem:
    """A seeded stack of 2D slices sharing one geometry.

    The object is a cylinder of intensity 1 (radius 0.45 FOV) plus additive
    axis-aligned-in-z ellipsoids (rotated in plane); slice ``k`` sits at
    ``z_k = (k - (S-1)/2) * slice_mm`` and sees the ellipse cut of each
    ellipsoid.  No attenuation.  Totals are scaled over the whole stack.
    """
    geom = Geometry(nx, ny, float(pixel_mm), n_views, n_bins, float(bin_mm))
    dz = float(slice_mm if slice_mm is not None else pixel_mm)
    rng = np.random.Generator(np.random.PCG64(1000 + seed))
    fov = min(nx, ny) * pixel_mm
    radius = 0.45 * fov
    zext = n_slices * dz
    ells2 = _draw_ellipses(rng, fov, radius, n_ellipsoids)
    ellz = [(rng.uniform(-0.4, 0.4) * zext, rng.uniform(0.1, 0.4) * zext) for _ in ells2]
    X, Y = _pixel_subsamples(geom)
    disc = (X * X + Y * Y) <= radius * radius
    px, py, dx, dy = _ray_lines(geom)
    disc_chord = _ellipse_chords(px, py, dx, dy, 0.0, 0.0, radius, radius, 0.0)
    P = np.empty((n_slices, geom.n_rays))
    F = np.empty((n_slices, geom.n_pixels))
    for k in range(n_slices):
        z = (k - (n_slices - 1) / 2.0) * dz
        p = disc_chord.copy()
        val = disc.astype(np.float64)
        for (cx, cy, a, b, phi, rho), (cz, cc) in zip(ells2, ellz):
            q = 1.0 - ((z - cz) / cc) ** 2
            if q <= 0.0:
                continue
            sc = math.sqrt(q)
            p += (rho - 1.0) * _ellipse_chords(px, py, dx, dy, cx, cy, a * sc, b * sc, phi)
            val += (rho - 1.0) * _inside_ellipse(X, Y, cx, cy, a * sc, b * sc, phi)
        P[k] = p
        F[k] = np.maximum(val, 0.0).mean(axis=2).reshape(-1)
    kk = counts / P.sum()
    ybar = kk * P
    bg = bg_frac * ybar.mean()
    w = np.full_like(ybar, bg)
    prng = np.random.Generator(np.random.PCG64(2000 + seed))
    g = prng.poisson(ybar + w).astype(np.float32)
    return Problem(geom=geom, n_subsets=n_subsets, g=g, w=w.astype(np.float32), f_true=kk * F,
                   mu=None, ybar_true=ybar,
                   meta=dict(counts=counts, bg=bg, seed=seed, n_ellipsoids=n_ellipsoids,
                             slice_mm=dz))


def make_order(n_subsets: int, n_iter: int, seed: int) -> np.ndarray:
    """Subset indices drawn i.i.d. uniformly (with replacement) from
    ``[0, n_subsets)`` with a PCG64 generator seeded ``3000+seed``."""
    rng = np.random.Generator(np.random.PCG64(3000 + seed))
    return rng.integers(0, n_subsets, size=n_iter).astype(np.int32)


def serving_requests(n: int, rate_per_s: float, seed: int = 0,
                     sizes=(128, 192, 256, 384), epochs: int = 30) -> List[dict]:
    """A seeded Poisson-arrival request stream (seed ``4000+seed``).

    Each request: image ``N x N`` with N drawn from ``sizes``, views uniform
    in [120, 400], bins ``round(1.35 N)``, subsets in {8, 14, 21}, counts
    log-uniform in [1e5, 1e7], SVREM for ``epochs`` epochs.
    """
    rng = np.random.Generator(np.random.PCG64(4000 + seed))
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        N = int(rng.choice(sizes))
        V = int(rng.integers(120, 401))
        B = int(round(1.35 * N))
        ns = int(rng.choice([8, 14, 21]))
        counts = float(10.0 ** rng.uniform(5.0, 7.0))
        out.append(dict(id=i, arrival_s=t, nx=N, ny=N, pixel_mm=2.0, n_views=V, n_bins=B,
                        bin_mm=2.0, n_subsets=ns, counts=counts, epochs=epochs,
                        seed=100 + i))
    return out


def scanner_requests(n: int, seed: int = 0, epochs: int = 30) -> List[dict]:
    """A seeded stream of ``n`` requests from one scanner: the headline
    geometry (256 x 256, 2 mm; 252 views x 344 bins, 21 subsets) for every
    request, counts log-uniform in [1e5, 1e7], SVREM for ``epochs`` epochs
    (seed ``5000+seed``)."""
    rng = np.random.Generator(np.random.PCG64(5000 + seed))
    return [dict(id=i, nx=256, ny=256, pixel_mm=2.0, n_views=252, n_bins=344, bin_mm=2.0, n_subsets=21,
                 counts=float(10.0 ** rng.uniform(5.0, 7.0)), epochs=epochs, seed=300 + i) for i in range(n)]

