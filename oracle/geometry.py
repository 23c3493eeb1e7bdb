"""System matrix of the linear Poisson model (oracle, FP64).

The paper models the mean data as ``E[g] = A f + w`` with a non-negative
system matrix ``A`` (Sec. 2.1, eq. voxel_td).  It does not fix a projector;
this oracle uses exact line/pixel intersection lengths of a 2D parallel-beam
scanner (Siddon's method: merge the ray's crossings with the vertical and
horizontal grid lines, then assign each piece to the pixel containing its
midpoint).

Conventions (all computed in pixel units, lengths scaled to mm at the end):

* view ``v``: ``theta = v * arc / V``; ``cos``/``sin`` with magnitude below
  1e-12 are snapped to exactly 0 (and the other to +-1), so that the
  axis-aligned views are exactly axis-aligned;
* bin ``b``: detector offset ``u = (b - (B-1)/2) * bin_mm / pixel_mm``;
* ray: origin ``(u cos + nx/2, u sin + ny/2)`` in grid coordinates (grid
  spans ``[0, nx] x [0, ny]``), unit direction ``(-sin, cos)``, parameter
  ``t`` increasing along it;
* pieces shorter than ``SEGMENT_EPS`` pixel are dropped;
* pixels are half-open, so a ray lying exactly on a grid line belongs to the
  pixel on its higher-index side and a ray on the outer high edge to none;
* within a row the entries are in increasing ``t``;
* optional attenuation multiplies every entry of a ray by
  ``exp(-sum_n a_mn mu_n)`` (the ray's own line integral of ``mu``).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

SEGMENT_EPS = 1e-9  # pixel units


def view_trig(v: int, n_views: int, arc: float):
    """(cos, sin) of view ``v`` with the axis snapping rule."""
    th = v * arc / n_views
    c, s = math.cos(th), math.sin(th)
    if abs(c) < 1e-12:
        c, s = 0.0, math.copysign(1.0, s)
    if abs(s) < 1e-12:
        s, c = 0.0, math.copysign(1.0, c)
    return c, s


def siddon_rays(geom, v: int):
    """Intersection lists of every bin of view ``v``.

    Returns ``(ray_of_entry, pixel, length_mm)`` arrays, ordered by bin and
    then by ray parameter.
    """
    nx, ny, B = geom.nx, geom.ny, geom.n_bins
    c, s = view_trig(v, geom.n_views, geom.arc_rad)
    u = (np.arange(B, dtype=np.float64) - (B - 1) / 2.0) * (geom.bin_mm / geom.pixel_mm)
    ox = u * c + nx / 2.0
    oy = u * s + ny / 2.0
    dx, dy = -s, c
    parts = []
    if dx != 0.0:
        parts.append((np.arange(nx + 1, dtype=np.float64)[None, :] - ox[:, None]) / dx)
    if dy != 0.0:
        parts.append((np.arange(ny + 1, dtype=np.float64)[None, :] - oy[:, None]) / dy)
    T = np.sort(np.concatenate(parts, axis=1), axis=1)
    ta, tb = T[:, :-1], T[:, 1:]
    seg = tb - ta
    tm = (ta + tb) * 0.5
    ix = np.floor(ox[:, None] + tm * dx)
    iy = np.floor(oy[:, None] + tm * dy)
    keep = (seg >= SEGMENT_EPS) & (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny)
    ray = np.broadcast_to(np.arange(B)[:, None], keep.shape)[keep]
    pix = (iy[keep].astype(np.int64) * nx + ix[keep].astype(np.int64))
    return ray, pix, seg[keep] * geom.pixel_mm


def system_matrix(geom, mu=None) -> sp.csr_matrix:
    """``A`` as an (M x N) FP64 CSR matrix, rows in natural order ``m = v*B + b``.

    ``mu`` (length N, 1/mm) applies the attenuation factor of each ray.
    """
    B = geom.n_bins
    indptr = [np.zeros(1, dtype=np.int64)]
    cols, vals = [], []
    offset = 0
    for v in range(geom.n_views):
        ray, pix, ln = siddon_rays(geom, v)
        if mu is not None:
            lineint = np.zeros(B)
            np.add.at(lineint, ray, ln * np.asarray(mu, dtype=np.float64)[pix])
            ln = ln * np.exp(-lineint)[ray]
        counts = np.bincount(ray, minlength=B)
        indptr.append(offset + np.cumsum(counts))
        offset += int(counts.sum())
        cols.append(pix)
        vals.append(ln)
    indptr = np.concatenate(indptr)
    A = sp.csr_matrix((np.concatenate(vals), np.concatenate(cols), indptr),
                      shape=(geom.n_rays, geom.n_pixels))
    return A


def subset_rows(geom, n_subsets: int):
    """Row sets of the ordered-subset partition (Sec. 2.1, partition of [M]).

    Subset ``t`` holds every bin of the views ``v = t (mod Ns)`` ("interleaved"
    views, so consecutive subsets see well separated angles), view-major and
    bin-minor.  Returns a list of index arrays into the natural row order.
    """
    B = geom.n_bins
    out = []
    for t in range(n_subsets):
        views = np.arange(t, geom.n_views, n_subsets)
        out.append((views[:, None] * B + np.arange(B)[None, :]).ravel())
    return out
