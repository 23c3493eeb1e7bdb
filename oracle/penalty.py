"""Pairwise penalty, its gradient and the separable parabolic surrogate (oracle).

Sec. 3 of the paper: ``R(f) = 1/2 sum_n sum_{j in N_n} w_nj rho(f_n - f_j)``
with a potential ``rho`` from Table 1 that satisfies Assumption 1.

Readings (the paper leaves these open):

* neighbourhood: the 8 in-plane neighbours, weight 1 for the 4 edge
  neighbours and 1/sqrt(2) for the 4 diagonal ones; for a stack of slices
  optionally the 2 axial neighbours with weight 1;
* neighbours falling outside the image are omitted (no wrap, no mirror).

Images are arrays of shape ``(S, ny * nx)``.
"""

from __future__ import annotations

import math

import numpy as np

POT_QUADRATIC, POT_HUBER, POT_LOGCOSH, POT_HYPERBOLA = 0, 1, 2, 3


def neighbours(axial: bool = False):
    """List of ``(dz, dy, dx, w)`` offsets of the neighbourhood."""
    r = 1.0 / math.sqrt(2.0)
    nb = [(0, 0, -1, 1.0), (0, 0, 1, 1.0), (0, -1, 0, 1.0), (0, 1, 0, 1.0),
          (0, -1, -1, r), (0, -1, 1, r), (0, 1, -1, r), (0, 1, 1, r)]
    if axial:
        nb += [(-1, 0, 0, 1.0), (1, 0, 0, 1.0)]
    return nb


def potential(kind: int, delta: float):
    """``(rho, rho', gamma)`` of Table 1 as vectorised functions."""
    if kind == POT_QUADRATIC:
        return (lambda t: 0.5 * t * t, lambda t: t, lambda t: np.ones_like(t))
    if kind == POT_HUBER:
        def rho(t):
            a = np.abs(t)
            return np.where(a <= delta, 0.5 * t * t, delta * a - 0.5 * delta * delta)

        def drho(t):
            return np.clip(t, -delta, delta)

        def gam(t):
            a = np.abs(t)
            return np.where(a <= delta, 1.0, delta / np.maximum(a, delta))
        return rho, drho, gam
    if kind == POT_LOGCOSH:
        def rho(t):
            x = np.abs(t) / delta
            # log cosh x = x + log1p(exp(-2x)) - log 2, stable for large x
            return delta * delta * (x + np.log1p(np.exp(-2.0 * x)) - math.log(2.0))

        def drho(t):
            return delta * np.tanh(t / delta)

        def gam(t):
            t = np.asarray(t, dtype=np.float64)
            small = np.abs(t) < 1e-8 * delta
            safe = np.where(small, 1.0, t)
            return np.where(small, 1.0, delta * np.tanh(safe / delta) / safe)
        return rho, drho, gam
    if kind == POT_HYPERBOLA:
        # Table 1 prints delta*(sqrt(1+(t/delta)^2)-1) next to rho' = t/sqrt(1+(t/delta)^2)
        # and gamma = 1/sqrt(1+(t/delta)^2); those two are the derivative and
        # curvature of delta^2*(sqrt(1+(t/delta)^2)-1), which (like the other rows)
        # is t^2/2 near 0.  The printed derivative and curvature are kept.
        def rho(t):
            return delta * delta * (np.sqrt(1.0 + (t / delta) ** 2) - 1.0)

        def drho(t):
            return t / np.sqrt(1.0 + (t / delta) ** 2)

        def gam(t):
            return 1.0 / np.sqrt(1.0 + (t / delta) ** 2)
        return rho, drho, gam
    raise ValueError(f"unknown potential {kind}")


def _pairs(f, ny, nx, axial):
    """Yield ``(w, f_n view, f_j view, index view into the flat image)`` for
    every neighbour offset, restricted to pixels whose neighbour exists."""
    S = f.shape[0]
    vol = f.reshape(S, ny, nx)
    for (dz, dy, dx, w) in neighbours(axial and S > 1):
        z0, z1 = max(0, -dz), S - max(0, dz)
        y0, y1 = max(0, -dy), ny - max(0, dy)
        x0, x1 = max(0, -dx), nx - max(0, dx)
        if z1 <= z0 or y1 <= y0 or x1 <= x0:
            continue
        fn = vol[z0:z1, y0:y1, x0:x1]
        fj = vol[z0 + dz:z1 + dz, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
        yield w, fn, fj, (slice(z0, z1), slice(y0, y1), slice(x0, x1))


def penalty_value(f, ny, nx, kind=POT_QUADRATIC, delta=1.0, axial=False) -> float:
    """``R(f)`` (Sec. 3, penalty definition), summed over slices."""
    f = np.atleast_2d(np.asarray(f, dtype=np.float64))
    rho, _, _ = potential(kind, delta)
    tot = 0.0
    for w, fn, fj, _ in _pairs(f, ny, nx, axial):
        tot += 0.5 * w * float(rho(fn - fj).sum())
    return tot


def penalty_grad(f, ny, nx, kind=POT_QUADRATIC, delta=1.0, axial=False):
    """``grad R(f)_n = sum_j w_nj rho'(f_n - f_j)`` (symmetric neighbourhood and
    odd ``rho'`` make the two occurrences of each pair add up)."""
    f = np.atleast_2d(np.asarray(f, dtype=np.float64))
    _, drho, _ = potential(kind, delta)
    S = f.shape[0]
    out = np.zeros((S, ny, nx))
    for w, fn, fj, idx in _pairs(f, ny, nx, axial):
        out[idx] += w * drho(fn - fj)
    return out.reshape(S, ny * nx)


def surrogate_terms(f, ny, nx, kind=POT_QUADRATIC, delta=1.0, axial=False):
    """Sums entering the penalised M-step (Sec. 3, eq. svrsurder):
    ``D_n = sum_j d_nj`` and ``E_n = sum_j d_nj f_j`` with
    ``d_nj = w_nj gamma_rho(f_n - f_j)`` evaluated at the expansion point ``f``."""
    f = np.atleast_2d(np.asarray(f, dtype=np.float64))
    _, _, gam = potential(kind, delta)
    S = f.shape[0]
    D = np.zeros((S, ny, nx))
    E = np.zeros((S, ny, nx))
    for w, fn, fj, idx in _pairs(f, ny, nx, axial):
        d = w * gam(fn - fj)
        D[idx] += d
        E[idx] += d * fj
    return D.reshape(S, ny * nx), E.reshape(S, ny * nx)
