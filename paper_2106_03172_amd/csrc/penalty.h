// Pairwise penalty R(f) = 1/2 sum_n sum_{j in N_n} w_nj rho(f_n - f_j) (Sec. 3),
// potentials of Table 1, and the per-pixel stencil sums used by the fused
// updates.  Everything is evaluated in FP64.
//
// Neighbourhood: 8 in-plane neighbours, weight 1 (edges) and 1/sqrt(2)
// (diagonals); neighbours outside the image are omitted.
#pragma once

#include <hip/hip_runtime.h>

#include "common.h"

namespace svr {

constexpr double INV_SQRT2 = 0.70710678118654752440;

__device__ inline double pot_rho(int kind, double t, double delta) {
    switch (kind) {
        case SVR_PEN_HUBER: {
            double a = fabs(t);
            return a <= delta ? 0.5 * t * t : delta * a - 0.5 * delta * delta;
        }
        case SVR_PEN_LOGCOSH: {
            double x = fabs(t) / delta;  // log cosh x = x + log1p(exp(-2x)) - log 2
            return delta * delta * (x + log1p(exp(-2.0 * x)) - 0.69314718055994530942);
        }
        case SVR_PEN_HYPERBOLA: {
            double q = t / delta;
            return delta * delta * (sqrt(1.0 + q * q) - 1.0);
        }
        default:
            return 0.5 * t * t;
    }
}

__device__ inline double pot_drho(int kind, double t, double delta) {
    switch (kind) {
        case SVR_PEN_HUBER: return fmin(fmax(t, -delta), delta);
        case SVR_PEN_LOGCOSH: return delta * tanh(t / delta);
        case SVR_PEN_HYPERBOLA: { double q = t / delta; return t / sqrt(1.0 + q * q); }
        default: return t;
    }
}

// curvature gamma(t) = rho'(t)/t (finite and non-zero at 0, Assumption 1)
__device__ inline double pot_gamma(int kind, double t, double delta) {
    switch (kind) {
        case SVR_PEN_HUBER: { double a = fabs(t); return a <= delta ? 1.0 : delta / a; }
        case SVR_PEN_LOGCOSH: {
            if (fabs(t) < 1e-8 * delta) return 1.0;
            return delta * tanh(t / delta) / t;
        }
        case SVR_PEN_HYPERBOLA: { double q = t / delta; return 1.0 / sqrt(1.0 + q * q); }
        default: return 1.0;
    }
}

// Visits the existing in-plane neighbours of pixel (ix, iy): fn(j, w_nj).
template <class F>
__device__ inline void for_neighbours(int ix, int iy, int nx, int ny, F &&fn) {
    const bool l = ix > 0, r = ix + 1 < nx, d = iy > 0, u = iy + 1 < ny;
    const int n = iy * nx + ix;
    if (l) fn(n - 1, 1.0);
    if (r) fn(n + 1, 1.0);
    if (d) fn(n - nx, 1.0);
    if (u) fn(n + nx, 1.0);
    if (d && l) fn(n - nx - 1, INV_SQRT2);
    if (d && r) fn(n - nx + 1, INV_SQRT2);
    if (u && l) fn(n + nx - 1, INV_SQRT2);
    if (u && r) fn(n + nx + 1, INV_SQRT2);
}

// grad R(f)_n = sum_j w_nj rho'(f_n - f_j)
__device__ inline double penalty_grad_at(const float *f, int n, const PenaltyArgs &p) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const double fn = (double)f[n];
    double g = 0.0;
    for_neighbours(ix, iy, p.nx, p.ny, [&](int j, double w) {
        g = g + w * pot_drho(p.potential, fn - (double)f[j], p.delta);
    });
    return g;
}

// Surrogate sums of the penalised M-step: D = sum_j d_nj, E = sum_j d_nj f_j,
// d_nj = w_nj gamma(f_n - f_j) at the expansion point f (Sec. 3, eq. svrsurder).
__device__ inline void surrogate_at(const float *f, int n, const PenaltyArgs &p, double &D, double &E) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const double fn = (double)f[n];
    D = 0.0;
    E = 0.0;
    for_neighbours(ix, iy, p.nx, p.ny, [&](int j, double w) {
        const double fj = (double)f[j];
        const double d = w * pot_gamma(p.potential, fn - fj, p.delta);
        D = D + d;
        E = E + d * fj;
    });
}

// 1/2 sum_j w_nj rho(f_n - f_j): pixel n's share of R(f)
__device__ inline double penalty_share_at(const float *f, int n, const PenaltyArgs &p) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const double fn = (double)f[n];
    double r = 0.0;
    for_neighbours(ix, iy, p.nx, p.ny, [&](int j, double w) {
        r = r + w * pot_rho(p.potential, fn - (double)f[j], p.delta);
    });
    return 0.5 * r;
}

// Non-negative root of a/f - 2 b f + c = 0 (Sec. 3, below eq. svrsurder).
//  b > 0, a > 0 : (c + sqrt(c^2 + 8ab)) / (4b), as 2a / (sqrt(D) - c) when c < 0;
//  b > 0, a = 0 : max(c, 0) / (2b);   b = 0 : -a/c (a > 0, c < 0);
//  a < 0 or a pixel with sens = 0 : 0.
__device__ inline double mstep_root(double a, double b, double c, double sens) {
    if (!(sens > 0.0)) return 0.0;
    if (b > 0.0) {
        if (a > 0.0) {
            double sq = sqrt(c * c + 8.0 * a * b);
            return c >= 0.0 ? (c + sq) / (4.0 * b) : 2.0 * a / (sq - c);
        }
        if (a == 0.0) return fmax(c, 0.0) / (2.0 * b);
        return 0.0;
    }
    if (a > 0.0 && c < 0.0) return -a / c;
    return 0.0;
}

}  // namespace svr
