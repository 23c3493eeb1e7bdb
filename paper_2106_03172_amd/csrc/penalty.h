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

// The 8 in-plane neighbours of pixel n = iy*nx + ix (values at f[j*stride + off])
// in a fixed order (left,
// right, down, up, down-left, down-right, up-left, up-right): their values,
// loaded together and unconditionally (outside the image the coordinate is
// clamped, so the load stays in bounds, and the neighbour is flagged
// absent), and their weights w_nj.  Loading them first lets all eight loads
// be in flight at once; the sums below then add the present neighbours in
// that order.
struct Neighbours {
    float v[8];
    bool ok[8];  // false for a neighbour outside the image
};

__device__ inline Neighbours load_neighbours(const float *f, int ix, int iy, int nx, int ny, int64_t stride = 1,
                                             int64_t off = 0) {
    const bool l = ix > 0, r = ix + 1 < nx, d = iy > 0, u = iy + 1 < ny;
    const int xl = l ? ix - 1 : ix, xr = r ? ix + 1 : ix, yd = d ? iy - 1 : iy, yu = u ? iy + 1 : iy;
    const int jj[8] = {iy * nx + xl, iy * nx + xr, yd * nx + ix, yu * nx + ix,
                       yd * nx + xl, yd * nx + xr, yu * nx + xl, yu * nx + xr};
    Neighbours nb;
    nb.ok[0] = l; nb.ok[1] = r; nb.ok[2] = d; nb.ok[3] = u;
    nb.ok[4] = d && l; nb.ok[5] = d && r; nb.ok[6] = u && l; nb.ok[7] = u && r;
#pragma unroll
    for (int k = 0; k < 8; ++k) nb.v[k] = f[(int64_t)jj[k] * stride + off];
    return nb;
}

__device__ inline double nb_weight(int k) { return k < 4 ? 1.0 : INV_SQRT2; }

__device__ inline Neighbours load_neighbours_of(const float *f, int n, const PenaltyArgs &p) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    return load_neighbours(f, ix, iy, p.nx, p.ny);
}

// The stencil sums below take the potential as a template argument (one
// switch per pixel, outside the loop) and add every neighbour without a
// branch: an absent one contributes +0.0, which leaves each sum unchanged
// (none of them can be -0.0 at that point), so the sums equal those over the
// present neighbours in the fixed order, bitwise.
template <int POT>
__device__ inline double penalty_grad_pot(double fn, const Neighbours &nb, double delta) {
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double term = nb_weight(k) * pot_drho(POT, fn - (double)nb.v[k], delta);
        g = g + (nb.ok[k] ? term : 0.0);
    }
    return g;
}

// grad R(f)_n = sum_j w_nj rho'(f_n - f_j), from pixel n's value and its neighbours
__device__ inline double penalty_grad_nb(double fn, const Neighbours &nb, const PenaltyArgs &p) {
    switch (p.potential) {
        case SVR_PEN_HUBER: return penalty_grad_pot<SVR_PEN_HUBER>(fn, nb, p.delta);
        case SVR_PEN_LOGCOSH: return penalty_grad_pot<SVR_PEN_LOGCOSH>(fn, nb, p.delta);
        case SVR_PEN_HYPERBOLA: return penalty_grad_pot<SVR_PEN_HYPERBOLA>(fn, nb, p.delta);
        default: return penalty_grad_pot<SVR_PEN_QUADRATIC>(fn, nb, p.delta);
    }
}

__device__ inline double penalty_grad_at(const float *f, int n, const PenaltyArgs &p) {
    return penalty_grad_nb((double)f[n], load_neighbours_of(f, n, p), p);
}

template <int POT>
__device__ inline void surrogate_pot(double fn, const Neighbours &nb, double delta, double &D, double &E) {
    D = 0.0;
    E = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double fj = (double)nb.v[k];
        const double d = nb_weight(k) * pot_gamma(POT, fn - fj, delta);
        D = D + (nb.ok[k] ? d : 0.0);
        E = E + (nb.ok[k] ? d * fj : 0.0);
    }
}

// Surrogate sums of the penalised M-step: D = sum_j d_nj, E = sum_j d_nj f_j,
// d_nj = w_nj gamma(f_n - f_j) at the expansion point f (Sec. 3, eq. svrsurder).
__device__ inline void surrogate_nb(double fn, const Neighbours &nb, const PenaltyArgs &p, double &D, double &E) {
    switch (p.potential) {
        case SVR_PEN_HUBER: surrogate_pot<SVR_PEN_HUBER>(fn, nb, p.delta, D, E); break;
        case SVR_PEN_LOGCOSH: surrogate_pot<SVR_PEN_LOGCOSH>(fn, nb, p.delta, D, E); break;
        case SVR_PEN_HYPERBOLA: surrogate_pot<SVR_PEN_HYPERBOLA>(fn, nb, p.delta, D, E); break;
        default: surrogate_pot<SVR_PEN_QUADRATIC>(fn, nb, p.delta, D, E);
    }
}

__device__ inline void surrogate_at(const float *f, int n, const PenaltyArgs &p, double &D, double &E) {
    surrogate_nb((double)f[n], load_neighbours_of(f, n, p), p, D, E);
}

template <int POT>
__device__ inline double penalty_share_pot(double fn, const Neighbours &nb, double delta) {
    double r = 0.0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const double term = nb_weight(k) * pot_rho(POT, fn - (double)nb.v[k], delta);
        r = r + (nb.ok[k] ? term : 0.0);
    }
    return 0.5 * r;
}

// 1/2 sum_j w_nj rho(f_n - f_j): pixel n's share of R(f)
__device__ inline double penalty_share_at(const float *f, int n, const PenaltyArgs &p) {
    const int iy = n / p.nx, ix = n - iy * p.nx;
    const double fn = (double)f[n];
    const Neighbours nb = load_neighbours(f, ix, iy, p.nx, p.ny);
    switch (p.potential) {
        case SVR_PEN_HUBER: return penalty_share_pot<SVR_PEN_HUBER>(fn, nb, p.delta);
        case SVR_PEN_LOGCOSH: return penalty_share_pot<SVR_PEN_LOGCOSH>(fn, nb, p.delta);
        case SVR_PEN_HYPERBOLA: return penalty_share_pot<SVR_PEN_HYPERBOLA>(fn, nb, p.delta);
        default: return penalty_share_pot<SVR_PEN_QUADRATIC>(fn, nb, p.delta);
    }
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
