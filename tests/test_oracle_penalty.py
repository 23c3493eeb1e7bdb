"""Pins of the oracle's penalty (Sec. 3, Table 1) and M-step root."""

import json
import math
import os

import numpy as np
import pytest

import oracle
from oracle.penalty import potential

POTS = [oracle.POT_QUADRATIC, oracle.POT_HUBER, oracle.POT_LOGCOSH, oracle.POT_HYPERBOLA]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("kind", POTS)
def test_potential_table_consistency(kind):
    """rho' is the derivative of rho and gamma = rho'(t)/t (Table 1);
    Assumption 1: rho even, rho' non-decreasing, gamma non-increasing on t>0."""
    rho, drho, gam = potential(kind, 0.7)
    t = np.linspace(-5, 5, 2001)
    h = 1e-6
    fd = (rho(t + h) - rho(t - h)) / (2 * h)
    np.testing.assert_allclose(fd, drho(t), atol=2e-6)
    nz = np.abs(t) > 1e-3
    np.testing.assert_allclose(gam(t[nz]) * t[nz], drho(t[nz]), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(rho(t), rho(-t), rtol=1e-14)
    assert np.all(np.diff(drho(t)) >= -1e-15)
    tp = t[t > 0]
    assert np.all(np.diff(gam(tp)) <= 1e-15)
    assert 0 < gam(np.array([1e-12]))[0] < np.inf


def _rand_img(rng, S, ny, nx):
    return rng.uniform(0.0, 3.0, (S, ny * nx))


@pytest.mark.parametrize("kind", POTS)
@pytest.mark.parametrize("axial", [False, True])
def test_grad_is_finite_difference(kind, axial):
    """P12: grad R equals a central finite difference of R."""
    rng = np.random.default_rng(5)
    S, ny, nx = (3 if axial else 1), 5, 6
    f = _rand_img(rng, S, ny, nx)
    g = oracle.penalty_grad(f, ny, nx, kind, 0.8, axial)
    h = 1e-6
    for idx in rng.choice(S * ny * nx, 25, replace=False):
        e = np.zeros(S * ny * nx)
        e[idx] = h
        e = e.reshape(S, ny * nx)
        fd = (oracle.penalty_value(f + e, ny, nx, kind, 0.8, axial)
              - oracle.penalty_value(f - e, ny, nx, kind, 0.8, axial)) / (2 * h)
        assert abs(fd - g.ravel()[idx]) < 1e-6 * (1 + abs(fd))


@pytest.mark.parametrize("kind", POTS)
def test_grad_of_constant_is_zero(kind):
    """P12: grad R(const) = 0 and R(const) = 0."""
    f = np.full((2, 30), 1.7)
    np.testing.assert_array_equal(oracle.penalty_grad(f, 5, 6, kind, 0.5, True), 0.0)
    assert oracle.penalty_value(f, 5, 6, kind, 0.5, True) == 0.0


def test_quadratic_homogeneity():
    """P12: for rho = t^2/2, R is 2-homogeneous: <grad R(f), f> = 2 R(f)."""
    rng = np.random.default_rng(2)
    f = _rand_img(rng, 1, 7, 9)
    g = oracle.penalty_grad(f, 7, 9)
    assert abs(np.sum(g * f) - 2 * oracle.penalty_value(f, 7, 9)) < 1e-10


def test_quadratic_penalty_explicit_small():
    """2x2 image: R = 1/4 sum_n sum_j w (f_n - f_j)^2 over the 3 neighbours of each pixel."""
    f = np.array([[1.0, 2.0, 4.0, 8.0]])  # (iy,ix): (0,0)=1 (0,1)=2 (1,0)=4 (1,1)=8
    r = 1 / math.sqrt(2)
    pairs = [(1, 2, 1.0), (1, 4, 1.0), (2, 8, 1.0), (4, 8, 1.0), (1, 8, r), (2, 4, r)]
    R = sum(w * (a - b) ** 2 / 2 for a, b, w in pairs)  # each unordered pair twice * 1/2 * rho
    assert abs(oracle.penalty_value(f, 2, 2) - R) < 1e-13


@pytest.mark.parametrize("kind", POTS)
def test_surrogate_gradient_match(kind):
    """The M-step's penalty term at f = f_k reproduces grad R (surrogate
    property, Sec. 2.2 and Sec. 3): f_k * sum d - sum d f_j = grad R(f_k)."""
    rng = np.random.default_rng(9)
    f = _rand_img(rng, 1, 6, 7)
    D, E = oracle.surrogate_terms(f, 6, 7, kind, 0.6)
    np.testing.assert_allclose(f * D - E, oracle.penalty_grad(f, 6, 7, kind, 0.6),
                               rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kind", POTS)
def test_parabolic_surrogate_majorises(kind):
    """The parabolic surrogate of Sec. 3 lies above rho and touches it at f_k."""
    rho, drho, gam = potential(kind, 0.9)
    rng = np.random.default_rng(4)
    fn_k, fj_k = rng.uniform(0, 3, 500), rng.uniform(0, 3, 500)
    fn, fj = rng.uniform(0, 3, 500), rng.uniform(0, 3, 500)
    tk = fn_k - fj_k
    hat = (rho(tk) + drho(tk) * (fn - fj - tk)
           + gam(tk) * ((fn - fn_k) ** 2 + (fj - fj_k) ** 2))
    assert np.all(hat >= rho(fn - fj) - 1e-12)
    hat0 = rho(tk)
    np.testing.assert_allclose(hat0, rho(tk))


def test_mstep_root_golden():
    """P11: hand-solved roots of a/f - 2bf + c = 0 (tests/golden/mstep_roots.json)."""
    with open(os.path.join(GOLDEN, "mstep_roots.json")) as fh:
        cases = json.load(fh)["cases"]
    for cse in cases:
        f = oracle.mstep_root(cse["a"], cse["b"], cse["c"], 1.0)
        assert abs(float(f) - cse["f"]) <= 1e-15 * max(1.0, cse["f"]), cse


def test_mstep_root_residual_and_limits():
    """P11: residual of a/f - 2bf + c at the root, the b -> 0 limit -a/c, and the
    stable and textbook forms agreeing where both are well conditioned."""
    rng = np.random.default_rng(1)
    a = rng.uniform(1e-3, 10, 10000)
    b = 10 ** rng.uniform(-8, 2, 10000)
    c = rng.uniform(-20, 20, 10000)
    f = oracle.mstep_root(a, b, c, 1.0)
    assert np.all(f > 0)
    res = a / f - 2 * b * f + c
    scale = a / f + 2 * b * f + np.abs(c)
    assert np.max(np.abs(res) / scale) < 1e-12
    # stable and textbook forms agree where both are well conditioned
    m = (c > 0.1)
    tb = (c[m] + np.sqrt(c[m] ** 2 + 8 * a[m] * b[m])) / (4 * b[m])
    np.testing.assert_allclose(f[m], tb, rtol=1e-12)
    # beta -> 0 is continuous to the linear solution -a/c (c < 0)
    a1, c1 = 2.5, -3.0
    for bb in (1e-6, 1e-9, 1e-12):
        assert abs(oracle.mstep_root(a1, bb, c1, 1.0) - (-a1 / c1)) < 10 * bb
    assert oracle.mstep_root(a1, 0.0, c1, 1.0) == -a1 / c1
    # a <= 0 readings
    assert oracle.mstep_root(-1.0, 1.0, 5.0, 1.0) == 0.0
    assert oracle.mstep_root(0.0, 2.0, 3.0, 1.0) == 0.75
    assert oracle.mstep_root(0.0, 2.0, -3.0, 1.0) == 0.0
    # unseen pixel
    assert oracle.mstep_root(1.0, 1.0, 1.0, 0.0) == 0.0
