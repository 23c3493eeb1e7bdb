"""Pins of the oracle's variants: the modified likelihood of Sec. 2.3
(eq. modified_LL) used by the gradient methods, and the SAGA-type online EM
of the remark after eq. tempsvrem.

Each pin checks the oracle against something other than itself: the
analytic properties the paper states for the modified likelihood (the
quadratic expansion about eps, C^1 matching, constant curvature, unchanged
maximisers for small eps), finite differences, textbook special cases (MLEM)
and an independent L-BFGS-B maximiser.
"""

import numpy as np
import pytest
import scipy.optimize

import datagen
import oracle


def _problem(nx=8, V=12, B=13, counts=2e4, Ns=3, beta=0.0, bg=0.1, seed=3, eps=0.0):
    P = datagen.make_problem(nx, nx, 3.0, V, B, 3.0, Ns, counts, attenuation=False, seed=seed, bg_frac=bg)
    A = oracle.system_matrix(P.geom)
    w = P.w if bg > 0 else np.zeros_like(P.w)
    return P, A, oracle.Model(A, P.g, w, P.geom, Ns, beta=beta, ll_eps=eps)


# ---------------------------------------------------------------------------
# modified likelihood (eq. modified_LL)
# ---------------------------------------------------------------------------

def _phi(g, l):
    return g * np.log(l) - l


def test_modified_rows_equal_plain_off_the_modified_region():
    rng = np.random.default_rng(0)
    g = rng.integers(0, 20, 1000).astype(float)
    yb = rng.uniform(0.01, 3.0, 1000)
    w = np.where(rng.uniform(size=1000) < 0.5, 0.0, 0.1)
    eps = 0.7
    plain = oracle.loglik_rows(g, yb, w)
    mod = oracle.loglik_rows(g, yb, w, eps)
    keep = (w > 0) | (yb > eps) | (g == 0)
    assert np.array_equal(plain[keep], mod[keep])
    assert np.array_equal(oracle.lik_ratio(g, yb, w)[keep], oracle.lik_ratio(g, yb, w, eps)[keep])
    # g = 0 rows: phi = -l in both forms, ratio 0
    z = g == 0
    assert np.array_equal(mod[z], -yb[z]) and np.all(oracle.lik_ratio(g, yb, w, eps)[z] == 0)


def test_modified_value_is_the_second_order_expansion_about_eps():
    """Below eps the modified term is the Taylor polynomial of degree 2 of
    phi about eps: it matches phi, phi' at eps (C^1), and its second
    difference is the constant phi''(eps) = -g/eps^2."""
    g, eps = 7.0, 0.4
    w = np.zeros(1)
    f = lambda l: oracle.loglik_rows(np.array([g]), np.array([l]), w, eps)[0]
    assert f(eps) == pytest.approx(_phi(g, eps), rel=1e-15)
    h = 1e-6
    left = (f(eps) - f(eps - h)) / h
    right = (f(eps + h) - f(eps)) / h
    assert left == pytest.approx(g / eps - 1.0, rel=1e-5)
    assert right == pytest.approx(g / eps - 1.0, rel=1e-5)
    for l in (-0.5, 0.0, 0.1, 0.3):
        h = 1e-3
        d2 = (f(l + h) - 2 * f(l) + f(l - h)) / h ** 2
        assert d2 == pytest.approx(-g / eps ** 2, rel=1e-6)
    # finite where the plain likelihood is -inf
    assert np.isfinite(f(0.0)) and oracle.loglik_rows(np.array([g]), np.array([0.0]), w)[0] == -np.inf


def test_modified_ratio_is_one_plus_the_derivative():
    rng = np.random.default_rng(1)
    g = rng.integers(1, 30, 400).astype(float)
    yb = rng.uniform(-0.3, 2.0, 400)
    w = np.zeros(400)
    eps = 0.8
    h = 1e-6
    d = (oracle.loglik_rows(g, yb + h, w, eps) - oracle.loglik_rows(g, yb - h, w, eps)) / (2 * h)
    r = oracle.lik_ratio(g, yb, w, eps)
    away = np.abs(yb - eps) > 2 * h
    np.testing.assert_allclose(r[away] - 1.0, d[away], rtol=1e-6, atol=1e-6)
    # Lipschitz derivative (Theorem 1's premise): |phi'(a) - phi'(b)| <= g/eps^2 |a - b| on the whole line
    a, b = yb[:200], yb[200:]
    lhs = np.abs(oracle.lik_ratio(g[:200], a, w[:200], eps) - oracle.lik_ratio(g[:200], b, w[:200], eps))
    assert np.all(lhs <= g[:200] / eps ** 2 * np.abs(a - b) * (1 + 1e-12) + 1e-12)


def test_modified_model_gradient_matches_finite_differences():
    """With w = 0 and eps at the median of ybar many rows sit in the modified
    branch; the model's grad Phi (through A^T of the modified ratio) matches
    central differences of its modified objective."""
    P, A, m0 = _problem(bg=0.0, beta=0.1)
    f = oracle.osem_epoch(m0, np.ones((1, A.shape[1])), range(3))
    f[0, ::3] *= 0.05
    yb = A @ f[0]
    eps = float(np.median(yb[P.g[0] > 0]))
    m = oracle.Model(A, P.g, np.zeros_like(P.w), P.geom, 3, beta=0.1, ll_eps=eps)
    assert np.count_nonzero((yb <= eps) & (P.g[0] > 0)) > 10
    g = m.grad_Phi(f)[0]
    rng = np.random.default_rng(2)
    for n in rng.choice(A.shape[1], 12, replace=False):
        h = 1e-5 * max(1.0, abs(f[0, n]))
        fp, fm = f.copy(), f.copy()
        fp[0, n] += h
        fm[0, n] -= h
        fd = (m.objective(fp) - m.objective(fm)) / (2 * h)
        assert fd == pytest.approx(g[n], rel=1e-5, abs=1e-6 * np.abs(g).max())
    # the subset gradients add up to the full gradient
    tot = sum(m.grad_Phi_t(f, t) for t in range(3))
    np.testing.assert_allclose(tot, m.grad_Phi(f), rtol=1e-12, atol=1e-9)


def test_modified_likelihood_is_inert_with_background():
    """Every row has w > 0: the modified likelihood changes nothing (the
    paper's remark that it is not needed when the background is nonzero)."""
    P, A, m = _problem(bg=0.1, beta=0.05)
    mm = oracle.Model(A, P.g, P.w, P.geom, 3, beta=0.05, ll_eps=1e3)
    f0 = oracle.osem_epoch(m, np.ones((1, A.shape[1])), range(3))
    order = datagen.make_order(3, 9, seed=4)
    a = oracle.SVRG(m, f0, 0.5, 1).run(order)
    b = oracle.SVRG(mm, f0, 0.5, 1).run(order)
    assert np.array_equal(a, b)
    assert mm.objective(b) == pytest.approx(m.objective(a), rel=1e-14)  # same terms, one FP64 sum


@pytest.mark.slow
def test_small_eps_keeps_the_maximiser():
    """For eps below the maximiser's smallest ybar over rows with counts, the
    L-BFGS-B maximiser of the plain penalised likelihood (w = 0) also
    satisfies the KKT conditions of the modified problem (Sec. 2.3: a small
    enough eps does not change the solution set)."""
    P, A, m = _problem(bg=0.0, beta=0.2, counts=3e4)
    N = A.shape[1]

    def negphi(x):
        f = x[None, :]
        return -m.objective(f), -m.grad_Phi(f)[0]

    f_init = oracle.osem_epoch(m, np.ones((1, N)), range(3))
    res = scipy.optimize.minimize(negphi, f_init[0], jac=True, method="L-BFGS-B", bounds=[(0, None)] * N,
                                  options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12, maxcor=30))
    fstar = res.x[None, :]
    yb = A @ fstar[0]
    eps = 0.5 * float(yb[P.g[0] > 0].min())
    mm = oracle.Model(A, P.g, np.zeros_like(P.w), P.geom, 3, beta=0.2, ll_eps=eps)
    assert mm.objective(fstar) == pytest.approx(m.objective(fstar), rel=1e-14)
    gp, gm = m.grad_Phi(fstar)[0], mm.grad_Phi(fstar)[0]
    np.testing.assert_allclose(gm, gp, rtol=1e-12, atol=1e-12 * np.abs(gp).max())
    pos = fstar[0] > 1e-8 * fstar.max()
    scale = np.abs(m.sens).max()
    assert np.abs(gm[pos]).max() / scale < 1e-6 and gm[~pos].max(initial=0.0) / scale < 1e-6
    # a large eps does change it: the modified gradient no longer vanishes there
    big = oracle.Model(A, P.g, np.zeros_like(P.w), P.geom, 3, beta=0.2, ll_eps=4.0 * float(np.median(yb)))
    assert np.abs(big.grad_Phi(fstar)[0][pos]).max() / scale > 1e-3


# ---------------------------------------------------------------------------
# SAGA-type online EM (remark after eq. tempsvrem)
# ---------------------------------------------------------------------------

def test_sagaem_one_subset_unit_step_is_mlem():
    """Ns = 1, alpha = 1, beta = 0: s_hat = tau(f) - S + S = s(f), so every
    iteration is the MLEM update f * A^T(g / ybar) / A^T 1."""
    P, A, m = _problem(Ns=1)
    f0 = np.ones((1, A.shape[1]))
    f = oracle.SAGAEM(m, f0, 1.0).run([0] * 6)
    ref = oracle.mlem(m, f0, 6)
    np.testing.assert_allclose(f, ref, rtol=1e-12, atol=1e-12 * ref.max())


def test_sagaem_first_step_is_the_full_statistic_step():
    """With the table fresh at f^(0), tau_t(f^(0)) - S_t = 0 and s_hat^1 = s(f^(0))
    for any alpha and t: the first image is the M-step of the full
    statistic, the same as SVREM's first step."""
    P, A, m = _problem(beta=0.1)
    f0 = oracle.osem_epoch(m, np.ones((1, A.shape[1])), range(3))
    for alpha, t in ((0.3, 0), (1.0, 2), (1.7, 1)):
        a = oracle.SAGAEM(m, f0, alpha)
        a.step(t)
        ref = m.mstep(m.s_full(f0), f0)
        np.testing.assert_allclose(a.f, ref, rtol=1e-12, atol=1e-14)
        b = oracle.SVREM(m, f0, alpha, 1)
        b.step(t)
        np.testing.assert_allclose(a.f, b.f, rtol=1e-12, atol=1e-14)


def test_sagaem_refresh_stores_the_statistic_before_the_update():
    P, A, m = _problem(beta=0.1)
    f0 = oracle.osem_epoch(m, np.ones((1, A.shape[1])), range(3))
    a = oracle.SAGAEM(m, f0, 0.8)
    a.run([1, 2, 0], refresh=[0, 0, 2])
    before = a.f.copy()
    S_old = [s.copy() for s in a.S]
    s_hat_old = a.s_hat.copy()
    a.step(1, 2)
    np.testing.assert_allclose(a.S[2], m.tau_t(before, 2), rtol=1e-14)
    for t in (0, 1):
        assert np.array_equal(a.S[t], S_old[t])
    # the statistic used the old entry S_1 and the old table mean
    expect = 0.2 * s_hat_old + 0.8 * (m.tau_t(before, 1) - S_old[1] + sum(S_old) / 3)
    np.testing.assert_allclose(a.s_hat, expect, rtol=1e-13)


@pytest.mark.slow
def test_sagaem_converges_to_the_map_point():
    """A long SAGA-EM run reaches the MAP maximiser of an independent L-BFGS-B
    solve (as the P15 pin does for SVREM, SVRG and SAGA)."""
    P, A, m = _problem(beta=0.2, seed=3)
    N = A.shape[1]

    def negphi(x):
        f = x[None, :]
        return -m.objective(f), -m.grad_Phi(f)[0]

    f_init = oracle.osem_epoch(m, np.ones((1, N)), range(3))
    res = scipy.optimize.minimize(negphi, f_init[0], jac=True, method="L-BFGS-B", bounds=[(0, None)] * N,
                                  options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12, maxcor=30))
    fstar = res.x[None, :]
    order = datagen.make_order(3, 3000, seed=1)
    refresh = datagen.make_order(3, 3000, seed=2)
    for rf in (None, refresh):
        f = oracle.SAGAEM(m, f_init, 0.7).run(order, rf)
        rel = np.linalg.norm(f - fstar) / np.linalg.norm(fstar)
        assert rel < 1e-6, rel


# ---------------------------------------------------------------------------
# iteration-dependent preconditioner: the fixed-point bias of Sec. 4
# ---------------------------------------------------------------------------

def _bias_problem():
    """12 x 12, 10 views in 4 interleaved subsets of 3, 3, 2 and 2 views: the
    subset sensitivities A_t^T 1 differ by half, so d_t(f) = f / A_t^T 1 differ."""
    P = datagen.make_problem(12, 12, 3.0, 10, 19, 3.0, 4, 3e4, attenuation=False, seed=5, bg_frac=0.1)
    A = oracle.system_matrix(P.geom)
    m = oracle.Model(A, P.g, P.w, P.geom, 4, beta=0.05)
    f0 = oracle.osem_epoch(m, np.ones((1, 144)), range(4))
    return m, f0


def _kkt_residual(m, f):
    """|grad Phi| on the support of f, relative to |A^T 1| there."""
    g = m.grad_Phi(f)[0]
    sup = f[0] > 1e-8 * f.max()
    return float(np.linalg.norm(g[sup]) / np.linalg.norm(m.sens[sup]))


def _preconditioned_sum(m, f):
    """|sum_t d_t(f) grad Phi_t(f)| on the support, relative to |f| there."""
    s = sum(oracle.em._safe_div(f, m.sens_t[t]) * m.grad_Phi_t(f, t) for t in range(m.Ns))[0]
    sup = f[0] > 1e-8 * f.max()
    return float(np.linalg.norm(s[sup]) / np.linalg.norm(f[0][sup]))


def test_iterate_preconditioner_fixed_point_bias():
    """Sec. 4, remark on iteration-dependent preconditioners: a preconditioned
    incremental ascent with d_t(f^k) and a vanishing step converges to a point
    where sum_t d_t(f*) grad Phi_t(f*) = 0, which is not the MAP point
    (grad Phi(f*) != 0 on the support) unless all d_t coincide.  BSREM (step
    1/(0.01 k + 1), cyclic order) shows it: the preconditioned sum goes to 0 like
    the step while the KKT residual stays put, 3% away from the MAP image.
    SVRG reaches the MAP point with the frozen preconditioner d = f^0 / A^T 1
    and also with d_t(f^k): its direction at a fixed point is grad Phi / Ns."""
    m, f0 = _bias_problem()
    b = oracle.BSREM(m, f0, alpha=1.0, decay=0.01)
    b.run(np.tile(np.arange(4), 5000))
    bias_sum, bias_kkt = _preconditioned_sum(m, b.f), _kkt_residual(m, b.f)
    assert bias_sum <= 1e-3, bias_sum
    assert bias_kkt >= 5e-3, bias_kkt
    assert bias_kkt >= 10 * bias_sum
    s = oracle.SVRG(m, f0, alpha=1.0, eta=2, precond=oracle.PRECOND_FULL_FROZEN)
    s.run(np.tile(np.arange(4), 3000))
    assert _kkt_residual(m, s.f) <= 1e-10
    assert _preconditioned_sum(m, s.f) >= 1e-2  # the MAP point is not BSREM's fixed point
    si = oracle.SVRG(m, f0, alpha=0.5, eta=2, precond=oracle.PRECOND_ITERATE)
    si.run(np.tile(np.arange(4), 3000))
    assert _kkt_residual(m, si.f) <= 1e-5
    d_map = np.linalg.norm(b.f - s.f) / np.linalg.norm(s.f)
    assert d_map >= 1e-2, d_map
    # the MAP point is the L-BFGS-B maximiser of Phi on f >= 0 (Sec. 5.1's reference method)
    res = scipy.optimize.minimize(lambda x: -m.objective(x[None]), f0[0],
                                  jac=lambda x: -m.grad_Phi(x[None])[0], method="L-BFGS-B",
                                  bounds=[(0, None)] * f0.size,
                                  options=dict(maxiter=5000, ftol=1e-15, gtol=1e-12))
    assert np.linalg.norm(res.x - s.f[0]) / np.linalg.norm(s.f) <= 1e-5
