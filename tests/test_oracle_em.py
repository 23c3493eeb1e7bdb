"""Pins of the oracle's EM family (Sec. 2, Sec. 3, Appendix B of the paper)
and of its gradient family (Sec. 4): closed forms, invariants and special
cases that reduce to a textbook routine."""

import numpy as np
import pytest
import scipy.optimize

import datagen
import oracle


def _tiny_problem(nx=12, V=18, B=19, counts=3e4, beta=0.0, Ns=3, bg=0.1, seed=5, attenuation=False):
    P = datagen.make_problem(nx, nx, 3.0, V, B, 3.0, Ns, counts, attenuation=attenuation,
                             seed=seed, bg_frac=bg)
    A = oracle.system_matrix(P.geom, P.mu)
    w = P.w if bg > 0 else np.zeros_like(P.w)
    return P, A, oracle.Model(A, P.g, w, P.geom, Ns, beta=beta)


@pytest.fixture(scope="module")
def small():
    P = datagen.make_problem(**datagen.CONFIG_SMALL)
    A = oracle.system_matrix(P.geom, P.mu)
    return P, A


def test_adjoint_identity(small):
    """<A_t x, y> = <x, A_t^T y> (P2) for every subset of the partition."""
    P, A = small
    m = oracle.Model(A, P.g, P.w, P.geom, 6)
    rng = np.random.default_rng(0)
    for t in range(6):
        x = rng.uniform(size=A.shape[1])
        y = rng.uniform(size=len(m.rows[t]))
        lhs = float(np.dot(m.A_t[t] @ x, y))
        rhs = float(np.dot(x, m.AT_t[t] @ y))
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_partition_is_a_partition(small):
    """The subsets are disjoint, cover [M] and are balanced (Sec. 2.1)."""
    P, _ = small
    rows = oracle.subset_rows(P.geom, 6)
    allr = np.concatenate(rows)
    assert len(allr) == P.geom.n_rays and len(np.unique(allr)) == P.geom.n_rays
    assert len({len(r) for r in rows}) == 1


@pytest.mark.parametrize("bg", [0.0, 0.1])
def test_osem_count_preservation(small, bg):
    """P3: after an OSEM step on subset t, sum_n (A_t^T 1)_n f+_n equals
    sum_{m in S_t} g_m (A_t f)_m / (A_t f + w_t)_m (= sum g_m when w = 0)."""
    P, A = small
    w = P.w * (bg / 0.1)
    m = oracle.Model(A, P.g, w, P.geom, 6)
    rng = np.random.default_rng(1)
    f = rng.uniform(0.5, 2.0, (1, A.shape[1]))
    for t in range(6):
        fp = oracle.em.osem_step(m, f, t)
        Af = m.A_t[t] @ f[0]
        gt = m.g_t[t][0]
        yb = Af + m.w_t[t][0]
        seen = yb > 0  # rays that miss the image carry no information (ratio 0)
        expect = np.sum(gt[seen] * Af[seen] / yb[seen])
        got = np.sum(m.sens_t[t] * fp[0])
        assert abs(got - expect) <= 1e-11 * expect
        if bg == 0.0:
            assert abs(got - gt[seen].sum()) <= 1e-11 * gt.sum()


def test_mlem_monotone_likelihood(small):
    """P4: MLEM never decreases L (Sec. 2.2, surrogate property)."""
    P, A = small
    m = oracle.Model(A, P.g, P.w, P.geom, 1)
    f = np.ones((1, A.shape[1]))
    vals = [m.loglik(f)]
    oracle.mlem(m, f, 15, callback=lambda x: vals.append(m.loglik(x)))
    assert np.all(np.diff(vals) >= -1e-9 * np.abs(vals[1:]))
    assert vals[-1] > vals[0]


def test_osem_one_subset_is_mlem(small):
    """P6: OSEM with Ns = 1 is MLEM, bitwise."""
    P, A = small
    m = oracle.Model(A, P.g, P.w, P.geom, 1)
    f0 = np.ones((1, A.shape[1]))
    a = oracle.osem_epoch(m, f0, [0, 0, 0])
    b = oracle.mlem(m, f0, 3)
    np.testing.assert_array_equal(a, b)


def test_osem_additive_equals_multiplicative(small):
    """P10: f + (f / A_t^T 1) grad L_t(f) equals the multiplicative update
    (Sec. 4, eq. osem_additive vs Sec. 2.2, eq. Mstep)."""
    P, A = small
    m = oracle.Model(A, P.g, P.w, P.geom, 6)
    rng = np.random.default_rng(2)
    f = rng.uniform(0.5, 2.0, (1, A.shape[1]))
    for t in range(6):
        mult = oracle.em.osem_step(m, f, t)
        d = oracle.em._safe_div(f, m.sens_t[t])
        add = f + d * m.grad_L_t(f, t)
        np.testing.assert_allclose(add, mult, rtol=1e-13, atol=1e-13)


def test_subset_statistic_identity(small):
    """eq. subsetstat = eq. tau_t: Ns f (grad L_t + A_t^T 1) = Ns f A_t^T(g/ybar),
    and (1/Ns) sum_t tau_t = f A^T(g/ybar) from the full data."""
    P, A = small
    m = oracle.Model(A, P.g, P.w, P.geom, 6)
    f = np.random.default_rng(3).uniform(0.5, 2.0, (1, A.shape[1]))
    for t in range(6):
        np.testing.assert_allclose(m.tau_t(f, t), 6 * f * (m.grad_L_t(f, t) + m.sens_t[t]),
                                   rtol=1e-12, atol=1e-10)
    np.testing.assert_allclose(m.s_full(f), f * m.back_full(f), rtol=1e-12, atol=1e-10)


def test_svrem_one_subset_is_mlem():
    """P8: SVREM with Ns = 1, alpha = 1, beta = 0 is MLEM."""
    P, A, m = _tiny_problem(Ns=1)
    f0 = np.ones((1, A.shape[1]))
    s = oracle.SVREM(m, f0, alpha=1.0, eta=1)
    s.run([0] * 8)
    np.testing.assert_allclose(s.f, oracle.mlem(m, f0, 8), rtol=1e-11, atol=1e-12)


def test_svrem_map_em_monotone():
    """P5: SVREM with Ns = 1, alpha = 1 is full-data MAP-EM with separable
    surrogates, which never decreases Phi (Sec. 3)."""
    P, A, m = _tiny_problem(Ns=1, beta=0.5)
    f = np.ones((1, A.shape[1]))
    s = oracle.SVREM(m, f, alpha=1.0, eta=1)
    vals = [m.objective(s.f)]
    for _ in range(25):
        s.step(0)
        vals.append(m.objective(s.f))
    assert np.all(np.diff(vals) >= -1e-9 * np.abs(vals[1:]))
    assert vals[-1] > vals[0]


def test_svrem_first_step_is_full_statistic_mstep():
    """P13 (SVREM): at f = f_anc the update is (1-alpha) s_hat + alpha s_anc,
    and with s_hat^0 = s(f^0) the first iterate is the M-step of s(f^0)."""
    P, A, m = _tiny_problem(Ns=3, beta=0.3)
    f0 = np.random.default_rng(4).uniform(0.5, 2.0, (1, A.shape[1]))
    s = oracle.SVREM(m, f0, alpha=0.7, eta=1)
    s.step(2)
    np.testing.assert_allclose(s.f, m.mstep(f0 * m.back_full(f0), f0), rtol=1e-11, atol=1e-12)


def test_svrem_appendix_b_direction():
    """P7: with beta = 0 and s_hat = f (.) A^T 1 the SVREM update equals
    f + alpha h with Appendix B's closed-form direction h."""
    P, A, m = _tiny_problem(Ns=3)
    rng = np.random.default_rng(6)
    f_anc = rng.uniform(0.5, 2.0, (1, A.shape[1]))
    f = f_anc * rng.uniform(0.8, 1.2, f_anc.shape)
    alpha, t = 0.6, 1
    s = oracle.SVREM(m, f_anc, alpha=alpha, eta=1)
    s.anchor()
    s.k = 1
    s.f = f.copy()
    s.s_hat = f * m.sens
    s.step(t)
    d = lambda x: oracle.em._safe_div(x, m.sens)  # noqa: E731
    gradL = m.back_full(f_anc) - m.sens
    h = 3 * (d(f) * m.grad_L_t(f, t) - d(f_anc) * m.grad_L_t(f_anc, t)
             + d(f_anc) * gradL / 3 + (f - f_anc) * (m.sens_t[t] / m.sens - 1.0 / 3))
    np.testing.assert_allclose(s.f, f + alpha * h, rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("cls", ["SVRG", "SAGA", "SGA"])
def test_gradient_methods_one_subset_are_mlem(cls):
    """P9: Ns = 1, alpha = 1, beta = 0, d = f / A^T 1 turns every
    preconditioned gradient method into MLEM (Sec. 4, eq. osem_additive)."""
    P, A, m = _tiny_problem(Ns=1)
    f0 = np.ones((1, A.shape[1]))
    if cls == "SVRG":
        alg = oracle.SVRG(m, f0, 1.0, 1, precond=oracle.PRECOND_ITERATE)
    elif cls == "SAGA":
        alg = oracle.SAGA(m, f0, 1.0, precond=oracle.PRECOND_ITERATE)
    else:
        alg = oracle.SGA(m, f0, 1.0)
    alg.run([0] * 6)
    np.testing.assert_allclose(alg.f, oracle.mlem(m, f0, 6), rtol=1e-10, atol=1e-12)


def test_svrg_first_direction_is_full_gradient():
    """P13 (SVRG): at f = f_anc the direction is g_tilde = grad Phi(f_anc)/Ns."""
    P, A, m = _tiny_problem(Ns=3, beta=0.2)
    f0 = np.random.default_rng(8).uniform(0.5, 2.0, (1, A.shape[1]))
    alg = oracle.SVRG(m, f0, 1.5, 2, precond=oracle.PRECOND_SUBSET_FROZEN)
    alg.step(1)
    d = oracle.em._safe_div(f0, m.sens_t[1])
    expect = np.maximum(0, f0 + 1.5 * d * m.grad_Phi(f0) / 3)
    np.testing.assert_allclose(alg.f, expect, rtol=1e-11, atol=1e-12)


def test_saga_table_identity():
    """P14: after the table is filled at f, the SAGA direction at the same f
    is grad Phi(f) / Ns, computed through the full-data gradient."""
    P, A, m = _tiny_problem(Ns=4, beta=0.2)
    f0 = np.random.default_rng(9).uniform(0.5, 2.0, (1, A.shape[1]))
    alg = oracle.SAGA(m, f0, 2.0, precond=oracle.PRECOND_FULL_FROZEN)
    alg.step(3)
    d = oracle.em._safe_div(f0, m.sens)
    expect = np.maximum(0, f0 + 2.0 * d * m.grad_Phi(f0) / 4)
    np.testing.assert_allclose(alg.f, expect, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(sum(alg.q), m.grad_Phi(f0), rtol=1e-10, atol=1e-9)


def test_objective_is_poisson_loglik():
    """Phi with beta = 0 equals the Poisson log-likelihood up to the
    f-independent constant -sum log g! (Sec. 2.1, eq. pdf and log_likelihood)."""
    from scipy.special import gammaln
    P, A, m = _tiny_problem(Ns=2)
    f = np.random.default_rng(1).uniform(0.5, 2.0, (1, A.shape[1]))
    yb = A @ f[0] + P.w[0]
    g = P.g[0].astype(np.float64)
    logpmf = np.sum(g * np.log(yb) - yb - gammaln(g + 1))
    assert abs(m.objective(f) - (logpmf + np.sum(gammaln(g + 1)))) < 1e-8 * abs(logpmf)


def _kkt_residual(m, f):
    g = m.grad_Phi(f)[0]
    f = f[0]
    scale = np.abs(m.sens).max()
    pos = f > 1e-8 * f.max()
    return max(np.abs(g[pos]).max() / scale, max(0.0, g[~pos].max() / scale) if (~pos).any() else 0.0)


@pytest.mark.slow
def test_vr_methods_converge_to_lbfgsb_maximiser():
    """P15: long SVREM, SVRG and SAGA runs reach the MAP maximiser given by a
    library L-BFGS-B solve (the paper's reference method, Sec. 5.1), which
    satisfies the KKT conditions of the non-negativity constrained problem."""
    P, A, m = _tiny_problem(nx=8, V=12, B=13, counts=2e4, Ns=3, beta=0.2, seed=3)
    N = A.shape[1]

    def negphi(x):
        f = x[None, :]
        return -m.objective(f), -m.grad_Phi(f)[0]

    f_init = oracle.osem_epoch(m, np.ones((1, N)), range(3))
    res = scipy.optimize.minimize(negphi, f_init[0], jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * N,
                                  options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12, maxcor=30))
    fstar = res.x[None, :]
    assert _kkt_residual(m, fstar) < 1e-6
    assert np.count_nonzero(fstar == 0) > 0  # some constraints are active
    order = datagen.make_order(3, 3000, seed=1)
    runs = {
        "SVREM": oracle.SVREM(m, f_init, alpha=0.7, eta=1),
        "SVRG": oracle.SVRG(m, f_init, 1.0, 2, precond=oracle.PRECOND_SUBSET_FROZEN),
        "SAGA": oracle.SAGA(m, f_init, 0.5, precond=oracle.PRECOND_SUBSET_FROZEN),
    }
    for name, alg in runs.items():
        alg.run(order)
        rel = np.linalg.norm(alg.f - fstar) / np.linalg.norm(fstar)
        assert rel < 1e-6, (name, rel)
