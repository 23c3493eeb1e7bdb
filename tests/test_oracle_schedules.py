"""Pins of the oracle's schedules and of its subset partition.

* SEM (Sec. 2.3, eq. tempsem) and its decaying weight a_k = a_0/(0.001 k + 1)
  (Sec. 5.1): the unit weight reduces it to SVREM with one subset; the first
  step is the M-step of the subset statistic at the start; with the harmonic
  schedule a_k = 1/(k + 1) (decay 1) the running statistic is exactly the
  arithmetic mean of the statistics seen so far (the Robbins-Monro average);
  the paper's schedule halves the weight at k = 1000.
* BSREM (Sec. 5.1): without decay it is SGA; at k = 1000 its step is half the
  starting step.
* The anchor period of SVREM and SVRG (eq. tempsvrem, eq. svrg_update): a full
  pass at every k with k mod (eta Ns) = 0 and only there.  At an anchor the
  variance-reduced update collapses to the full-data update (SVREM with
  alpha = 1: the M-step of the full statistic s(f^k); SVRG: a step along
  grad Phi(f^k)/Ns), which no other iteration takes.
* The interleaved partition (Sec. 2.1): subsets are to be balanced, the
  emission probabilities sum_{m in S_t} a_mn nearly independent of t.
"""

import math

import numpy as np
import pytest

import datagen
import oracle


def _model(nx=12, V=18, B=19, Ns=3, beta=0.02, counts=3e4, seed=5):
    P = datagen.make_problem(nx, nx, 3.0, V, B, 3.0, Ns, counts, attenuation=False, seed=seed, bg_frac=0.1)
    A = oracle.system_matrix(P.geom)
    return P, oracle.Model(A, P.g, P.w, P.geom, Ns, beta=beta)


def _start(m, P):
    """One OSEM epoch from the uniform image (the paper's initialisation)."""
    return oracle.osem_epoch(m, np.ones((1, P.geom.n_pixels)), range(m.Ns))


# ---------------------------------------------------------------------------
# SEM
# ---------------------------------------------------------------------------

def test_sem_with_unit_weight_is_single_subset_svrem():
    """SEM with a_k = 1 (no decay) and one subset equals SVREM with one subset
    and alpha = 1 bitwise: every SVREM iteration is then an anchor, so its
    statistic tau(f) - tau(f_anc) + s_anc collapses to tau(f)."""
    P, m = _model(Ns=1)
    f0 = _start(m, P)
    sem = oracle.SEM(m, f0, a0=1.0, decay=0.0)
    svrem = oracle.SVREM(m, f0, alpha=1.0, eta=1)
    for _ in range(6):
        sem.step(0)
        svrem.step(0)
        assert np.array_equal(sem.f, svrem.f)
        assert np.array_equal(sem.s_hat, svrem.s_hat)


def test_sem_first_step_is_the_mstep_of_the_subset_statistic():
    """a_0 = 1: the first SEM iterate is the M-step of tau_t0(f^0), whatever
    the starting statistic."""
    P, m = _model()
    f0 = _start(m, P)
    sem = oracle.SEM(m, f0)
    sem.s_hat = np.full_like(f0, 1e6)  # irrelevant when a_0 = 1
    sem.step(2)
    assert np.array_equal(sem.f, m.mstep(m.tau_t(f0, 2), f0))


def test_sem_harmonic_schedule_is_the_running_mean():
    """With decay 1 the weights a_k = 1/(k + 1) make s_hat^K the arithmetic mean
    of tau_{t_j}(f^j), j < K (the stochastic-approximation average)."""
    P, m = _model()
    f0 = _start(m, P)
    sem = oracle.SEM(m, f0, a0=1.0, decay=1.0)
    order = datagen.make_order(m.Ns, 12, seed=7)
    taus = []
    for t in order:
        taus.append(m.tau_t(sem.f, int(t)))
        sem.step(int(t))
        mean = sum(taus) / len(taus)
        assert np.allclose(sem.s_hat, mean, rtol=1e-12, atol=1e-12 * np.abs(mean).max())


def test_sem_weight_halves_at_k_1000():
    """The schedule of Sec. 5.1, a_k = 1/(0.001 k + 1), is 1/2 at k = 1000: a step
    taken there equals a step with the constant weight 1/2 from the same state."""
    P, m = _model()
    f0 = _start(m, P)
    a = oracle.SEM(m, f0)
    a.s_hat = m.s_full(f0)
    a.k = 1000
    b = oracle.SEM(m, f0, a0=0.5, decay=0.0)
    b.s_hat = a.s_hat.copy()
    a.step(1)
    b.step(1)
    assert np.array_equal(a.f, b.f)


# ---------------------------------------------------------------------------
# BSREM
# ---------------------------------------------------------------------------

def test_bsrem_without_decay_is_sga():
    P, m = _model()
    f0 = _start(m, P)
    b = oracle.BSREM(m, f0, alpha=0.8, decay=0.0)
    s = oracle.SGA(m, f0, alpha=0.8)
    for t in datagen.make_order(m.Ns, 9, seed=3):
        b.step(int(t))
        s.step(int(t))
        assert np.array_equal(b.f, s.f)


def test_bsrem_step_halves_at_k_1000():
    """At k = 0 the BSREM step is SGA's with alpha, at k = 1000 SGA's with alpha/2
    (Sec. 5.1, alpha_k = alpha/(0.001 k + 1))."""
    P, m = _model()
    f0 = _start(m, P)
    for k, scale in ((0, 1.0), (1000, 0.5)):
        b = oracle.BSREM(m, f0, alpha=0.9)
        b.k = k
        s = oracle.SGA(m, f0, alpha=0.9 * scale)
        b.step(1)
        s.step(1)
        assert np.array_equal(b.f, s.f)
    # and the two steps differ (the decay acts)
    b0, b1 = oracle.BSREM(m, f0, alpha=0.9), oracle.BSREM(m, f0, alpha=0.9)
    b1.k = 1000
    b0.step(1)
    b1.step(1)
    assert not np.allclose(b0.f, b1.f, rtol=1e-6)


# ---------------------------------------------------------------------------
# Anchor period of SVREM and SVRG
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("eta", [1, 2, 3])
def test_svrem_takes_the_full_mstep_exactly_at_anchors(eta):
    """SVREM, alpha = 1: f^{k+1} = M-step(s(f^k)) at k = 0, eta Ns, 2 eta Ns, ...
    (the anchor iterations) and at no other k; ceil(n / (eta Ns)) full passes."""
    P, m = _model(Ns=3)
    f0 = _start(m, P)
    alg = oracle.SVREM(m, f0, alpha=1.0, eta=eta)
    order = datagen.make_order(m.Ns, 20, seed=11)
    period = eta * m.Ns
    for k, t in enumerate(order):
        f = alg.f.copy()
        full = m.mstep(m.s_full(f), f)
        alg.step(int(t))
        err = np.linalg.norm(alg.f - full) / np.linalg.norm(full)
        if k % period == 0:
            assert err <= 1e-13, (k, err)
        else:
            assert err > 1e-8, (k, err)
    assert alg.n_anchors == math.ceil(len(order) / period)


@pytest.mark.parametrize("eta", [1, 2])
def test_svrg_takes_the_full_gradient_step_exactly_at_anchors(eta):
    """SVRG: at an anchor the direction is g_tilde = grad Phi(f^k)/Ns, so
    f^{k+1} = max(0, f^k + alpha d grad Phi(f^k)/Ns); elsewhere it is not."""
    P, m = _model(Ns=3)
    f0 = _start(m, P)
    alpha = 0.5
    alg = oracle.SVRG(m, f0, alpha=alpha, eta=eta, precond=oracle.PRECOND_FULL_FROZEN)
    d = np.zeros_like(f0)
    np.divide(f0, m.sens, out=d, where=m.sens != 0)
    order = datagen.make_order(m.Ns, 14, seed=12)
    period = eta * m.Ns
    for k, t in enumerate(order):
        f = alg.f.copy()
        full = np.maximum(0.0, f + alpha * d * m.grad_Phi(f) / m.Ns)
        alg.step(int(t))
        err = np.linalg.norm(alg.f - full) / np.linalg.norm(full)
        if k % period == 0:
            assert err <= 1e-13, (k, err)
        else:
            assert err > 1e-8, (k, err)
    assert alg.n_anchors == math.ceil(len(order) / period)


# ---------------------------------------------------------------------------
# Partition
# ---------------------------------------------------------------------------

def test_interleaved_subsets_are_balanced():
    """Sec. 2.1: sum_{m in S_t} a_mn nearly independent of t.  With attenuation
    a view's weight sum of an off-centre pixel depends on the view angle, so only
    subsets that each span the whole arc are balanced: on the 64 x 64
    attenuated problem (6 subsets) every A_t^T 1 is within 5% (relative L2) and
    25% (worst pixel) of A^T 1 / Ns; a partition into contiguous arcs is off by
    about 66% (and 170%)."""
    P = datagen.make_problem(**datagen.CONFIG_SMALL)
    A = oracle.system_matrix(P.geom, P.mu)
    m = oracle.Model(A, P.g, P.w, P.geom, P.n_subsets)
    seen = m.sens > 0
    ref = m.sens[seen] / m.Ns
    dev = m.sens_t[:, seen] - ref
    rel_l2 = np.linalg.norm(dev) / (math.sqrt(m.Ns) * np.linalg.norm(ref))
    worst = np.max(np.abs(dev) / ref)
    assert rel_l2 <= 0.05, rel_l2
    assert worst <= 0.25, worst
    # each subset has the same number of views and its views cover the arc
    rows = oracle.subset_rows(P.geom, m.Ns)
    for t, r in enumerate(rows):
        views = np.unique(r // P.geom.n_bins)
        assert len(views) == P.geom.n_views // m.Ns
        assert views.min() < m.Ns and views.max() >= P.geom.n_views - m.Ns
