"""Planted mistakes: each test swaps a plausible bug into the oracle (on the
CPU, through monkeypatch) and checks that a pin catches it.  This shows the
pins are strong enough to trust the oracle they guard."""

import numpy as np
import pytest

import datagen
import oracle
import oracle.em as em
import oracle.gradient as gradient
import oracle.geometry as geometry
import oracle.penalty as penalty

import test_oracle_em as T_em
import test_oracle_penalty as T_pen
import test_oracle_schedules as T_sch
import test_oracle_siddon as T_sid
import test_oracle_variants as T_var


@pytest.fixture(scope="module")
def small():
    P = datagen.make_problem(**datagen.CONFIG_SMALL)
    return P, oracle.system_matrix(P.geom, P.mu)


def test_dropped_background_is_caught(small, monkeypatch):
    def ratio_no_bg(self, f, t):
        yb = (self.A_t[t] @ np.atleast_2d(f).T).T
        out = np.zeros_like(yb)
        np.divide(self.g_t[t], yb, out=out, where=yb > 0)
        return out
    monkeypatch.setattr(em.Model, "ratio_t", ratio_no_bg)
    with pytest.raises(AssertionError):
        T_em.test_osem_count_preservation(small, 0.1)


def test_penalty_sign_is_caught(monkeypatch):
    orig = penalty.penalty_grad
    monkeypatch.setattr(penalty, "penalty_grad", lambda *a, **k: -orig(*a, **k))
    monkeypatch.setattr(oracle, "penalty_grad", penalty.penalty_grad)
    with pytest.raises(AssertionError):
        T_pen.test_grad_is_finite_difference(oracle.POT_QUADRATIC, False)


def test_wrong_root_branch_is_caught(monkeypatch):
    def bad_root(a, b, c, sens):
        a, b, c = np.broadcast_arrays(np.asarray(a, float), np.asarray(b, float), np.asarray(c, float))
        with np.errstate(all="ignore"):
            f = np.where(b > 0, (c - np.sqrt(c * c + 8 * a * b)) / (4 * b), -a / c)
        return f
    monkeypatch.setattr(oracle, "mstep_root", bad_root)
    with pytest.raises(AssertionError):
        T_pen.test_mstep_root_golden()


def test_subset_sensitivity_in_mstep_is_caught(monkeypatch):
    """Using A_t^T 1 instead of A^T 1 in the M-step breaks Appendix B."""
    def mstep_subset(self, s_hat, f_k):
        f_k = np.atleast_2d(f_k)
        return em.mstep_root(np.atleast_2d(s_hat), 0.0, -self.sens_t[0], self.sens_t[0])
    monkeypatch.setattr(em.Model, "mstep", mstep_subset)
    with pytest.raises(AssertionError):
        T_em.test_svrem_appendix_b_direction()


def test_missing_ns_factor_is_caught(monkeypatch):
    monkeypatch.setattr(em.Model, "tau_t", lambda self, f, t: np.atleast_2d(f) * self.back_t(f, t))
    with pytest.raises(AssertionError):
        T_em.test_svrem_appendix_b_direction()


def test_swapped_pixel_axes_are_caught(monkeypatch):
    orig = geometry.siddon_rays

    def swapped(geom, v):
        ray, pix, ln = orig(geom, v)
        iy, ix = pix // geom.nx, pix % geom.nx
        return ray, ix * geom.nx + iy, ln
    monkeypatch.setattr(geometry, "siddon_rays", swapped)
    with pytest.raises(AssertionError):
        T_sid.test_siddon_random_rays_brute_force()


def test_missing_half_open_rule_is_caught(monkeypatch):
    """Counting a grid-line ray in both neighbouring pixels breaks the brute force."""
    orig = geometry.siddon_rays

    def doubled(geom, v):
        ray, pix, ln = orig(geom, v)
        c, s = geometry.view_trig(v, geom.n_views, geom.arc_rad)
        if s == 0.0:  # vertical rays on grid lines: also credit the lower column
            ix = pix % geom.nx
            extra = ix > 0
            return (np.concatenate([ray, ray[extra]]), np.concatenate([pix, pix[extra] - 1]),
                    np.concatenate([ln, ln[extra]]))
        return ray, pix, ln
    monkeypatch.setattr(geometry, "siddon_rays", doubled)
    with pytest.raises(AssertionError):
        T_sid.test_vertical_view_gives_pixel_size_per_pixel()


def test_modified_curvature_sign_is_caught(monkeypatch):
    """A modified ratio with the curvature term's sign flipped (g (2 eps + ybar)
    / eps^2) breaks the derivative pin."""
    orig = em.lik_ratio

    def bad(g, yb, w, eps=0.0):
        out = orig(g, yb, w, eps)
        if eps > 0:
            g, yb, w = np.broadcast_arrays(np.asarray(g, float), np.asarray(yb, float), np.asarray(w, float))
            mod = (g > 0) & (w == 0) & (yb <= eps)
            out[mod] = g[mod] * (2.0 * eps + yb[mod]) / eps ** 2
        return out
    monkeypatch.setattr(em, "lik_ratio", bad)
    monkeypatch.setattr(oracle, "lik_ratio", bad)
    with pytest.raises(AssertionError):
        T_var.test_modified_ratio_is_one_plus_the_derivative()


def test_sagaem_refresh_before_use_is_caught(monkeypatch):
    """Refreshing the table entry before s_hat has used the old one (so the
    subset term cancels to mean(S)) breaks the refresh pin."""
    def bad_step(self, t, t_refresh=None):
        m = self.m
        if self.k == 0:
            self.init_table()
        t_refresh = t if t_refresh is None else t_refresh
        self.S[t_refresh] = m.tau_t(self.f, t_refresh)
        tau = m.tau_t(self.f, t)
        self.s_hat = (1.0 - self.alpha) * self.s_hat + self.alpha * (tau - self.S[t] + sum(self.S) / m.Ns)
        self.f = m.mstep(self.s_hat, self.f)
        self.k += 1
    monkeypatch.setattr(em.SAGAEM, "step", bad_step)
    with pytest.raises(AssertionError):
        T_var.test_sagaem_refresh_stores_the_statistic_before_the_update()


def test_sem_schedule_off_by_one_is_caught(monkeypatch):
    """a_k = 1/(decay (k + 1) + 1): the first weight is no longer 1, so the
    running mean of the harmonic schedule breaks."""
    def bad_step(self, t):
        a = self.a0 / (self.decay * (self.k + 1) + 1.0)
        self.s_hat = (1.0 - a) * self.s_hat + a * self.m.tau_t(self.f, t)
        self.f = self.m.mstep(self.s_hat, self.f)
        self.k += 1
    monkeypatch.setattr(em.SEM, "step", bad_step)
    with pytest.raises(AssertionError):
        T_sch.test_sem_harmonic_schedule_is_the_running_mean()


def test_bsrem_without_decay_is_caught(monkeypatch):
    def bad_step(self, t):
        d = em._safe_div(self.f, self.m.sens_t[t])
        self.f = np.maximum(0.0, self.f + self.alpha * d * self.m.grad_Phi_t(self.f, t))
        self.k += 1
    monkeypatch.setattr(gradient.BSREM, "step", bad_step)
    with pytest.raises(AssertionError):
        T_sch.test_bsrem_step_halves_at_k_1000()


def test_svrem_anchor_every_ns_is_caught(monkeypatch):
    """An anchor every Ns iterations whatever eta."""
    def bad_step(self, t):
        if self.k % self.m.Ns == 0:
            self.anchor()
        tau = self.m.tau_t(self.f, t)
        self.s_hat = (1.0 - self.alpha) * self.s_hat + self.alpha * (tau - self.tau_anc[t] + self.s_anc)
        self.f = self.m.mstep(self.s_hat, self.f)
        self.k += 1
    monkeypatch.setattr(em.SVREM, "step", bad_step)
    with pytest.raises(AssertionError):
        T_sch.test_svrem_takes_the_full_mstep_exactly_at_anchors(2)


def test_svrg_anchor_every_ns_is_caught(monkeypatch):
    def bad_step(self, t):
        if self.k == 0:
            self.f0 = self.f.copy()
        if self.k % self.m.Ns == 0:
            self.anchor()
        d = gradient._precond(self.m, self.f, t, self.precond, self.f0)
        direction = self.m.grad_Phi_t(self.f, t) - self.grad_anc[t] + self.g_tilde
        self.f = np.maximum(0.0, self.f + self.alpha * d * direction)
        self.k += 1
    monkeypatch.setattr(gradient.SVRG, "step", bad_step)
    with pytest.raises(AssertionError):
        T_sch.test_svrg_takes_the_full_gradient_step_exactly_at_anchors(2)


def test_contiguous_view_subsets_are_caught(monkeypatch):
    """Subsets made of contiguous arcs of views are not balanced (Sec. 2.1)."""
    def contiguous(geom, n_subsets):
        B, per = geom.n_bins, geom.n_views // n_subsets
        return [(np.arange(t * per, (t + 1) * per)[:, None] * B + np.arange(B)[None, :]).ravel()
                for t in range(n_subsets)]
    monkeypatch.setattr(em, "subset_rows", contiguous)
    monkeypatch.setattr(oracle, "subset_rows", contiguous)
    with pytest.raises(AssertionError):
        T_sch.test_interleaved_subsets_are_balanced()
