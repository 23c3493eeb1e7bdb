"""EM-family algorithms (oracle, FP64): MLEM, OSEM, SEM and SVREM.

Follows Sec. 2 (ML problem, ordered subsets, EM, stochastic EM) and Sec. 3
(penalised M-step with a separable parabolic surrogate) of the paper.

Readings of passages the paper leaves open or prints garbled:

* background ``w`` is kept in every denominator, as in the subset statistic
  of Sec. 2.3 (eq. tau_t) -- other displays omit it for brevity;
* zero denominators: a ratio ``g_m / ybar_m`` with ``ybar_m <= 0`` and any
  division by a zero sensitivity give 0 (the practical remedy of Sec. 2.3:
  set the value to 0 where the denominator vanishes);
* the log-likelihood is ``sum_m g_m log ybar_m - ybar_m`` (the ``+w_m`` printed
  in eq. log_likelihood is a constant and does not change the maximiser);
  ``0 * log(0)`` is 0;
* SVREM's running statistic starts from the anchor statistic at the first
  iteration, ``s_hat^0 = s(f^0)``, and is not reset at later anchors (the
  recursion of eq. tempsvrem only refreshes ``f_anc`` and ``s_anc``);
* the anchor statistics ``tau_t(f_anc)`` of all subsets are stored at each
  anchor, which is what the paper's epoch count (``eta Ns`` updates =
  ``eta + 1`` epochs, Sec. 5.1) implies;
* M-step root (Sec. 3, below eq. svrsurder) for ``a/f - 2 b f + c = 0``:
  ``b > 0, a > 0``: ``(c + sqrt(c^2 + 8ab)) / (4b)``, evaluated as
  ``2a / (sqrt(D) - c)`` when ``c < 0`` (same value, no cancellation);
  ``b = 0``: the linear case, ``f = -a/c`` (printed as ``-c/a``, a typo;
  ``-a/c = a / sum_m a_mn``);
  ``a = 0``: ``max(c, 0) / (2b)`` (0 when ``b = 0``);
  ``a < 0`` (possible when ``alpha > 1``): the surrogate is unbounded as
  ``f -> 0``, so ``f = 0``;
  pixels never seen (``sum_m a_mn = 0``) are 0.
* modified likelihood (Sec. 2.3, eq. modified_LL), optional (``ll_eps > 0``):
  rows with ``w_m = 0`` and ``ybar_m <= eps`` use the second-order expansion
  of ``phi_m(l) = g_m log l - l`` about ``eps``.  It is the theoretical remedy
  for the gradient methods (Theorem 1); the EM statistics ``tau_t`` keep the
  practical zero-denominator rule;
* SAGA-type online EM (Sec. 2.3, the remark after eq. tempsvrem, which the
  paper does not examine): the table ``S_t`` starts from one full pass at
  ``f^(0)`` and ``s_hat^0 = s(f^(0))``; the refreshed index ``t~_k`` is an
  explicit input (by default ``t~_k = t_k``); the refresh uses ``f^(k)``, the
  image before the update, and happens after ``s_hat`` has used the old
  entry.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import subset_rows
from .penalty import POT_QUADRATIC, penalty_grad, penalty_value, surrogate_terms


def _safe_div(x, d):
    """``x / d`` with 0 wherever ``d == 0``."""
    out = np.zeros(np.broadcast(x, d).shape)
    np.divide(x, d, out=out, where=np.broadcast_to(d != 0, out.shape))
    return out


def loglik_rows(g, yb, w, eps: float = 0.0):
    """Per-row ``phi_m(ybar_m) = g_m log ybar_m - ybar_m`` (``0 log 0 = 0``;
    ``-inf`` where ``g_m > 0`` and ``ybar_m <= 0``).  With ``eps > 0``, rows with
    ``w_m = 0`` and ``ybar_m <= eps`` take the modified value of eq. modified_LL:
    ``phi(eps) + phi'(eps) (ybar - eps) + phi''(eps)/2 (ybar - eps)^2`` with
    ``phi'(l) = g/l - 1`` and ``phi''(l) = -g/l^2``."""
    g, yb, w = np.broadcast_arrays(np.asarray(g, float), np.asarray(yb, float), np.asarray(w, float))
    out = -yb.copy()
    pos = g > 0
    ok = pos & (yb > 0)
    out[ok] = g[ok] * np.log(yb[ok]) - yb[ok]
    out[pos & (yb <= 0)] = -np.inf
    if eps > 0:
        mod = pos & (w == 0) & (yb <= eps)
        gm, d = g[mod], yb[mod] - eps
        out[mod] = (gm * np.log(eps) - eps) + (gm / eps - 1.0) * d - 0.5 * (gm / eps ** 2) * d * d
    return out


def lik_ratio(g, yb, w, eps: float = 0.0):
    """``phi_m'(ybar_m) + 1``, the ratio whose back-projection minus ``A^T 1`` is
    the likelihood gradient: ``g/ybar`` (0 where ``g = 0`` or ``ybar <= 0``);
    with ``eps > 0``, rows with ``w = 0`` and ``ybar <= eps`` take the
    modified derivative ``phi''(eps) (ybar - eps) + phi'(eps) + 1
    = g (2 eps - ybar) / eps^2`` (eq. modified_LL)."""
    g, yb, w = np.broadcast_arrays(np.asarray(g, float), np.asarray(yb, float), np.asarray(w, float))
    out = np.zeros(yb.shape)
    np.divide(g, yb, out=out, where=(yb > 0) & (g != 0))
    if eps > 0:
        mod = (g > 0) & (w == 0) & (yb <= eps)
        out[mod] = g[mod] * (2.0 * eps - yb[mod]) / eps ** 2
    return out


class Model:
    """The penalised Poisson problem of Sec. 2.1 and Sec. 3 with its partition.

    ``A``: (M x N) CSR, rows in natural order.  ``g``, ``w``: (S, M).
    Images are (S, N): ``S`` slices share ``A`` and are coupled only through
    an optional axial penalty.
    """

    def __init__(self, A: sp.csr_matrix, g, w, geom, n_subsets: int, beta: float = 0.0,
                 potential: int = POT_QUADRATIC, delta: float = 1.0, axial: bool = False,
                 ll_eps: float = 0.0):
        self.A = A.tocsr()
        self.geom = geom
        self.ny, self.nx = geom.ny, geom.nx
        self.Ns = int(n_subsets)
        self.g = np.atleast_2d(np.asarray(g, dtype=np.float64))
        self.w = np.atleast_2d(np.asarray(w, dtype=np.float64))
        self.beta = float(beta)
        self.potential = potential
        self.delta = float(delta)
        self.axial = axial
        self.ll_eps = float(ll_eps)  # > 0: modified likelihood (eq. modified_LL) in L and grad L
        self.rows = subset_rows(geom, n_subsets)
        self.A_t = [self.A[r] for r in self.rows]
        self.AT_t = [a.T.tocsr() for a in self.A_t]
        self.AT = self.A.T.tocsr()
        self.g_t = [self.g[:, r] for r in self.rows]
        self.w_t = [self.w[:, r] for r in self.rows]
        M = self.A.shape[0]
        # sensitivities A_t^T 1 and A^T 1 (used by the M-step, eq. Mstep)
        self.sens_t = np.stack([self.AT_t[t] @ np.ones(len(self.rows[t]))
                                for t in range(self.Ns)])
        self.sens = self.AT @ np.ones(M)

    # -- projections -------------------------------------------------------
    def fwd_t(self, f, t):
        """``A_t f + w_t`` per slice (the mean data of subset t, eq. voxel_td)."""
        f = np.atleast_2d(f)
        return (self.A_t[t] @ f.T).T + self.w_t[t]

    def ratio_t(self, f, t):
        """``g_t / (A_t f + w_t)`` with the zero-denominator rule."""
        yb = self.fwd_t(f, t)
        gt = self.g_t[t]
        out = np.zeros_like(yb)
        np.divide(gt, yb, out=out, where=(yb > 0) & (gt != 0))
        return out

    def back_t(self, f, t):
        """``b_t(f) = A_t^T (g_t / (A_t f + w_t))`` (the E-step sum of eq. EMsurrogate)."""
        r = self.ratio_t(f, t)
        return (self.AT_t[t] @ r.T).T

    def back_full(self, f):
        f = np.atleast_2d(f)
        yb = (self.A @ f.T).T + self.w
        r = np.zeros_like(yb)
        np.divide(self.g, yb, out=r, where=(yb > 0) & (self.g != 0))
        return (self.AT @ r.T).T

    def tau_t(self, f, t):
        """Subset statistic ``Ns f (.) A_t^T (g_t / (A_t f + w_t))`` (Sec. 2.3, eq. tau_t)."""
        return self.Ns * np.atleast_2d(f) * self.back_t(f, t)

    def s_full(self, f):
        """Full statistic ``s(f) = (1/Ns) sum_t tau_t(f)`` (Sec. 2.3)."""
        return sum(self.tau_t(f, t) for t in range(self.Ns)) / self.Ns

    # -- objective and gradients ------------------------------------------
    def loglik(self, f) -> float:
        """``L(f) = sum_m g_m log ybar_m - ybar_m`` (eq. log_likelihood, up to a constant);
        with ``ll_eps > 0`` the modified likelihood of eq. modified_LL."""
        f = np.atleast_2d(f)
        yb = (self.A @ f.T).T + self.w
        if self.ll_eps > 0:
            return float(np.sum(loglik_rows(self.g, yb, self.w, self.ll_eps)))
        if np.any((yb <= 0) & (self.g > 0)):
            return -np.inf
        lg = np.zeros_like(yb)
        np.log(yb, out=lg, where=self.g > 0)
        return float(np.sum(self.g * lg) - np.sum(yb))

    def penalty(self, f) -> float:
        return penalty_value(f, self.ny, self.nx, self.potential, self.delta, self.axial)

    def grad_R(self, f):
        return penalty_grad(f, self.ny, self.nx, self.potential, self.delta, self.axial)

    def objective(self, f) -> float:
        """``Phi(f) = L(f) - beta R(f)`` (Sec. 3, eq. PET-MAP)."""
        return self.loglik(f) - self.beta * self.penalty(f)

    def grad_L_t(self, f, t):
        """``grad L_t(f) = A_t^T (g_t / ybar_t - 1)`` (Sec. 4, eq. osem_additive), or
        ``A_t^T phi_hat'(ybar_t)`` with the modified likelihood."""
        if self.ll_eps > 0:
            r = lik_ratio(self.g_t[t], self.fwd_t(f, t), self.w_t[t], self.ll_eps)
            return (self.AT_t[t] @ r.T).T - self.sens_t[t]
        return self.back_t(f, t) - self.sens_t[t]

    def grad_Phi_t(self, f, t):
        """``grad Phi_t = grad L_t - (beta/Ns) grad R`` (Sec. 4, definition of Phi_t)."""
        return self.grad_L_t(f, t) - (self.beta / self.Ns) * self.grad_R(f)

    def grad_Phi(self, f):
        if self.ll_eps > 0:
            f = np.atleast_2d(f)
            r = lik_ratio(self.g, (self.A @ f.T).T + self.w, self.w, self.ll_eps)
            return (self.AT @ r.T).T - self.sens - self.beta * self.grad_R(f)
        return self.back_full(f) - self.sens - self.beta * self.grad_R(f)

    # -- M-step ------------------------------------------------------------
    def mstep(self, s_hat, f_k):
        """Maximiser of ``zeta(f)^T s_hat - U(f) - beta R_hat(f; f_k)`` over ``f >= 0``
        (Sec. 3, eq. vrsemreg with the parabolic surrogate, eq. svrsurder)."""
        f_k = np.atleast_2d(f_k)
        D, E = surrogate_terms(f_k, self.ny, self.nx, self.potential, self.delta, self.axial)
        a = np.atleast_2d(s_hat)
        b = self.beta * D
        c = self.beta * f_k * D + self.beta * E - self.sens
        return mstep_root(a, b, c, np.broadcast_to(self.sens, a.shape))


def mstep_root(a, b, c, sens):
    """Non-negative root of ``a/f - 2 b f + c = 0`` (Sec. 3), with the readings
    listed in the module docstring."""
    a, b, c = np.broadcast_arrays(np.asarray(a, float), np.asarray(b, float),
                                  np.asarray(c, float))
    sens = np.broadcast_to(sens, a.shape)
    f = np.zeros(a.shape)
    pos_b = b > 0
    # b > 0, a > 0: the quadratic 2 b f^2 - c f - a = 0 has one positive root
    m = pos_b & (a > 0)
    D = c[m] * c[m] + 8.0 * a[m] * b[m]
    sq = np.sqrt(D)
    cm = c[m]
    f[m] = np.where(cm >= 0, (cm + sq) / (4.0 * b[m]), 2.0 * a[m] / (sq - cm))
    # b > 0, a == 0
    m0 = pos_b & (a == 0)
    f[m0] = np.maximum(c[m0], 0.0) / (2.0 * b[m0])
    # b == 0: linear case, f = -a/c
    ml = (~pos_b) & (a > 0) & (c < 0)
    f[ml] = -a[ml] / c[ml]
    f[sens == 0] = 0.0
    return f


# ---------------------------------------------------------------------------
# MLEM / OSEM
# ---------------------------------------------------------------------------

def osem_step(model: Model, f, t):
    """One OSEM update on subset ``t``: ``f (.) A_t^T(g_t/ybar_t) / A_t^T 1``
    (Sec. 2.2, eq. Mstep)."""
    f = np.atleast_2d(f)
    return _safe_div(f * model.back_t(f, t), model.sens_t[t])


def osem_epoch(model: Model, f, order):
    """OSEM over the subset sequence ``order``."""
    f = np.atleast_2d(np.asarray(f, dtype=np.float64)).copy()
    for t in order:
        f = osem_step(model, f, int(t))
    return f


def mlem(model: Model, f, n_iter: int, callback=None):
    """MLEM with the full data (Sec. 2.2, the ``Ns = 1`` update)."""
    f = np.atleast_2d(np.asarray(f, dtype=np.float64)).copy()
    for _ in range(n_iter):
        f = _safe_div(f * model.back_full(f), model.sens)
        if callback is not None:
            callback(f)
    return f


# ---------------------------------------------------------------------------
# SEM and SVREM (Sec. 2.3 and Sec. 3)
# ---------------------------------------------------------------------------

class SVREM:
    """Stochastic variance reduced EM (Sec. 2.3, eq. tempsvrem) with the
    penalised M-step of Sec. 3.

    Iteration ``k`` on subset ``t``:
      * if ``k mod (eta Ns) == 0``: ``f_anc = f``, ``tau_anc[t'] = tau_t'(f_anc)``
        for all ``t'``, ``s_anc = mean_t' tau_anc[t']`` (and ``s_hat = s_anc``
        at ``k = 0``);
      * ``s_hat <- (1 - alpha) s_hat + alpha (tau_t(f) - tau_anc[t] + s_anc)``;
      * ``f <- M-step(s_hat)`` about the current ``f``.
    """

    def __init__(self, model: Model, f0, alpha: float, eta: int, reset_at_anchor: bool = False):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.alpha = float(alpha)
        self.eta = int(eta)
        self.reset = reset_at_anchor
        self.k = 0
        self.s_hat = None
        self.n_negative_a = 0
        self.n_anchors = 0  # full passes taken (bookkeeping only)

    def anchor(self):
        m = self.m
        self.n_anchors += 1
        self.f_anc = self.f.copy()
        self.tau_anc = [m.tau_t(self.f_anc, t) for t in range(m.Ns)]
        self.s_anc = sum(self.tau_anc) / m.Ns
        if self.k == 0 or self.reset:
            self.s_hat = self.s_anc.copy()

    def step(self, t: int):
        if self.k % (self.eta * self.m.Ns) == 0:
            self.anchor()
        tau = self.m.tau_t(self.f, t)
        self.s_hat = (1.0 - self.alpha) * self.s_hat + self.alpha * (tau - self.tau_anc[t] + self.s_anc)
        self.n_negative_a += int(np.count_nonzero(self.s_hat < 0))
        self.f = self.m.mstep(self.s_hat, self.f)
        self.k += 1

    def run(self, order):
        for t in order:
            self.step(int(t))
        return self.f


class SEM:
    """Stochastic EM (Sec. 2.3, eq. tempsem): ``s_hat <- (1-a_k) s_hat + a_k tau_t(f)``
    with the decaying schedule ``a_k = 1/(0.001 k + 1)`` of Sec. 5.1, then the
    M-step.  ``a_0 = 1`` makes the starting value of ``s_hat`` irrelevant."""

    def __init__(self, model: Model, f0, a0: float = 1.0, decay: float = 0.001):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.s_hat = np.zeros_like(self.f)
        self.a0, self.decay = float(a0), float(decay)
        self.k = 0

    def step(self, t: int):
        a = self.a0 / (self.decay * self.k + 1.0)
        self.s_hat = (1.0 - a) * self.s_hat + a * self.m.tau_t(self.f, t)
        self.f = self.m.mstep(self.s_hat, self.f)
        self.k += 1

    def run(self, order):
        for t in order:
            self.step(int(t))
        return self.f


class SAGAEM:
    """SAGA-type online EM (Sec. 2.3, the remark after eq. tempsvrem) with the
    penalised M-step of Sec. 3.

    A table ``S_t`` of subset statistics, filled with ``tau_t(f^(0))`` for every
    ``t`` before the first iteration, and ``s_hat^0 = mean_t S_t = s(f^(0))``.
    Iteration ``k`` on subset ``t`` with refreshed index ``t~``:
      * ``s_hat <- (1 - alpha) s_hat + alpha (tau_t(f) - S_t + mean_t' S_t')``;
      * ``S_t~ <- tau_t~(f)`` (``f`` the image before this update);
      * ``f <- M-step(s_hat)`` about the current ``f``.
    """

    def __init__(self, model: Model, f0, alpha: float):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.alpha = float(alpha)
        self.k = 0
        self.s_hat = None

    def init_table(self):
        m = self.m
        self.S = [m.tau_t(self.f, t) for t in range(m.Ns)]
        self.s_hat = sum(self.S) / m.Ns

    def step(self, t: int, t_refresh: int = None):
        m = self.m
        if self.k == 0:
            self.init_table()
        if t_refresh is None:
            t_refresh = t
        tau = m.tau_t(self.f, t)
        mean_S = sum(self.S) / m.Ns
        self.s_hat = (1.0 - self.alpha) * self.s_hat + self.alpha * (tau - self.S[t] + mean_S)
        self.S[t_refresh] = tau if t_refresh == t else m.tau_t(self.f, t_refresh)
        self.f = m.mstep(self.s_hat, self.f)
        self.k += 1

    def run(self, order, refresh=None):
        for i, t in enumerate(order):
            self.step(int(t), None if refresh is None else int(refresh[i]))
        return self.f
