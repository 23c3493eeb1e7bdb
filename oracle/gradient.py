"""Preconditioned stochastic gradient ascent family (oracle, FP64):
SGA, BSREM, SAGA and SVRG (Sec. 4 and Sec. 5.1 of the paper).

Every update is projected onto ``f >= 0`` (``P_{>=0}``, Sec. 4).

Readings:

* ``grad Phi_t(f) = A_t^T(g_t / ybar_t) - A_t^T 1 - (beta/Ns) grad R(f)``;
* preconditioner: the experiments freeze it at the starting image,
  ``d = d(f^(0))`` (Sec. 4 remark and Sec. 5).  ``PRECOND_FULL_FROZEN``
  (default) uses one vector ``f^(0) / A^T 1`` for every subset, as Theorem 1
  and Appendix B do; ``PRECOND_SUBSET_FROZEN`` keeps the subset index of
  eq. preconditioners, ``d_t = f^(0) / A_t^T 1``; ``PRECOND_ITERATE``
  re-evaluates ``d_t(f^k) = f^k / A_t^T 1`` every iteration;
* SAGA's table starts from one full pass at ``f^(0)`` (the paper does not
  say); the direction uses the table *before* the current update, and the
  index printed as ``i`` in eq. saga_update is the current subset ``t_k``;
* SVRG stores ``grad Phi_t(f_anc)`` for every subset at each anchor;
* BSREM and SGA use ``d_t(f^k)`` (Sec. 5.1); BSREM's step is
  ``alpha_k = alpha / (0.001 k + 1)`` with ``k`` the subset-update count.
"""

from __future__ import annotations

import numpy as np

from .em import Model, _safe_div

PRECOND_SUBSET_FROZEN, PRECOND_FULL_FROZEN, PRECOND_ITERATE = 0, 1, 2


def _precond(m: Model, f, t, mode, f0):
    if mode == PRECOND_SUBSET_FROZEN:
        return _safe_div(f0, m.sens_t[t])
    if mode == PRECOND_FULL_FROZEN:
        return _safe_div(f0, m.sens)
    if mode == PRECOND_ITERATE:
        return _safe_div(f, m.sens_t[t])
    raise ValueError(mode)


class SVRG:
    """Preconditioned proximal SVRG (Sec. 4, eq. svrg_update).

    At ``k mod (eta Ns) == 0``: ``f_anc = f``, store ``grad Phi_t(f_anc)`` for all
    ``t`` and ``g_tilde = (1/Ns) grad Phi(f_anc)``.  Then
    ``f <- max(0, f + alpha d_t (.) (grad Phi_t(f) - grad Phi_t(f_anc) + g_tilde))``.
    """

    def __init__(self, model: Model, f0, alpha: float, eta: int, precond: int = PRECOND_FULL_FROZEN):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.f0 = self.f.copy()
        self.alpha, self.eta, self.precond = float(alpha), int(eta), precond
        self.k = 0
        self.n_anchors = 0  # full passes taken (bookkeeping only)

    def anchor(self):
        m = self.m
        self.n_anchors += 1
        self.f_anc = self.f.copy()
        self.grad_anc = [m.grad_Phi_t(self.f_anc, t) for t in range(m.Ns)]
        self.g_tilde = sum(self.grad_anc) / m.Ns

    def step(self, t: int):
        if self.k == 0:
            self.f0 = self.f.copy()
        if self.k % (self.eta * self.m.Ns) == 0:
            self.anchor()
        d = _precond(self.m, self.f, t, self.precond, self.f0)
        direction = self.m.grad_Phi_t(self.f, t) - self.grad_anc[t] + self.g_tilde
        self.f = np.maximum(0.0, self.f + self.alpha * d * direction)
        self.k += 1

    def run(self, order):
        for t in order:
            self.step(int(t))
        return self.f


class SAGA:
    """Preconditioned proximal SAGA (Sec. 4, eq. saga_update).

    Table ``q_t`` of the last gradient seen per subset (initialised at ``f^(0)``):
    ``q_new = grad Phi_t(f)``; ``f <- max(0, f + alpha d_t (.) (q_new - q_t + mean_t' q_t'))``;
    then ``q_t <- q_new``.
    """

    def __init__(self, model: Model, f0, alpha: float, precond: int = PRECOND_FULL_FROZEN):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.f0 = self.f.copy()
        self.alpha, self.precond = float(alpha), precond
        self.k = 0

    def init_table(self):
        m = self.m
        self.f0 = self.f.copy()
        self.q = [m.grad_Phi_t(self.f, t) for t in range(m.Ns)]

    def step(self, t: int):
        if self.k == 0:
            self.init_table()
        m = self.m
        q_new = m.grad_Phi_t(self.f, t)
        mean_q = sum(self.q) / m.Ns
        d = _precond(m, self.f, t, self.precond, self.f0)
        self.f = np.maximum(0.0, self.f + self.alpha * d * (q_new - self.q[t] + mean_q))
        self.q[t] = q_new
        self.k += 1

    def run(self, order):
        for t in order:
            self.step(int(t))
        return self.f


class SGA:
    """Preconditioned stochastic gradient ascent (Sec. 4, eq. sga; Sec. 5.1):
    ``f <- max(0, f + alpha d_t(f) (.) grad Phi_t(f))`` with ``d_t(f) = f / A_t^T 1``."""

    def __init__(self, model: Model, f0, alpha: float = 1.0):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.alpha = float(alpha)
        self.k = 0

    def step(self, t: int):
        d = _safe_div(self.f, self.m.sens_t[t])
        self.f = np.maximum(0.0, self.f + self.alpha * d * self.m.grad_Phi_t(self.f, t))
        self.k += 1

    def run(self, order):
        for t in order:
            self.step(int(t))
        return self.f


class BSREM:
    """BSREM with the subset preconditioner used in Sec. 5.1:
    ``f <- max(0, f + a_k (f / A_t^T 1) (.) grad Phi_t(f))``, ``a_k = alpha/(0.001 k + 1)``."""

    def __init__(self, model: Model, f0, alpha: float = 1.0, decay: float = 0.001):
        self.m = model
        self.f = np.atleast_2d(np.asarray(f0, dtype=np.float64)).copy()
        self.alpha, self.decay = float(alpha), float(decay)
        self.k = 0

    def step(self, t: int):
        a = self.alpha / (self.decay * self.k + 1.0)
        d = _safe_div(self.f, self.m.sens_t[t])
        self.f = np.maximum(0.0, self.f + a * d * self.m.grad_Phi_t(self.f, t))
        self.k += 1

    def run(self, order):
        for t in order:
            self.step(int(t))
        return self.f
