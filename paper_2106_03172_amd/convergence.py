"""Convergence harness (Sec. 5 of the paper): runs reconstruction methods
through the library from a common start and records their convergence
curves.

Every method starts from one OSEM epoch in cyclic subset order (Sec. 5.1:
all algorithms are initialised with one epoch of OSEM) and then runs outer
loops of subset updates with subsets drawn uniformly at random.  After each
outer loop the harness records

* the epochs spent, in the paper's accounting (Sec. 5.1): an epoch is one
  pass over the data, so ``eta*Ns`` SVRG or SVREM updates count as ``eta + 1``
  epochs (the anchor pass is one); ``Ns`` updates of the other methods count
  as one epoch; the table fill of SAGA and SAGA-EM at the first iteration is
  a full pass and counts as one more epoch; a SAGA-EM refresh of a subset
  other than the updated one costs one more subset projection (``1/Ns``);
* the objective ``Phi(f)`` (``svr_objective``, FP64);
* given a reference image ``f*``, the relative error
  ``Delta(f) = ||f - f*|| / ||f*||`` (Sec. 5.1);
* the wall time of the loop's epoch calls (enqueue to completion).

``reference_image`` computes ``f*`` as a long run of a chosen method that
stops when the image no longer moves.  The paper uses L-BFGS-B for ``f*``;
the tests pin this reference to an L-BFGS-B maximiser on a small problem.

Nothing here computes any step of the method: every update runs in the
library's kernels; the harness only draws subset orders, calls epochs and
reduces images to the recorded numbers.
"""

from __future__ import annotations

import dataclasses
import json
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import binding

@dataclasses.dataclass
class Method:
    """One curve: a name, the algorithm and its ``svr_params`` keywords."""
    name: str
    algo: str
    kw: Dict = dataclasses.field(default_factory=dict)
    refresh: str = "same"  # SAGA-EM: "same" (t~ = t) or "independent" (t~ drawn separately)

    def params(self):
        return binding.params(self.algo, **self.kw)


@dataclasses.dataclass
class Curve:
    name: str
    algo: str
    kw: Dict
    epochs: List[float] = dataclasses.field(default_factory=list)
    phi: List[float] = dataclasses.field(default_factory=list)
    delta: List[Optional[float]] = dataclasses.field(default_factory=list)
    seconds: List[float] = dataclasses.field(default_factory=list)
    status: str = "ok"

    def epochs_to(self, delta: float) -> Optional[float]:
        """First recorded epoch count with Delta <= delta (None if never)."""
        for e, d in zip(self.epochs, self.delta):
            if d is not None and d <= delta:
                return e
        return None

    def as_dict(self):
        return dataclasses.asdict(self)


def outer_loop(algo: str, n_subsets: int, eta: int) -> tuple:
    """(subset updates, epochs) of one outer loop in the paper's accounting."""
    if algo in ("svrem", "svrg"):
        return eta * n_subsets, float(eta + 1)
    return n_subsets, 1.0


def _delta(f, f_ref, ref_norm):
    import torch
    return float(torch.linalg.vector_norm((f - f_ref).double()) / ref_norm)


def run_method(A, g, w, method: Method, epochs: float, f_ref=None, seed: int = 0, stream=None) -> Curve:
    """Runs ``method`` for at least ``epochs`` epochs after the OSEM start."""
    import torch
    Ns = A.n_subsets
    N = A.N
    rng = np.random.Generator(np.random.PCG64(seed))
    prm = method.params()
    R = binding.Recon(A, g, w, np.ones((1, N), np.float32), prm, stream)
    curve = Curve(method.name, method.algo, dict(method.kw))
    ref_norm = None
    if f_ref is not None:
        f_ref = torch.as_tensor(np.asarray(f_ref, np.float32).reshape(1, N), device="cuda")
        ref_norm = float(torch.linalg.vector_norm(f_ref.double()))
    try:
        R.osem_epoch(list(range(Ns)), stream)
        spent = 0.0

        def record(sec):
            curve.epochs.append(spent)
            curve.phi.append(R.objective(stream))
            curve.delta.append(_delta(R.image(stream), f_ref, ref_norm) if f_ref is not None else None)
            curve.seconds.append(sec)

        record(0.0)
        eta = int(method.kw.get("eta", 1))
        first = True
        while spent < epochs - 1e-9:
            n_upd, cost = outer_loop(method.algo, Ns, eta)
            order = rng.integers(0, Ns, n_upd).astype(np.int32)
            refresh = None
            if method.algo == "sagaem" and method.refresh == "independent":
                refresh = rng.integers(0, Ns, n_upd).astype(np.int32)
                cost += float(np.count_nonzero(refresh != order)) / Ns
            if first and method.algo in ("saga", "sagaem"):
                cost += 1.0  # the table fill at f^(0)
            first = False
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if method.algo == "sagaem":
                R.sagaem_epoch(order, refresh, stream)
            else:
                R.epoch(method.algo, order, stream)
            torch.cuda.synchronize()
            spent += cost
            record(time.perf_counter() - t0)
    except binding.SvrError as e:  # e.g. a diverging run whose objective is no longer finite
        curve.status = f"stopped: {e}"
    finally:
        R.close()
    return curve


def reference_image(A, g, w, method: Method, max_epochs: float = 4000, tol: float = 1e-7, seed: int = 12345,
                    stream=None):
    """``f*``: ``method`` from the OSEM start until the image moves by less
    than ``tol`` (relative) over three outer loops in a row, or for
    ``max_epochs``.  Returns ``(f*, epochs used, last relative change)``."""
    import torch
    Ns, N = A.n_subsets, A.N
    rng = np.random.Generator(np.random.PCG64(seed))
    R = binding.Recon(A, g, w, np.ones((1, N), np.float32), method.params(), stream)
    try:
        R.osem_epoch(list(range(Ns)), stream)
        prev = R.image(stream).clone()
        spent, change, quiet = 0.0, float("inf"), 0
        eta = int(method.kw.get("eta", 1))
        while spent < max_epochs:
            n_upd, cost = outer_loop(method.algo, Ns, eta)
            R.epoch(method.algo, rng.integers(0, Ns, n_upd).astype(np.int32), stream)
            spent += cost
            cur = R.image(stream)
            change = float(torch.linalg.vector_norm((cur - prev).double()) / torch.linalg.vector_norm(cur.double()))
            prev = cur.clone()
            quiet = quiet + 1 if change < tol else 0
            if quiet >= 3:
                break
        return prev.cpu().numpy().reshape(N), spent, change
    finally:
        R.close()


def compare(A, g, w, methods: Sequence[Method], epochs: float, f_ref=None, seed: int = 0, stream=None):
    """Curves of several methods on the same data and start (each method draws
    its own subset orders from ``seed``)."""
    return [run_method(A, g, w, m, epochs, f_ref, seed + i, stream) for i, m in enumerate(methods)]


def paper_methods(beta: float, penalty: str, delta: float, svrem_alpha: float = 0.7, svrem_eta: int = 1,
                  grad_alpha: float = 2.0, svrg_eta: int = 2) -> List[Method]:
    """The comparison of Sec. 5.1: SVREM (alpha 0.7, eta 1), SAGA and SVRG
    (alpha 2, SVRG eta 2, preconditioner f^(0) / A^T 1 frozen at the start),
    and the baselines OSEM, SGA, BSREM and SEM (a_k = 1 / (0.001 k + 1))."""
    pen = dict(beta=beta, penalty=penalty, delta=delta)
    return [
        Method("SVREM", "svrem", dict(alpha=svrem_alpha, eta=svrem_eta, **pen)),
        Method("SVRG", "svrg", dict(alpha=grad_alpha, eta=svrg_eta, precond="full_frozen", **pen)),
        Method("SAGA", "saga", dict(alpha=grad_alpha, precond="full_frozen", **pen)),
        Method("SAGA-EM", "sagaem", dict(alpha=svrem_alpha, **pen)),
        Method("OSEM", "osem", dict()),
        Method("SGA", "sga", dict(alpha=1.0, **pen)),
        Method("BSREM", "bsrem", dict(alpha=1.0, decay=0.001, **pen)),
        Method("SEM", "sem", dict(alpha=1.0, decay=0.001, **pen)),
    ]


def to_json(curves: Sequence[Curve]) -> str:
    return json.dumps([c.as_dict() for c in curves])
