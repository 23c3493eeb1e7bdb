"""FP64 CPU oracle for the variance-reduced stochastic EM path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, step-by-step FP64
implementation (NumPy + SciPy CSR) of what the HIP library computes, written
from Kereta, Twyman, Arridge, Thielemans and Jin, "Stochastic EM methods with
variance reduction for penalised PET reconstructions" (arXiv:2106.03172).
It exists so that the GPU path can be checked against something independent:
it shares no code, header, table or constant with the HIP library, and the
library never imports it.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may use it.

Every function cites the passage of the paper it follows.  Readings of
passages that are silent, ambiguous or garbled are stated where they are
used.  Parity status: every function here is pinned by a ``-m "not gpu"``
test against closed forms, invariants, brute force or library routines;
the only result with no closed form is the exact multi-subset stochastic
trajectory, which the pins constrain only through those invariants.
"""

from .geometry import (  # noqa: F401
    view_trig, siddon_rays, system_matrix, subset_rows, SEGMENT_EPS,
)
from .penalty import (  # noqa: F401
    neighbours, penalty_value, penalty_grad, surrogate_terms, potential,
    POT_QUADRATIC, POT_HUBER, POT_LOGCOSH, POT_HYPERBOLA,
)
from .em import (  # noqa: F401
    Model, mstep_root, osem_epoch, mlem, SVREM, SEM, SAGAEM, loglik_rows, lik_ratio,
)
from .gradient import SVRG, SAGA, SGA, BSREM, PRECOND_SUBSET_FROZEN, PRECOND_FULL_FROZEN, PRECOND_ITERATE  # noqa: F401
