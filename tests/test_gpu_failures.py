"""Failure handling, forced from the host: allocation failures surface as
SVR_ENOMEM without leaks or crashes, and a bad request in the server fails
alone while the others finish bitwise as they would have."""

import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402
from paper_2106_03172_amd import binding  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("after", [0, 3, 9])
def test_allocation_failure_is_reported(after):
    """SVR_FAULT_ALLOC_AFTER=n makes the (n+1)-th device allocation fail; the
    build (or the recon) then returns SVR_ENOMEM and the process carries on."""
    code = textwrap.dedent(f"""
        import sys; sys.path.insert(0, {ROOT!r})
        import numpy as np, torch, datagen, paper_2106_03172_amd as pkg
        P = datagen.make_problem(32, 32, 2.0, 20, 45, 2.0, 4, 1e4, seed=1)
        try:
            A = pkg.SystemMatrix(P.geom, 4)
            pkg.Recon(A, P.g, P.w, np.ones((1, 1024)), pkg.params("svrem"))
            print("NOFAIL")
        except pkg.SvrError as e:
            print("CODE", e.code)
        x = torch.ones(4, device="cuda"); print("ALIVE", float(x.sum()))
    """)
    env = dict(os.environ, SVR_FAULT_ALLOC_AFTER=str(after))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=180)
    assert "ALIVE 4.0" in r.stdout, r.stdout + r.stderr
    assert f"CODE {binding.SVR_ENOMEM}" in r.stdout, r.stdout + r.stderr


def test_bad_request_fails_alone():
    specs = [(40, 30, 55, 5, 2e4, 51), (48, 36, 65, 6, 3e4, 52), (32, 24, 45, 4, 1e4, 53)]
    probs = [datagen.make_problem(n, n, 2.0, V, B, 2.0, Ns, c, seed=s) for n, V, B, Ns, c, s in specs]
    bad = probs[1].g.copy()
    bad[0, 7] = np.nan
    prm = pkg.params("svrem", alpha=0.7, eta=1, beta=1e-3)

    def serve(items):
        S = pkg.Server(1 << 31, max_slots=4, n_streams=3)
        tk = [S.submit(P.geom, P.n_subsets, g, P.w, prm, 3, 900 + i) for i, (P, g) in enumerate(items)]
        S.step(0)
        out = [S.poll(t) for t in tk]
        S.close()
        return out

    mixed = serve([(probs[0], probs[0].g), (probs[1], bad), (probs[2], probs[2].g)])
    assert mixed[1]["status"] == binding.SVR_EINVAL
    assert mixed[0]["status"] == 0 and mixed[2]["status"] == 0
    clean = serve([(probs[0], probs[0].g), (probs[1], probs[1].g), (probs[2], probs[2].g)])
    np.testing.assert_array_equal(mixed[0]["f"], clean[0]["f"])
    np.testing.assert_array_equal(mixed[2]["f"], clean[2]["f"])
