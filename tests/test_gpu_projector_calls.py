"""GPU: the projector calls (svr_project / svr_backproject) keep their scratch
(the tiled image, the subset-ordered sinogram) in the matrix between calls.
A call takes it only when it is idle and its last use was on the same stream
or has completed; otherwise the call allocates its own.  Calls on two streams,
interleaved without synchronisation and each with its own input, must all
give their own results (against the FP64 oracle), per subset and over all
subsets, forward and back."""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def test_interleaved_calls_on_two_streams():
    P = datagen.make_problem(80, 72, 2.0, 36, 101, 2.0, 4, 1e5, attenuation=False, seed=61)
    Ao = oracle.system_matrix(P.geom)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    rng = np.random.default_rng(8)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    rows = np.arange(P.geom.n_rays).reshape(P.geom.n_views, P.geom.n_bins)
    jobs = []
    for i in range(24):
        s = streams[i % 2]
        t = (i // 2) % (P.n_subsets + 1) - 1  # -1 (all subsets), 0, 1, ...
        x = rng.uniform(0.0, 2.0, A.N).astype(np.float32)
        y = rng.uniform(0.0, 2.0, A.M).astype(np.float32)
        with torch.cuda.stream(s):
            xd = torch.as_tensor(x, device="cuda").reshape(1, -1)
            yd = torch.as_tensor(y, device="cuda").reshape(1, -1)
            yo = torch.zeros(1, A.M, device="cuda")
            xo = torch.zeros(1, A.N, device="cuda")
            A.project(xd, t, yo, stream=s)
            A.backproject(yd, t, xo, stream=s)
        jobs.append((t, x, y, yo, xo, xd, yd))
    torch.cuda.synchronize()
    for t, x, y, yo, xo, _, _ in jobs:
        r = rows.ravel() if t < 0 else rows[t::P.n_subsets].ravel()
        ref_f = Ao[r] @ x.astype(np.float64)
        assert rel(yo.cpu().numpy().ravel()[r], ref_f) < 1e-6, t
        ref_b = Ao[r].T @ y[r].astype(np.float64)
        assert rel(xo.cpu().numpy().ravel(), ref_b) < 1e-6, t
