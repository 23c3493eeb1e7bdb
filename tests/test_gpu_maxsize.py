"""GPU parity at the largest single-image size the recon path is sized for:
384 x 384 image (2 mm), 400 views x 518 bins, 21 interleaved subsets (19 or 20
views each, so the subsets are unbalanced), 1e7 counts -- 75 M non-zeros,
pixel indices above 16 bits in the forward rows.  The FP64 oracle runs the
same epochs on the whole image in seconds, so every pixel is compared."""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.fixture(scope="module")
def maxsize():
    P = datagen.make_problem(384, 384, 2.0, 400, 518, 2.0, 21, 1e7, attenuation=False, seed=5)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    Ao = oracle.system_matrix(P.geom)
    return P, A, Ao


def test_max_size_matrix(maxsize):
    P, A, Ao = maxsize
    inf, per = A.info()
    assert inf.nnz == Ao.nnz and per.sum() == inf.nnz
    views_per_subset = np.bincount(np.arange(P.geom.n_views) % P.n_subsets)
    assert set(views_per_subset) == {19, 20}
    ptr, idx, val = A.export(0)
    B = P.geom.n_bins
    for v in (0, 50, 100, 200, 300, 399):
        ray, pix, ln = oracle.siddon_rays(P.geom, v)
        for b in range(0, B, 7):
            m = v * B + b
            sel = ray == b
            np.testing.assert_array_equal(idx[ptr[m]:ptr[m + 1]], pix[sel])
            np.testing.assert_allclose(val[ptr[m]:ptr[m + 1]], ln[sel], rtol=2.5e-7)


@pytest.mark.parametrize("algo,alpha", [("svrem", 0.7), ("saga", 2.0)])
def test_max_size_epochs_match_oracle(maxsize, algo, alpha):
    P, A, Ao = maxsize
    beta = 1e-3
    m = oracle.Model(Ao, P.g, P.w, P.geom, P.n_subsets, beta=beta)
    f0 = np.ones((1, P.geom.n_pixels))
    R = pkg.Recon(A, P.g, P.w, f0, pkg.params(algo, alpha=alpha, eta=1, beta=beta))
    cyc = list(range(P.n_subsets))
    R.osem_epoch(cyc)
    fo = oracle.osem_epoch(m, f0, cyc)
    assert rel(R.image().cpu().numpy(), fo) <= 1e-5
    alg = oracle.SVREM(m, fo, alpha, 1) if algo == "svrem" else oracle.SAGA(m, fo, alpha)
    for e in range(2):
        order = datagen.make_order(P.n_subsets, P.n_subsets, seed=90 + e)
        R.epoch(algo, order)
        alg.run(order)
        fg = R.image().cpu().numpy()
        assert np.isfinite(fg).all()
        assert rel(fg, alg.f) <= 1e-5
    phi = R.objective()
    phi_o = m.objective(fg.astype(np.float64))
    assert abs(phi - phi_o) <= 1e-6 * abs(phi_o)
