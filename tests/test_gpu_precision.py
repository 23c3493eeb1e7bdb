"""Reduced-precision matrix weights (FP16, BF16) with FP64 accumulation:
stored weights within the rounding bound of the FP64 lengths, and the
SVREM iterate's error against the FP64 oracle (which uses exact lengths)."""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.fixture(scope="module")
def prob():
    P = datagen.make_problem(128, 128, 2.0, 126, 173, 2.0, 21, 1e6, seed=41)
    return P, oracle.system_matrix(P.geom)


@pytest.mark.parametrize("wtype,bound", [(pkg.SVR_W_F16, 2.0 ** -11), (pkg.SVR_W_BF16, 2.0 ** -8)])
def test_stored_weights_rounding(prob, wtype, bound):
    """Round to nearest: relative error <= half an ulp (2^-11 for FP16's 10-bit
    mantissa, 2^-8 for BF16's 7 bits, after the FP32 step) for normal values;
    FP16 weights below its normal range (6.1e-5 mm) keep an absolute error
    below half its subnormal spacing."""
    P, Ao = prob
    A = pkg.SystemMatrix(P.geom, P.n_subsets, wtype)
    ptr, idx, val = A.export(0)
    np.testing.assert_array_equal(idx, Ao.indices)
    a = Ao.data
    err = np.abs(val.astype(np.float64) - a)
    normal = a >= 6.1e-5
    assert np.all(err[normal] <= bound * a[normal] * (1 + 1e-6))
    if wtype == pkg.SVR_W_F16:
        assert np.all(err[~normal] <= 2.0 ** -25)


@pytest.mark.parametrize("wtype,tol", [(pkg.SVR_W_F32, 1e-5), (pkg.SVR_W_F16, 1e-3), (pkg.SVR_W_BF16, 1e-2)])
def test_svrem_error_vs_fp64_oracle(prob, wtype, tol):
    """Final-iterate and objective error of 5 SVREM epochs per weight type.
    The bound for 16-bit weights is the weight rounding itself: a relative
    perturbation eps of A moves the iterate by O(eps)."""
    P, Ao = prob
    beta = 1e-2
    A = pkg.SystemMatrix(P.geom, P.n_subsets, wtype)
    m = oracle.Model(Ao, P.g, P.w, P.geom, P.n_subsets, beta=beta)
    f0 = np.ones((1, P.geom.n_pixels))
    R = pkg.Recon(A, P.g, P.w, f0, pkg.params("svrem", alpha=0.7, eta=1, beta=beta))
    cyc = list(range(P.n_subsets))
    R.osem_epoch(cyc)
    alg = oracle.SVREM(m, oracle.osem_epoch(m, f0, cyc), 0.7, 1)
    for e in range(5):
        o = datagen.make_order(P.n_subsets, P.n_subsets, seed=500 + e)
        R.svrem_epoch(o)
        alg.run(o)
    fg = R.image().cpu().numpy()
    err = rel(fg, alg.f)
    phi_err = abs(R.objective() - m.objective(alg.f)) / abs(m.objective(alg.f))
    print(f"wtype {wtype}: iterate rel L2 {err:.3e}, objective rel {phi_err:.3e}")
    assert err <= tol
    assert phi_err <= tol * 1e-2
