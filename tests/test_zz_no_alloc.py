"""The allocation-free forward projection (svr_project_noalloc) against the
allocating one (svr_project), through the C ABI: the same kernels, so the
outputs must be bitwise equal, on two calls in a row (the second with a
smaller matrix and input, reusing the library's scratch array), for the whole
matrix and for one subset, and within the projector parity bar of the FP64
oracle.  A matrix whose tiled image exceeds the scratch is rejected."""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402
from paper_2106_03172_amd import binding  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


def _both(A, x, S, subset):
    y_ref = torch.full((S, A.M), -1.0, dtype=torch.float32, device="cuda")
    y_na = torch.full((S, A.M), -1.0, dtype=torch.float32, device="cuda")
    binding.svr_project(A.h, subset, x, S, y_ref)
    binding.svr_project_noalloc(A.h, subset, x, S, y_na)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y_na.cpu().numpy()


def test_noalloc_projection_equals_svr_project_twice():
    rng = np.random.default_rng(7)
    cases = [(datagen.Geometry(128, 128, 2.0, 126, 173, 2.0), 21, 2),   # first call: larger input
             (datagen.Geometry(45, 37, 3.0, 30, 61, 2.5), 5, 1)]        # second call: smaller
    for geom, Ns, S in cases:
        print(f"noalloc: {geom.nx}x{geom.ny}, {geom.n_views}x{geom.n_bins}, Ns {Ns}, {S} slice(s)", flush=True)
        A = pkg.SystemMatrix(geom, Ns, pkg.SVR_W_F32)
        Ao = oracle.system_matrix(geom)
        xh = rng.uniform(0.0, 2.0, (S, geom.n_pixels))
        x = _dev(xh)
        for subset in (-1, Ns // 2):
            y_ref, y_na = _both(A, x, S, subset)
            np.testing.assert_array_equal(y_na, y_ref)
            rows = (np.arange(geom.n_rays) if subset < 0 else
                    oracle.subset_rows(geom, Ns)[subset])
            for sl in range(S):
                exact = Ao[rows] @ xh[sl].astype(np.float32).astype(np.float64)
                err = np.linalg.norm(y_na[sl][rows] - exact) / np.linalg.norm(exact)
                assert err <= 1e-6, (subset, sl, err)
            if subset >= 0:  # bins outside the subset are left untouched
                out = np.setdiff1d(np.arange(geom.n_rays), rows)
                np.testing.assert_array_equal(y_na[:, out], -1.0)


def test_noalloc_rejects_images_beyond_the_scratch():
    geom = datagen.Geometry(1030, 1030, 1.0, 2, 1500, 1.0)   # tiled image 1032 * 1032 > 2^20 floats
    A = pkg.SystemMatrix(geom, 1, pkg.SVR_W_F32)
    x = torch.ones(1, geom.n_pixels, dtype=torch.float32, device="cuda")
    y = torch.zeros(1, geom.n_rays, dtype=torch.float32, device="cuda")
    with pytest.raises(pkg.SvrError) as ei:
        binding.svr_project_noalloc(A.h, -1, x, 1, y)
    assert ei.value.code == binding.SVR_EINVAL
    binding.svr_project(A.h, -1, x, 1, y)   # the allocating call handles it
    torch.cuda.synchronize()
    assert float(y.sum()) > 0
