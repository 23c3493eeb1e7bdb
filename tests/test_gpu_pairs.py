"""GPU: forward passes that run a pair of rows per wavefront.

Passes over more rows than the matrix's pair threshold (by default twice the
wavefronts the device holds at once: the whole-matrix passes of the anchor,
the objective and the projectors at the usual sizes) sum each row with the 32
lanes of one half of a wavefront.  Here the threshold is set to 1 so that
every pass of a small problem runs in pairs, on row counts that are odd for
the whole matrix (63 views x 131 bins = 8253 rows) and for every subset (7
views x 131 bins = 917), so the last pair of each pass has one row:

* projections over all subsets and per subset match the FP64 oracle;
* SVREM and SVRG epochs (anchor passes included) match the oracle;
* results are bitwise independent of the pair run length, ragged runs too;
* the persistent epoch kernel agrees bitwise with the per-phase kernels;
* pairs and single rows agree to the oracle-parity bar (their sums differ
  in order only);
* the default threshold is 2 * 32 * compute units.
"""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402
from paper_2106_03172_amd import binding  # noqa: E402


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


@pytest.fixture(scope="module")
def odd():
    P = datagen.make_problem(96, 96, 2.0, 63, 131, 2.0, 9, 3e5, attenuation=False, seed=41)
    assert P.geom.n_rays % 2 == 1 and (P.geom.n_rays // P.n_subsets) % 2 == 1
    Ao = oracle.system_matrix(P.geom)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    return P, Ao, A


def _pairs(A, on):
    A.set_tuning(0, 0, 1 if on else 0)
    assert (A.pair_rows() == 1) == on


def test_default_threshold_is_twice_the_resident_wavefronts(odd):
    _, _, A = odd
    _pairs(A, False)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert A.pair_rows() == 2 * 32 * cus


def test_pair_projections_match_oracle(odd):
    P, Ao, A = odd
    _pairs(A, True)
    rng = np.random.default_rng(7)
    x = rng.uniform(0.0, 2.0, A.N)
    xf = x.astype(np.float32).astype(np.float64)
    ref = Ao @ xf
    assert rel(A.project(dev(x)).cpu().numpy(), ref) < 1e-6
    rows = np.arange(P.geom.n_rays).reshape(P.geom.n_views, P.geom.n_bins)
    for t in range(P.n_subsets):
        r = rows[t::P.n_subsets].ravel()
        assert len(r) % 2 == 1
        yt = A.project(dev(x), t).cpu().numpy().ravel()
        assert rel(yt[r], ref[r]) < 1e-6, t
    _pairs(A, False)


@pytest.mark.parametrize("algo", ["svrem", "svrg"])
def test_pair_epochs_match_oracle(odd, algo):
    P, Ao, A = odd
    _pairs(A, True)
    Ns = P.n_subsets
    m = oracle.Model(Ao, P.g, P.w, P.geom, Ns, beta=1e-2)
    f0 = np.ones((1, P.geom.n_pixels))
    R = pkg.Recon(A, P.g, P.w, f0.astype(np.float32),
                  pkg.params(algo, alpha=0.5, eta=1, beta=1e-2, precond="subset_frozen"))
    R.osem_epoch(list(range(Ns)))
    f_or = oracle.osem_epoch(m, f0, list(range(Ns)))
    alg = (oracle.SVREM(m, f_or, 0.5, 1) if algo == "svrem"
           else oracle.SVRG(m, f_or, 0.5, 1, precond=oracle.PRECOND_SUBSET_FROZEN))
    for e in range(3):
        order = datagen.make_order(Ns, Ns, seed=50 + e)
        R.epoch(algo, order)
        alg.run(order)
        assert rel(R.image().cpu().numpy(), alg.f) < 1e-5, e
    phi = m.objective(R.image().cpu().numpy().astype(np.float64))
    assert abs(R.objective() - phi) < 1e-6 * abs(phi)
    R.close()
    _pairs(A, False)


def _run(P, A, flags=0):
    Ns = P.n_subsets
    x = dev(np.random.default_rng(3).uniform(0.0, 2.0, A.N))
    out = {"fwd": A.project(x).cpu().numpy()}
    for algo in ("svrem", "svrg", "saga"):
        R = pkg.Recon(A, P.g, P.w, np.ones((1, A.N), np.float32),
                      pkg.params(algo, alpha=0.5, eta=2, beta=1e-2, flags=flags))
        R.osem_epoch(list(range(Ns)))
        for i, n in enumerate((Ns, 5, 2 * Ns + 1)):
            R.epoch(algo, datagen.make_order(Ns, n, seed=70 + i))
        out[algo] = R.image().cpu().numpy()
        out[algo + "_phi"] = R.objective()
        out[algo + "_state"] = R.get_state()
        R.close()
    return out


def test_pair_results_independent_of_run_length(odd):
    P, _, A = odd
    ref = None
    for fw in (1, 2, 5):
        A.set_tuning(fw, 0, 1)
        got = _run(P, A)
        if ref is None:
            ref = got
            continue
        for k in ref:
            if k.endswith("_state"):
                assert got[k] == ref[k], (k, fw)
            else:
                assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (k, fw)
    A.set_tuning(0, 0, 0)


def test_pair_persistent_matches_per_phase(odd):
    P, _, A = odd
    _pairs(A, True)
    a = _run(P, A)
    b = _run(P, A, flags=binding.FLAG_PERSISTENT_EPOCH)
    for k in a:
        if k.endswith("_state"):
            assert a[k] == b[k], k
        else:
            assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), k
    _pairs(A, False)


def test_pairs_and_single_rows_agree_to_rounding(odd):
    P, _, A = odd
    _pairs(A, True)
    a = _run(P, A)
    _pairs(A, False)
    b = _run(P, A)
    assert rel(a["fwd"], b["fwd"]) < 1e-6
    for k in ("svrem", "svrg", "saga"):
        assert rel(a[k], b[k]) < 1e-5, k
    for k in ("svrem_phi", "svrg_phi", "saga_phi"):
        assert abs(a[k] - b[k]) <= 1e-7 * abs(b[k]), k
