"""GPU: the run lengths of the whole-matrix passes (svr_matrix_set_tuning /
svr_matrix_tune) never change a result.

A run length only decides which wavefront (or lane group) sums a row (a
forward wavefront sums pairs of rows, 32 lanes each); the row's own
arithmetic is the same code at every setting, so projections over
all subsets, back-projections, the objective and whole epochs of the
variance-reduced methods must be bitwise identical under every tuning,
including ragged last runs (rows not a multiple of the run length) and runs
longer than the pass.  The results are also checked once against the FP64
oracle, so a tuning that is consistently wrong would fail too.
"""

import numpy as np
import pytest

import datagen
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2106_03172_amd as pkg  # noqa: E402

# (row pairs per wavefront, rows per lane group, per-subset forward batch,
# per-subset update batch)
TUNINGS = [(1, 1, 4, 3), (2, 3, 6, 4), (7, 5, 8, 6), (13, 16, 0, 8), (31, 1024, 4, 5), (0, 0, 0, 0)]


def rel(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float32), device="cuda")


def run_all(P, A, x, y, f0, order):
    """Every whole-matrix result of A at its current tuning, on the host."""
    out = {"fwd": A.project(x).cpu().numpy(), "bp": A.backproject(y).cpu().numpy()}
    for algo, kw in (("svrem", dict(alpha=0.7, eta=1, beta=1e-2)),
                     ("svrg", dict(alpha=0.5, eta=1, beta=1e-2)),
                     ("saga", dict(alpha=0.5, beta=1e-2))):
        R = pkg.Recon(A, P.g, P.w, f0, pkg.params(algo, **kw))
        R.osem_epoch(list(range(P.n_subsets)))
        R.epoch(algo, order)
        out[algo] = R.image().cpu().numpy()
        out[algo + "_phi"] = R.objective()
        R.close()
    return out


@pytest.mark.parametrize("shape", ["medium", "headline"])
def test_results_are_bitwise_independent_of_tuning(shape):
    if shape == "medium":
        P = datagen.make_problem(96, 96, 2.0, 70, 131, 2.0, 7, 3e5, attenuation=False, seed=21)
    else:
        P = datagen.make_problem(**datagen.CONFIG_HEADLINE)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    rng = np.random.default_rng(5)
    x = dev(rng.uniform(0.0, 2.0, A.N))
    y = dev(rng.uniform(0.0, 2.0, A.M))
    f0 = np.ones(A.N, np.float32)
    order = datagen.make_order(P.n_subsets, 2 * P.n_subsets, seed=9)
    ref = None
    for fw, bp, fu, bu in TUNINGS:
        A.set_tuning(fw, bp, subset_fwd_batch=fu, subset_bp_batch=bu)
        eff = A.tuning()
        assert eff[0] == (fw or eff[0]) and eff[1] == (bp or eff[1])
        assert A.batch_widths() == (fu or 8, bu or 5)
        print("tuning", (fw, bp, fu, bu), "effective", eff, flush=True)
        got = run_all(P, A, x, y, f0, order)
        if ref is None:
            ref = got
            continue
        for k in ref:
            assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (k, fw, bp)
    tuned = A.tune()
    print("tuned", tuned, A.batch_widths(), flush=True)
    assert A.batch_widths()[0] in (4, 6, 8) and A.batch_widths()[1] in (3, 4, 5, 6, 8)
    assert 1 <= tuned[0] <= 31 and 1 <= tuned[1] <= 1024 and tuned[2] > 0 and tuned[3] > 0
    assert A.tuning() == tuned[:2]
    got = run_all(P, A, x, y, f0, order)
    for k in ref:
        assert np.array_equal(np.asarray(got[k]), np.asarray(ref[k])), (k, "tuned")

    if shape == "medium":  # the shared results against the oracle
        Ao = oracle.system_matrix(P.geom)
        xf = x.cpu().numpy().astype(np.float64)
        yf = y.cpu().numpy().astype(np.float64)
        assert rel(ref["fwd"].ravel(), Ao @ xf) < 1e-6
        assert rel(ref["bp"].ravel(), Ao.T @ yf) < 1e-6


def test_tuning_rejects_out_of_range():
    P = datagen.make_problem(**datagen.CONFIG_SMALL)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32, mu=P.mu)
    for bad in ((-1, 0), (32, 0), (0, -1), (0, 1025)):
        with pytest.raises(pkg.SvrError):
            A.set_tuning(*bad)
    for fu, bu in ((5, 0), (2, 0), (0, 7), (0, 2)):
        with pytest.raises(pkg.SvrError):
            A.set_tuning(0, 0, subset_fwd_batch=fu, subset_bp_batch=bu)
    A.set_tuning(31, 1024)
    assert A.tuning() == (31, 1024)
    A.set_tuning(0, 0)
    fw, bp = A.tuning()
    assert fw >= 1 and bp >= 1


@pytest.mark.parametrize("shape", ["medium", "headline", "ragged"])
def test_forward_row_order_is_bitwise_neutral(shape):
    """Per-subset forward passes give each XCD a band of bins of every view
    (default) or take the rows in order: a row is summed by one wavefront with
    the same code either way, so every result is bitwise the same (ragged:
    bins not a multiple of 8, unequal subsets)."""
    if shape == "medium":
        P = datagen.make_problem(96, 96, 2.0, 70, 131, 2.0, 7, 3e5, attenuation=False, seed=21)
    elif shape == "headline":
        P = datagen.make_problem(**datagen.CONFIG_HEADLINE)
    else:
        P = datagen.make_problem(37, 29, 3.0, 19, 43, 2.5, 4, 5e4, attenuation=False, seed=22)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    rng = np.random.default_rng(6)
    x = dev(rng.uniform(0.0, 2.0, A.N))
    y = dev(rng.uniform(0.0, 2.0, A.M))
    f0 = np.ones(A.N, np.float32)
    order = datagen.make_order(P.n_subsets, 2 * P.n_subsets, seed=10)
    out = []
    for natural in (0, 1):
        A.set_tuning(0, 0, fwd_natural_order=natural)
        got = run_all(P, A, x, y, f0, order)
        got["sub"] = [A.project(x, t).cpu().numpy() for t in range(P.n_subsets)]
        out.append(got)
    for k in out[0]:
        np.testing.assert_array_equal(np.asarray(out[0][k]), np.asarray(out[1][k]), err_msg=k)


def test_tuning_cache(tmp_path, monkeypatch):
    """SVR_TUNE_CACHE: the first tune of a geometry times the candidates and
    appends one line; a second matrix of the same geometry takes the recorded
    run lengths without timing (its own setting overridden, no new line); a
    different geometry appends its own line; lines that do not parse are
    ignored."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("SVR_TUNE_CACHE", str(path))
    P = datagen.make_problem(96, 96, 2.0, 70, 131, 2.0, 7, 3e5, attenuation=False, seed=21)
    A = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    t1 = A.tune()
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("svr-tune 2 96x96/"), lines
    B = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    fw = 3 if t1[0] != 3 else 4
    B.set_tuning(fw, 7, subset_fwd_batch=4 if A.batch_widths()[0] != 4 else 6, subset_bp_batch=3)
    t2 = B.tune()
    assert t2[:2] == t1[:2] and B.tuning() == t1[:2] and B.batch_widths() == A.batch_widths()
    assert abs(t2[2] - t1[2]) < 1e-3 and abs(t2[3] - t1[3]) < 1e-3
    assert len(path.read_text().splitlines()) == 1
    Q = datagen.make_problem(64, 64, 2.0, 40, 91, 2.0, 5, 1e5, attenuation=False, seed=22)
    C = pkg.SystemMatrix(Q.geom, Q.n_subsets, pkg.SVR_W_F32)
    C.tune()
    assert len(path.read_text().splitlines()) == 2
    path.write_text("not a tuning line\nsvr-tune 2 " + lines[0].split()[2] + " fwd 99 bp 1 fu 8 bu 5 fwd_us 1 bp_us 1\n"
                    + "svr-tune 1 " + lines[0].split()[2] + " fwd 5 bp 2 fwd_us 1 bp_us 1\n"
                    + "\n".join(path.read_text().splitlines()) + "\n")
    D = pkg.SystemMatrix(P.geom, P.n_subsets, pkg.SVR_W_F32)
    assert D.tune()[:2] == t1[:2]   # the out-of-range and the old-format lines are skipped, the valid one used
    assert D.batch_widths() == A.batch_widths()
