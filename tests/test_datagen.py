"""The seeded input generator: determinism, sizes, totals and its
closed-form chord lengths (checked against dense sampling of the line)."""

import math

import numpy as np

import datagen
from datagen.phantoms import _ellipse_chords, _inside_ellipse


def test_deterministic_and_shapes():
    a = datagen.make_problem(**datagen.CONFIG_SMALL)
    b = datagen.make_problem(**datagen.CONFIG_SMALL)
    np.testing.assert_array_equal(a.g, b.g)
    assert a.g.shape == (1, 60 * 95) and a.w.shape == (1, 60 * 95)
    assert a.g.dtype == np.float32 and np.all(a.g >= 0) and np.all(np.floor(a.g) == a.g)
    assert abs(a.ybar_true.sum() - 1e5) < 1e-6 * 1e5
    assert np.all(a.w == a.w[0, 0]) and abs(a.w[0, 0] - 0.1 * a.ybar_true.mean()) < 1e-4
    assert a.mu is not None and a.mu.max() == np.float32(0.0096)


def test_chords_match_sampling():
    rng = np.random.default_rng(0)
    for _ in range(20):
        cx, cy = rng.uniform(-3, 3, 2)
        a, b = rng.uniform(0.5, 4, 2)
        phi = rng.uniform(0, math.pi)
        th = rng.uniform(0, math.pi)
        s = rng.uniform(-4, 4)
        px, py = np.array([s * math.cos(th)]), np.array([s * math.sin(th)])
        dx, dy = np.array([-math.sin(th)]), np.array([math.cos(th)])
        L = _ellipse_chords(px, py, dx, dy, cx, cy, a, b, phi)[0]
        t = np.linspace(-20, 20, 400001)
        inside = _inside_ellipse(px[0] + t * dx[0], py[0] + t * dy[0], cx, cy, a, b, phi)
        assert abs(inside.sum() * (t[1] - t[0]) - L) < 1e-3


def test_order_is_uniform_with_replacement():
    o = datagen.make_order(21, 21000, seed=0)
    assert o.dtype == np.int32 and o.min() == 0 and o.max() == 20
    counts = np.bincount(o, minlength=21)
    assert np.all(np.abs(counts - 1000) < 150)
    assert len(np.unique(o[:21])) < 21  # with replacement: repeats within an epoch


def test_multislice_small():
    p = datagen.make_multislice_problem(16, 16, 2.5, 12, 23, 2.5, 4, 1e5, n_slices=5, seed=2)
    assert p.g.shape == (5, 12 * 23) and p.f_true.shape == (5, 256)
    assert abs(p.ybar_true.sum() - 1e5) < 1e-3


def test_serving_stream():
    reqs = datagen.serving_requests(50, 10.0, seed=0)
    assert len(reqs) == 50
    assert all(r["nx"] in (128, 192, 256, 384) and 120 <= r["n_views"] <= 400 for r in reqs)
    assert all(r["n_subsets"] in (8, 14, 21) for r in reqs)
    assert all(1e5 <= r["counts"] <= 1e7 for r in reqs)
    t = [r["arrival_s"] for r in reqs]
    assert np.all(np.diff(t) > 0)
