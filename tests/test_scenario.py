"""Scenario generator: determinism, shapes and the frozen recipe's statistics."""

import numpy as np

import scenario as S


def test_deterministic_per_seed():
    a = S.preset_layout("small_1000x50")
    b = S.preset_layout("small_1000x50")
    np.testing.assert_array_equal(a.dev_xy, b.dev_xy)
    np.testing.assert_array_equal(a.rrh_xy, b.rrh_xy)
    np.testing.assert_array_equal(a.lam, b.lam)
    assert a.shadow_key == b.shadow_key
    c = S.make_layout(1000, 50, 1000.0, seed=1)
    assert not np.array_equal(a.dev_xy, c.dev_xy)


def test_shapes_and_marginals():
    L = S.preset_layout("cran_20000x400")
    assert L.dev_xy.shape == (20000, 2) and L.dev_xy.dtype == np.float32
    assert L.rrh_xy.shape == (400, 2) and L.rrh_xy.dtype == np.float32
    assert abs(L.a.sum() - 1) < 1e-12 and abs(L.b.sum() - 1) < 1e-12
    assert (L.a > 0).all() and np.allclose(L.b, 1 / 400)
    assert (L.dev_xy >= 0).all() and (L.dev_xy <= 5000).all()
    # lambda is lognormal(0, 1)
    ll = np.log(L.lam)
    assert abs(ll.mean()) < 0.05 and abs(ll.std() - 1) < 0.05


def test_hot_spot_share():
    L = S.preset_layout("cran_20000x400")
    # the last 40 % of devices are the hot-spot ones; they are far more
    # clustered than the uniform ones
    hot = L.dev_xy[12000:]
    uni = L.dev_xy[:12000]
    def nn_density(p):
        g = np.floor(p / 100.0).astype(int)
        _, counts = np.unique(g[:, 0] * 1000 + g[:, 1], return_counts=True)
        return counts.max()
    assert nn_density(hot) > 5 * nn_density(uni)


def test_grid_shape_rule():
    assert S.grid_shape(50) == (5, 10)
    assert S.grid_shape(400) == (20, 20)
    assert S.grid_shape(2000) == (40, 50)
    r, c = S.grid_shape(23)  # prime: floor(sqrt) rows, enough columns
    assert r == 4 and r * c >= 23
    for J in range(1, 200):
        r, c = S.grid_shape(J)
        assert r * c >= J and r <= c + 1


def test_rrh_jitter_within_cells():
    L = S.preset_layout("small_1000x50")
    r, c = S.grid_shape(50)
    col = np.arange(50) % c
    row = np.arange(50) // c
    px, py = 1000.0 / c, 1000.0 / r
    dx = L.rrh_xy[:, 0] / px - (col + 0.5)
    dy = L.rrh_xy[:, 1] / py - (row + 0.5)
    assert (np.abs(dx) <= 0.25 + 1e-5).all() and (np.abs(dy) <= 0.25 + 1e-5).all()


def test_batch_sizes_log_uniform():
    sz = S.batch_sizes(256)
    Is = np.array([s[0] for s in sz])
    Js = np.array([s[1] for s in sz])
    assert Is.min() >= 500 and Is.max() <= 20000 and Js.min() >= 20 and Js.max() <= 400
    # log-uniform: the median sits near the geometric mean of the range
    assert 2000 < np.median(Is) < 5000 and 60 < np.median(Js) < 130


def test_drift_and_snapshots():
    L = S.make_layout(500, 30, 1000.0, seed=3)
    steps = S.drift_positions(L, 4, 5.0, seed=1)
    assert len(steps) == 4
    d = np.linalg.norm(steps[1].astype(np.float64) - steps[0], axis=1)
    assert (d <= 5.0 + 1e-3).all() and np.median(d) > 4.0
    assert (steps[3] >= 0).all() and (steps[3] <= 1000).all()
    A = S.snapshot_marginals(500, 8)
    assert A.shape == (8, 500) and np.allclose(A.sum(1), 1)
    t = S.poisson_arrivals(200.0, 20000)
    assert abs(np.diff(t).mean() - 1 / 200) < 2e-4
