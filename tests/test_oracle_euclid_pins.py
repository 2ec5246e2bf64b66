"""Pins of the oracle's Euclidean cost C_ij = ||x_i - X_j|| / scale (Sec. IV,
cost choice (i)): integer right triangles (a dropped square root or a wrong
axis fails them), scipy's cdist on a synthetic layout (an independent
implementation of the same definition), and the lower-median scale.
"""

from types import SimpleNamespace

import numpy as np
from scipy.spatial.distance import cdist

import scenario as S


def test_distance_cost_right_triangles(oracle_lib):
    L = SimpleNamespace(dev_xy=np.array([[3.0, 4.0], [0.0, 0.0], [-5.0, 12.0]], np.float32),
                        rrh_xy=np.array([[0.0, 0.0], [6.0, 8.0]], np.float32))
    C, s = oracle_lib.distance_cost(L, 1.0)
    assert s == 1.0
    np.testing.assert_array_equal(C, [[5.0, 5.0], [0.0, 10.0], [13.0, np.hypot(11.0, 4.0)]])
    C5, _ = oracle_lib.distance_cost(L, 5.0)
    np.testing.assert_array_equal(C5[:2], [[1.0, 1.0], [0.0, 2.0]])


def test_distance_cost_matches_cdist(oracle_lib):
    L = S.make_layout(700, 37, 2000.0, hot_spots=2, hot_share=0.4, seed=77)
    C, s = oracle_lib.distance_cost(L, 250.0)
    want = cdist(L.dev_xy.astype(np.float64), L.rrh_xy.astype(np.float64)) / 250.0
    np.testing.assert_allclose(C, want, rtol=2e-16 * 4, atol=0)
    assert C.shape == (700, 37) and s == 250.0


def test_distance_cost_median_scale(oracle_lib):
    L = S.make_layout(301, 9, 1500.0, seed=78)
    C, s = oracle_lib.distance_cost(L, 0.0)
    D = cdist(L.dev_xy.astype(np.float64), L.rrh_xy.astype(np.float64))
    n = D.size
    assert s == np.sort(D.ravel())[(n - 1) // 2]
    # the normalised cost has its lower median at exactly 1
    assert np.sort(C.ravel())[(n - 1) // 2] == 1.0
