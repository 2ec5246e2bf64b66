"""Pins of the oracle's association-quality functions and of the Adaptive
Sinkhorn Association (Alg. 2), tied to closed forms and to the paper's own
definitions rather than to the oracle itself:

* RRH loads of Sec. II-B under constant and separable costs, where the
  entropic plan is a b^T / mass in closed form;
* the processor-sharing quantities E[N] = rho / (1 - rho) and the completion
  times of Sec. II-B for a single RRH, and the reduction of rho_j and T_i to
  the normalised-cost form (kappa, tau) against the paper's variables
  (lambda, mu, R, pi = x / lambda);
* Alg. 2's control flow: the listing's q update (mass preserved, only j*
  decreases), j* = argmax of the loads of an independent solve at the same
  q, a strictly falling maximum load up to the stop, the delta guard and the
  one-RRH case.
"""

import numpy as np
import pytest


def test_loads_constant_cost_closed_form(oracle_lib):
    # constant C = c: the entropic plan is a b^T / sum(a), so rho_j = c b_j
    rng = np.random.default_rng(11)
    I, J, c = 30, 6, 0.7
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = rng.uniform(0.5, 1.5, J)
    b /= b.sum()
    C = np.full((I, J), c)
    r = oracle_lib.sinkhorn(C, a, b, 0.1, 1e-13, 5000)
    np.testing.assert_allclose(oracle_lib.rrh_loads(C, r.f, r.g, 0.1), c * b, rtol=1e-10)


def test_loads_separable_cost_closed_form(oracle_lib):
    # C_ij = u_i + v_j: the plan is still a b^T / m (the separable part is
    # absorbed by the potentials), so rho_j = b_j (sum_i u_i a_i / m + v_j)
    rng = np.random.default_rng(12)
    I, J = 25, 4
    u, v = rng.uniform(0, 2, I), rng.uniform(0, 2, J)
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = rng.uniform(0.5, 1.5, J)
    b /= b.sum()
    C = u[:, None] + v[None, :]
    r = oracle_lib.sinkhorn(C, a, b, 0.2, 1e-13, 5000)
    expect = b * ((u * a).sum() + v)
    np.testing.assert_allclose(oracle_lib.rrh_loads(C, r.f, r.g, 0.2), expect, rtol=1e-9)
    # and the loads add up to the transport cost <C, x>
    st = oracle_lib.plan_stats(C, a, b, r.f, r.g, 0.2)
    assert abs(oracle_lib.rrh_loads(C, r.f, r.g, 0.2).sum() - st["objective"]) < 1e-12


def test_processor_sharing_single_rrh(oracle_lib):
    # J = 1: every device is served by the one RRH (x_i = a_i), so
    # rho = kappa sum_i C_i a_i, E[N] = rho / (1 - rho) and each device's
    # completion time is tau C_i / (1 - rho) (M/G/1 processor sharing)
    rng = np.random.default_rng(13)
    I = 12
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    C = rng.uniform(0.1, 1.0, (I, 1))
    r = oracle_lib.sinkhorn(C, a, np.array([1.0]), 0.05, 1e-13, 100)
    kappa, tau = 0.9, 2.5
    ev = oracle_lib.evaluate(C, r.f, r.g, 0.05, a, kappa, tau)
    rho = kappa * (C[:, 0] * a).sum()
    assert abs(ev["rho"][0] - rho) < 1e-13
    assert abs(ev["EN"][0] - rho / (1 - rho)) < 1e-12
    np.testing.assert_allclose(ev["T"], tau * C[:, 0] / (1 - rho), rtol=1e-12)
    # overloaded: no finite queue
    ev2 = oracle_lib.evaluate(C, r.f, r.g, 0.05, a, 10.0, tau)
    assert ev2["rho"][0] > 1 and np.isinf(ev2["EN"][0]) and np.isinf(ev2["T_mean"])


def test_evaluation_matches_the_papers_variables(oracle_lib):
    # rho_j = sum_i lambda_i pi_ij / (mu R_ij) and T_i = sum_j pi_ij /
    # (mu R_ij (1 - rho_j)) with pi = x / a, lambda = Lambda_tot a,
    # R = 1 / (scale C): the oracle's kappa / tau form must agree
    rng = np.random.default_rng(14)
    I, J = 40, 5
    C = rng.uniform(0.2, 1.0, (I, J))
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = np.full(J, 1.0 / J)
    r = oracle_lib.sinkhorn(C, a, b, 0.05, 1e-13, 5000)
    lam_tot, mu, scale = 2.4e6, 1.0e5, 0.05  # kappa = 1.2: every RRH below full load
    kappa, tau = lam_tot * scale / mu, scale / mu
    ev = oracle_lib.evaluate(C, r.f, r.g, 0.05, a, kappa, tau)
    x = oracle_lib.plan(C, r.f, r.g, 0.05)
    pi = x / a[:, None]
    lam = lam_tot * a
    R = 1.0 / (scale * C)
    rho = (lam[:, None] * pi / (mu * R)).sum(axis=0)
    T = (pi / (mu * R * (1 - rho[None, :]))).sum(axis=1)
    np.testing.assert_allclose(ev["rho"], rho, rtol=1e-12)
    np.testing.assert_allclose(ev["T"], T, rtol=1e-12)
    assert abs(ev["objective"] - T.sum()) <= 1e-12 * T.sum()


def two_rrh_hotspot(seed=21, I=60):
    # RRH 1 costs more per unit of traffic (a lower rate): under equal q it
    # carries the larger load, and Alg. 2 must move traffic towards RRH 0
    rng = np.random.default_rng(seed)
    C = np.stack([rng.uniform(0.2, 0.6, I), rng.uniform(0.5, 1.0, I)], axis=1)
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    return C, a


def test_adaptive_follows_the_listing(oracle_lib):
    C, a = two_rrh_hotspot()
    J = C.shape[1]
    eps, tol = 0.05, 1e-12
    r = oracle_lib.adaptive_sinkhorn(C, a, eps, tol, 20000)
    hist = r["history"]
    d = 0.01 * a.sum() / J
    # replay: q starts at sum(a) / J; every solve's j* is the argmax of the
    # loads of an independent solve at that q; only q_j* falls, by delta
    q = np.full(J, a.sum() / J)
    maxes = []
    for k, (js, mx) in enumerate(hist):
        s = oracle_lib.sinkhorn(C, a, q, eps, tol, 20000)
        loads = oracle_lib.rrh_loads(C, s.f, s.g, eps)
        assert js == int(np.argmax(loads)) and abs(mx - loads.max()) < 1e-12
        maxes.append(mx)
        if k == r["outer"]:
            np.testing.assert_array_equal(q, r["q"])
        nq = q + d / (J - 1)
        nq[js] = q[js] - d
        assert abs(nq.sum() - q.sum()) < 1e-15
        q = nq
    # the maximum load falls strictly until the returned solve, and the solve
    # after it (if any) did not lower it
    assert all(maxes[k + 1] < maxes[k] for k in range(r["outer"]))
    if r["solves"] > r["outer"] + 1:
        assert maxes[r["outer"] + 1] >= maxes[r["outer"]]
    assert r["max_load"] == min(maxes) and r["max_load"] < maxes[0]
    # traffic moved from the most loaded RRH of the first solve to the other
    hot = hist[0][0]
    assert hot == 1 and r["q"][hot] < a.sum() / J < r["q"][1 - hot]


def test_adaptive_delta_guard_and_single_rrh(oracle_lib):
    C, a = two_rrh_hotspot(seed=22)
    # delta as large as an RRH's whole share: no step keeps q positive
    r = oracle_lib.adaptive_sinkhorn(C, a, 0.05, 1e-12, 20000, delta=a.sum() / 2)
    assert r["solves"] == 1 and r["outer"] == 0
    np.testing.assert_array_equal(r["q"], np.full(2, a.sum() / 2))
    # one RRH: a single solve, nothing to rebalance
    r1 = oracle_lib.adaptive_sinkhorn(C[:, :1], a, 0.05, 1e-12, 200)
    assert r1["solves"] == 1 and r1["q"][0] == pytest.approx(a.sum())
    # max_outer caps the number of solves
    r2 = oracle_lib.adaptive_sinkhorn(C, a, 0.05, 1e-12, 20000, delta=1e-5, max_outer=3)
    assert r2["solves"] == 3
