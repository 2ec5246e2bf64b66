"""Pins that tie the FP64 oracle to the paper and to mathematics, not to itself.

Each test names what fixes the expected value: a closed form, an identity of
the regularised problem (eq. (5) and its KKT form, Sec. III-B), brute force
over permutations (eqs. (2)-(4) via Birkhoff), an independent LP solver, the
Lemma of Sec. IV, or published generator outputs (tests/golden/).
"""

import math
import os

import numpy as np
import pytest
from scipy import stats
from scipy.optimize import linprog

import scenario as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_instance(rng, I, J, cost_scale=1.0):
    C = rng.uniform(0.0, cost_scale, size=(I, J))
    a = rng.uniform(0.5, 1.5, size=I)
    a /= a.sum()
    b = rng.uniform(0.5, 1.5, size=J)
    b /= b.sum()
    return C, a, b


# --------------------------------------------------------------- generator --

def test_splitmix64_published_outputs(oracle_lib):
    rows = [ln.split() for ln in open(os.path.join(GOLD, "splitmix64_seed0.txt")) if not ln.startswith("#")]
    for _, state, out in rows:
        assert oracle_lib.splitmix64(int(state, 16)) == int(out, 16)


def test_shadowing_is_standard_normal(oracle_lib):
    # Box-Muller of uniform hash outputs must be N(0, 1): a dropped factor 2,
    # a missing sqrt or a cos/sin slip changes the variance or the shape.
    key = 0x1234_5678_9ABC_DEF1
    xs = np.array([oracle_lib.shadow_normal(key, i, j) for i in range(300) for j in range(200)])
    assert abs(xs.mean()) < 5.0 / math.sqrt(xs.size)
    assert abs(xs.var() - 1.0) < 0.03
    assert stats.kstest(xs, "norm").pvalue > 1e-3
    # counter based: same (key, i, j) -> same draw; different key -> different draw
    assert oracle_lib.shadow_normal(key, 7, 3) == oracle_lib.shadow_normal(key, 7, 3)
    assert oracle_lib.shadow_normal(key, 7, 3) != oracle_lib.shadow_normal(key + 2, 7, 3)


def _closed_form_layout(K0, alpha, dmin, N0, dev, rrhs):
    radio = dict(S.RADIO, tx_power_w=1.0, ref_gain=K0, pathloss_exp=alpha, min_dist_m=dmin,
                 shadow_sigma_db=0.0, noise_w=N0, bandwidth_hz=1.0)
    return S.Layout(dev_xy=np.array([dev], dtype=np.float32), rrh_xy=np.array(rrhs, dtype=np.float32),
                    lam=np.ones(1), a=np.ones(1), b=np.ones(len(rrhs)) / len(rrhs), shadow_key=1,
                    side_m=1000.0, seed=0, radio=radio)


def test_rate_closed_forms(oracle_lib):
    for ln in open(os.path.join(GOLD, "rate_closed_forms.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        tok = ln.split()
        K0, alpha, dmin, N0 = map(float, tok[1:5])
        dev = (float(tok[5]), float(tok[6]))
        rest = list(map(float, tok[7:]))
        nr = len(rest) // 3
        rrhs = [(rest[2 * k], rest[2 * k + 1]) for k in range(nr)]
        expect = rest[2 * nr:]
        L = _closed_form_layout(K0, alpha, dmin, N0, dev, rrhs)
        R = oracle_lib.rates(L)[0]
        np.testing.assert_allclose(R, expect, rtol=1e-12, err_msg=tok[0])


# Shadowing pin: layouts in which every link has the same path loss and there
# is no noise, so the rate is a closed form of the shadowing draws alone
# (tests/golden/shadow_rates.txt, written from the definitions by
# make_shadow_golden.py without the oracle). Sec. II-A downlink model.
RRH_AT_100 = [(100.0, 0.0), (-100.0, 0.0), (0.0, 100.0), (0.0, -100.0)]


def _shadow_cases():
    for ln in open(os.path.join(GOLD, "shadow_rates.txt")):
        if ln.startswith("#") or not ln.strip():
            continue
        t = ln.split()
        n = int(t[3])
        per = t[5:5 + 3 * n]
        rest = list(map(float, t[5 + 3 * n:]))
        yield dict(name=t[0], key=int(t[1], 16), i=int(t[2]), n=n, sigma=float(t[4]),
                   h=[int(per[3 * j], 16) for j in range(n)], X=[float(per[3 * j + 1]) for j in range(n)],
                   R=[float(per[3 * j + 2]) for j in range(n)], R_slip=rest[:n], R_swap=rest[n:])


def _shadow_layout(c):
    radio = dict(S.RADIO, tx_power_w=1.0, ref_gain=10.0 ** -3.8, pathloss_exp=3.5, min_dist_m=10.0,
                 shadow_sigma_db=c["sigma"], noise_w=0.0, bandwidth_hz=20e6)
    return S.Layout(dev_xy=np.zeros((c["i"] + 1, 2), dtype=np.float32),
                    rrh_xy=np.array(RRH_AT_100[:c["n"]], dtype=np.float32), lam=np.ones(c["i"] + 1),
                    a=np.ones(c["i"] + 1) / (c["i"] + 1), b=np.ones(c["n"]) / c["n"], shadow_key=c["key"],
                    side_m=1000.0, seed=0, radio=radio)


def _shadow_check(shadow_normal, rates_rows):
    """Returns the first mismatch against the golden, or None."""
    for c in _shadow_cases():
        for j in range(c["n"]):
            x = shadow_normal(c["key"], c["i"], j)
            if not abs(x - c["X"][j]) <= 1e-13 * max(1.0, abs(c["X"][j])):
                return f"{c['name']}: X_{j} = {x!r}, golden {c['X'][j]!r}"
        R = rates_rows(_shadow_layout(c), [c["i"]])[0]
        if not np.allclose(R, c["R"], rtol=1e-12, atol=0):
            return f"{c['name']}: R = {R}, golden {c['R']}"
    return None


def test_shadowing_golden(oracle_lib):
    cases = list(_shadow_cases())
    assert len(cases) >= 6
    for c in cases:
        # the draws come from the pinned SplitMix64 mixer at state key ^ (i 2^32 + j)
        for j in range(c["n"]):
            assert oracle_lib.splitmix64(c["key"] ^ ((c["i"] << 32) + j)) == c["h"][j]
        # the golden separates the reading from the two plausible slips by far more than the tolerance
        for r, a, b in zip(c["R"], c["R_slip"], c["R_swap"]):
            assert abs(a - r) > 1e-3 * r and abs(b - r) > 1e-3 * r
    assert _shadow_check(oracle_lib.shadow_normal, oracle_lib.rates_rows) is None


def _mutant_oracle(tmp_path, old, new):
    """Builds a copy of the oracle with one planted mistake (CPU only) and
    returns (shadow_normal, rates_rows) bound to it."""
    import ctypes as ct
    import subprocess

    from oracle import oracle as O

    src = open(O.SRC_PATH).read()
    assert src.count(old) == 1, old
    path = tmp_path / "mut.c"
    path.write_text(src.replace(old, new))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                    "-D_DEFAULT_SOURCE", "-o", str(so), str(path), "-lm"], check=True)
    L = ct.CDLL(str(so))
    L.ora_shadow_normal.restype = ct.c_double
    L.ora_shadow_normal.argtypes = [ct.c_uint64, ct.c_int64, ct.c_int64]
    L.ora_rates_rows.argtypes = [ct.POINTER(ct.c_float), ct.POINTER(ct.c_float), ct.c_int64,
                                 ct.POINTER(O._Radio), ct.POINTER(ct.c_int64), ct.c_int64, ct.POINTER(ct.c_double)]

    def shadow_normal(key, i, j):
        return float(L.ora_shadow_normal(ct.c_uint64(key), i, j))

    def rates_rows(layout, rows):
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        dev = np.ascontiguousarray(layout.dev_xy, dtype=np.float32)
        rrh = np.ascontiguousarray(layout.rrh_xy, dtype=np.float32)
        out = np.empty((rows.size, layout.J))
        rad = O.radio_struct(layout)
        assert L.ora_rates_rows(dev.ctypes.data_as(ct.POINTER(ct.c_float)), rrh.ctypes.data_as(ct.POINTER(ct.c_float)),
                                layout.J, ct.byref(rad), rows.ctypes.data_as(ct.POINTER(ct.c_int64)), rows.size,
                                out.ctypes.data_as(ct.POINTER(ct.c_double))) == 0
        return out

    return shadow_normal, rates_rows


@pytest.mark.parametrize("old,new", [
    ("shadow_sigma_db * X / 10.0", "shadow_sigma_db * X / 20.0"),  # a /20 (amplitude dB) slip
    ("double u1 = ((double)(h >> 32) + 0.5)", "double u1 = ((double)(h & 0xFFFFFFFFULL) + 0.5)"),  # halves swapped
    ("double u2 = ((double)(h & 0xFFFFFFFFULL) + 0.5)", "double u2 = ((double)(h >> 32) + 0.5)"),
    ("cos(2.0 * M_PI * u2)", "sin(2.0 * M_PI * u2)"),
])
def test_shadowing_golden_catches_planted_mistakes(tmp_path, old, new):
    # the same check, run on an oracle with one plausible mistake planted, must fail
    assert _shadow_check(*_mutant_oracle(tmp_path, old, new)) is not None


def test_lower_median(oracle_lib):
    assert oracle_lib.lower_median([3.0, 1.0, 2.0, 4.0]) == 2.0
    assert oracle_lib.lower_median([5.0]) == 5.0
    assert oracle_lib.lower_median([9.0, 7.0, 8.0]) == 8.0


def test_cost_is_median_normalised(oracle_lib):
    L = S.make_layout(60, 7, 1000.0, seed=11)
    C, scale = oracle_lib.cost(L)
    R = oracle_lib.rates(L)
    assert scale == pytest.approx(np.sort((1.0 / R).ravel())[(R.size - 1) // 2], rel=0, abs=0)
    # the normalised cost has lower median exactly 1
    assert np.sort(C.ravel())[(C.size - 1) // 2] == pytest.approx(1.0, rel=1e-15)
    # rates are positive and a closer RRH never has a lower rate without shadowing
    assert (R > 0).all()


def test_rate_rows_match_full(oracle_lib):
    L = S.make_layout(40, 9, 1000.0, seed=5)
    R = oracle_lib.rates(L)
    rows = np.array([3, 17, 39])
    np.testing.assert_array_equal(oracle_lib.rates_rows(L, rows), R[rows])


def test_rates_against_brute_force_interference(oracle_lib):
    # Sec. II-A: SINR_ji = P G_ji / (sum over every other RRH of P G_li + N0).
    # Without shadowing the gain is K0 max(d, d_min)^-alpha; the interference
    # is summed here term by term with math.fsum (exactly rounded).
    L = S.make_layout(6, 11, 1000.0, seed=21)
    L.radio = dict(L.radio, shadow_sigma_db=0.0)
    R = oracle_lib.rates(L)
    r = L.radio
    for i in range(L.I):
        d = [max(math.hypot(float(L.dev_xy[i, 0]) - float(L.rrh_xy[j, 0]),
                            float(L.dev_xy[i, 1]) - float(L.rrh_xy[j, 1])), r["min_dist_m"]) for j in range(L.J)]
        pg = [r["tx_power_w"] * r["ref_gain"] * dj ** -r["pathloss_exp"] for dj in d]
        for j in range(L.J):
            interf = math.fsum(pg[k] for k in range(L.J) if k != j)
            expect = r["bandwidth_hz"] * math.log2(1.0 + pg[j] / (interf + r["noise_w"]))
            assert R[i, j] == pytest.approx(expect, rel=1e-13)
    # relabelling the RRHs relabels the columns (no shadowing, so no draw moves)
    perm = np.random.default_rng(21).permutation(L.J)
    Lp = S.Layout(dev_xy=L.dev_xy, rrh_xy=L.rrh_xy[perm].copy(), lam=L.lam, a=L.a, b=L.b, shadow_key=L.shadow_key,
                  side_m=L.side_m, seed=L.seed, radio=L.radio)
    np.testing.assert_allclose(oracle_lib.rates(Lp), R[:, perm], rtol=1e-14)


def test_geometry_plan_stats_matches_dense_stats(oracle_lib):
    # the row-by-row statistics equal those of the materialised cost
    L = S.make_layout(300, 17, 1000.0, seed=22)
    C, scale = oracle_lib.cost(L)
    rng = np.random.default_rng(22)
    eps = 0.05
    r = oracle_lib.sinkhorn(C, L.a, L.b, eps, 1e-6, 1000)
    f = r.f + rng.normal(0, 1e-3, L.I)
    g = r.g + rng.normal(0, 1e-3, L.J)
    ref = oracle_lib.plan_stats(C, L.a, L.b, f, g, eps)
    got = oracle_lib.geometry_plan_stats(L, scale, f, g, eps)
    assert got["marginal_violation"] == pytest.approx(ref["marginal_violation"], rel=1e-12)
    assert got["objective"] == pytest.approx(ref["objective"], rel=1e-13)
    assert got["mass"] == pytest.approx(ref["mass"], rel=1e-14)
    np.testing.assert_allclose(got["row_sums"], ref["row_sums"], rtol=1e-14)
    np.testing.assert_allclose(got["col_sums"], ref["col_sums"], rtol=1e-13)


# ------------------------------------------------------------- Sinkhorn -----

def test_P1_separable_cost_gives_product_plan(oracle_lib):
    # C_ij = u_i + v_j: the kernel is rank one, so one row and one column
    # update already give pi = a b^T / sum(a) (KKT form of Sec. III-B).
    rng = np.random.default_rng(1)
    I, J = 37, 11
    u, v = rng.uniform(0, 3, I), rng.uniform(0, 3, J)
    C = u[:, None] + v[None, :]
    _, a, b = rand_instance(rng, I, J)
    res = oracle_lib.sinkhorn(C, a, b, 0.07, 1e-14, 5)
    pi = oracle_lib.plan(C, res.f, res.g, 0.07)
    expect = np.outer(a, b) / a.sum()
    assert np.abs(pi - expect).max() <= 1e-13 * expect.max()
    assert res.iters == 1
    # constant cost: the named special case
    res = oracle_lib.sinkhorn(np.full((I, J), 0.3), a, b, 0.05, 1e-14, 5)
    pi = oracle_lib.plan(np.full((I, J), 0.3), res.f, res.g, 0.05)
    assert np.abs(pi - expect).max() <= 1e-13 * expect.max()


def test_P2_marginals_at_return(oracle_lib):
    rng = np.random.default_rng(2)
    C, a, b = rand_instance(rng, 50, 20)
    for tol in (1e-3, 1e-6, 1e-10):
        res = oracle_lib.sinkhorn(C, a, b, 0.05, tol, 5000)
        st = oracle_lib.plan_stats(C, a, b, res.f, res.g, 0.05)
        assert res.status == 0 and st["marginal_violation"] < tol
        assert st["marginal_violation"] == pytest.approx(res.residual, rel=1e-9, abs=1e-16)
        # column marginals are met exactly after the column update
        assert np.abs(st["col_sums"] - b).max() < 1e-14


def test_P3_primal_dual_gap_identity(oracle_lib):
    # P_eps(pi(f,g)) - D_eps(f,g) = sum_i f_i (r_i - a_i) + sum_j g_j (c_j - b_j)
    rng = np.random.default_rng(3)
    C, a, b = rand_instance(rng, 30, 12)
    eps = 0.08
    for k in (1, 2, 4, 8, 30):
        res = oracle_lib.sinkhorn(C, a, b, eps, 0.0, k)
        st = oracle_lib.plan_stats(C, a, b, res.f, res.g, eps)
        gap = st["reg_objective"] - st["dual_objective"]
        rhs = (res.f * (st["row_sums"] - a)).sum() + (res.g * (st["col_sums"] - b)).sum()
        assert gap == pytest.approx(rhs, abs=1e-13)
    assert abs(gap) < 1e-9  # and the gap closes at convergence


def test_P4_unique_optimum_from_any_start(oracle_lib):
    rng = np.random.default_rng(4)
    C, a, b = rand_instance(rng, 40, 15)
    eps, tol = 0.05, 1e-11
    ref = oracle_lib.sinkhorn(C, a, b, eps, tol, 20000)
    pi0 = oracle_lib.plan(C, ref.f, ref.g, eps)
    for s in range(3):
        g0 = rng.normal(0, 1.0, size=15)
        res = oracle_lib.sinkhorn(C, a, b, eps, tol, 20000, g0=g0)
        pi = oracle_lib.plan(C, res.f, res.g, eps)
        assert np.abs(pi - pi0).sum() <= 10 * tol
        # the potentials agree up to the gauge f + c, g - c
        d = (res.f[:, None] + res.g[None, :]) - (ref.f[:, None] + ref.g[None, :])
        assert np.abs(d).max() < 1e-8


def test_P5_dual_ascent(oracle_lib):
    rng = np.random.default_rng(5)
    C, a, b = rand_instance(rng, 25, 10)
    eps = 0.03
    duals = []
    for k in range(1, 40):
        res = oracle_lib.sinkhorn(C, a, b, eps, 0.0, k)
        duals.append(oracle_lib.plan_stats(C, a, b, res.f, res.g, eps)["dual_objective"])
    duals = np.array(duals)
    assert (np.diff(duals) >= -1e-14 * np.abs(duals[1:])).all()
    assert duals[-1] > duals[0]


@pytest.mark.parametrize("n", [4, 6, 7])
def test_P6_eps_to_zero_against_brute_force(oracle_lib, n):
    rng = np.random.default_rng(60 + n)
    C = rng.uniform(0.0, 1.0, size=(n, n))
    a = b = np.full(n, 1.0 / n)
    ot0, sigma = oracle_lib.brute_force_ot(C)
    P = np.zeros((n, n))
    P[np.arange(n), sigma] = 1.0 / n
    l1 = []
    for eps in (1e-1, 3e-2, 1e-2):
        # small eps converges slowly when permutations nearly tie: cap the
        # work and widen the bound by the infeasibility actually left
        res = oracle_lib.sinkhorn(C, a, b, eps, 1e-9, 400000)
        assert res.residual < 1e-5
        slack = C.max() * res.residual + 1e-12
        st = oracle_lib.plan_stats(C, a, b, res.f, res.g, eps)
        gap = st["objective"] - ot0
        assert -slack <= gap <= eps * math.log(n) + slack
        l1.append(np.abs(oracle_lib.plan(C, res.f, res.g, eps) - P).sum())
    assert l1[2] <= l1[0]


def test_P7_against_independent_lp(oracle_lib):
    rng = np.random.default_rng(7)
    for I, J in [(5, 3), (7, 4), (3, 6)]:
        C, a, b = rand_instance(rng, I, J)
        A_eq = np.zeros((I + J, I * J))
        for i in range(I):
            A_eq[i, i * J:(i + 1) * J] = 1.0
        for j in range(J):
            A_eq[I + j, j::J] = 1.0
        lp = linprog(C.ravel(), A_eq=A_eq, b_eq=np.concatenate([a, b]), bounds=(0, None), method="highs")
        assert lp.status == 0
        for eps in (0.05, 0.01):
            res = oracle_lib.sinkhorn(C, a, b, eps, 1e-11, 400000)
            st = oracle_lib.plan_stats(C, a, b, res.f, res.g, eps)
            bound = eps * min(oracle_lib.entropy(a), oracle_lib.entropy(b))
            assert -1e-7 <= st["objective"] - lp.fun <= bound + 1e-7


def test_P8_lemma1_maxsinr_marginal(oracle_lib):
    # With C = 1/R (any positive scale), p = lambda and q = Lambda (maxSINR
    # traffic), the OT value equals sum_i a_i min_j C_ij (Lemma 1); the
    # regularised plan sits within eps * min(H(a), H(b)) above it.
    L = S.make_layout(300, 12, 1000.0, seed=8)
    R = oracle_lib.rates(L)
    C = 1.0 / R
    C = C / C.min(axis=1).max()  # row minima in (0, 1]
    lam = L.lam
    Lam = oracle_lib.maxsinr_traffic(R, lam)
    keep = Lam > 0  # RRHs that nobody picks carry no mass; drop those columns
    C, q = C[:, keep], Lam[keep] / lam.sum()
    a = lam / lam.sum()
    lb = oracle_lib.lemma1_lower_bound(C, a)
    for eps in (0.05, 0.02):
        # q = Lambda puts the LP optimum on a face where Sinkhorn converges
        # slowly; cap the work and allow for the residual left
        res = oracle_lib.sinkhorn(C, a, q, eps, 1e-9, 100000)
        assert res.residual < 1e-5
        st = oracle_lib.plan_stats(C, a, q, res.f, res.g, eps)
        obj = st["objective"]
        # any coupling pays at least sum_i rowsum_i min_j C_ij (exact, even off the marginals)
        assert obj >= (st["row_sums"] * C.min(axis=1)).sum() * (1 - 1e-12)
        assert obj <= lb + eps * min(oracle_lib.entropy(a), oracle_lib.entropy(q)) + 1e-4
    # and the bound is tight: with a generic q the value is strictly larger
    res = oracle_lib.sinkhorn(C, a, np.full(q.size, 1.0 / q.size), 0.02, 1e-9, 100000)
    obj_eq = oracle_lib.plan_stats(C, a, np.full(q.size, 1.0 / q.size), res.f, res.g, 0.02)["objective"]
    assert obj_eq > obj


def test_P9_invariances(oracle_lib):
    rng = np.random.default_rng(9)
    C, a, b = rand_instance(rng, 20, 9)
    eps, tol = 0.04, 1e-12
    ref = oracle_lib.sinkhorn(C, a, b, eps, tol, 50000)
    pi = oracle_lib.plan(C, ref.f, ref.g, eps)
    # adding a separable term leaves the plan unchanged
    C2 = C + rng.uniform(-2, 2, 20)[:, None] + rng.uniform(-2, 2, 9)[None, :]
    r2 = oracle_lib.sinkhorn(C2, a, b, eps, tol, 50000)
    assert np.abs(oracle_lib.plan(C2, r2.f, r2.g, eps) - pi).max() < 1e-11
    # scaling cost and eps together leaves the plan unchanged
    r3 = oracle_lib.sinkhorn(3.0 * C, a, b, 3.0 * eps, tol, 50000)
    assert np.abs(oracle_lib.plan(3.0 * C, r3.f, r3.g, 3.0 * eps) - pi).max() < 1e-11
    # the transposed problem gives the transposed plan
    r4 = oracle_lib.sinkhorn(C.T.copy(), b, a, eps, tol, 50000)
    assert np.abs(oracle_lib.plan(C.T.copy(), r4.f, r4.g, eps) - pi.T).max() < 1e-11


def test_P10_degenerate_shapes(oracle_lib):
    rng = np.random.default_rng(10)
    _, a, b = rand_instance(rng, 13, 6)
    r = oracle_lib.sinkhorn(rng.uniform(size=(13, 1)), a, np.ones(1), 0.1, 1e-14, 3)
    np.testing.assert_allclose(oracle_lib.plan(np.zeros((13, 1)) + 0, r.f, r.g, 0.1).ravel() * 0 + 1, 1)
    C = rng.uniform(size=(13, 1))
    r = oracle_lib.sinkhorn(C, a, np.ones(1), 0.1, 1e-14, 3)
    np.testing.assert_allclose(oracle_lib.plan(C, r.f, r.g, 0.1).ravel(), a, rtol=1e-14)
    C = rng.uniform(size=(1, 6))
    r = oracle_lib.sinkhorn(C, np.ones(1), b, 0.1, 1e-14, 3)
    np.testing.assert_allclose(oracle_lib.plan(C, r.f, r.g, 0.1).ravel(), b, rtol=1e-14)


def test_rejects_invalid_inputs(oracle_lib):
    rng = np.random.default_rng(11)
    C, a, b = rand_instance(rng, 6, 4)
    bad = [
        (C, a, b, 0.0),  # eps must be positive
        (C, a * 2, b, 0.1),  # unbalanced mass
        (C, np.r_[0.0, a[1:] * (1 / a[1:].sum())], b, 0.1),  # zero marginal
        (np.where(np.eye(6, 4) > 0, np.nan, C), a, b, 0.1),  # non-finite cost
    ]
    for Cb, ab, bb, eps in bad:
        with pytest.raises(ValueError):
            oracle_lib.sinkhorn(Cb, ab, bb, eps, 1e-6, 10)


def test_residual_matches_paper_stop_rule_on_cfg_small(oracle_lib):
    # the 1000 x 50 workload converges to its 1e-9 stop rule, with the
    # residual decreasing geometrically (linear convergence of Sinkhorn)
    L = S.preset_layout("small_1000x50")
    C, _ = oracle_lib.cost(L)
    res = oracle_lib.sinkhorn(C, L.a, L.b, 0.05, 1e-9, 2000, history=True)
    assert res.status == 0 and res.residual < 1e-9
    h = res.hist
    assert (h[5:] < h[4:-1]).all()
