"""GPU tests of the Euclidean cost C_ij = ||x_i - X_j|| / scale (Sec. IV,
cost choice (i)), regenerated from the positions on the fly, against the
FP64 oracle's distance cost.

Bars: the materialised FP32 cost is the FP64 distance rounded once (relative
error <= 2^-23 with one FP64 ulp of slack); the FP32 median selection is
within 2e-6 of the oracle's FP64 lower median; solves on both the cooperative
and the chunked path meet the FP32-path bar of the other parity tests
(marginal violation < tol, transport cost within 1e-6 relative of the
oracle's converged solution, plan L1 <= 1e-6); the maxSINR rule under this
cost is the nearest RRH wherever the two nearest differ by more than 1e-9
relative; batches and snapshots take the materialised FP32 cost.
"""

import numpy as np
import pytest

import scenario as S

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-6
PLAN_L1 = 1e-6


@pytest.fixture(scope="module")
def A():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_01559_amd import ot_assoc
    ot_assoc.lib()
    return ot_assoc


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def check(O, C, a, b, eps, tol, f, g, res, ref):
    chk = O.plan_stats(C, a, b, f, g, eps)
    rst = O.plan_stats(C, a, b, ref.f, ref.g, eps)
    assert res.marginal_violation < tol, res.marginal_violation
    assert chk["marginal_violation"] < tol * 1.05, chk["marginal_violation"]
    assert abs(chk["objective"] - rst["objective"]) <= OBJ_RTOL * abs(rst["objective"])
    assert abs(res.objective - chk["objective"]) <= 1e-9 * abs(chk["objective"])
    l1 = np.abs(O.plan(C, f, g, eps) - O.plan(C, ref.f, ref.g, eps)).sum()
    assert l1 <= PLAN_L1, l1


@pytest.fixture(scope="module")
def lay(oracle_lib):
    L = S.make_layout(3000, 150, 2000.0, hot_spots=2, hot_share=0.4, seed=8150)
    C, scale = oracle_lib.distance_cost(L, 0.0)
    return dict(L=L, C=C, scale=scale)


def test_euclid_materialise_and_median(A, oracle_lib, lay):
    announce("distance cost 3000x150: materialised FP32 cost and FP32 median")
    import torch
    L, C, scale = lay["L"], lay["C"], lay["scale"]
    with A.Solver(L.I, L.J) as s:
        d, keep = A.euclid_desc(L.dev_xy, L.rrh_xy, 1.0)
        med = s.cost_median(d)
        assert abs(med - scale) <= 2e-6 * scale, (med, scale)
        Cdev = torch.empty((L.I, L.J), dtype=torch.float32, device="cuda:0")
        d, keep = A.euclid_desc(L.dev_xy, L.rrh_xy, scale)
        s.materialize_cost(d, Cdev)
    Cm = Cdev.cpu().numpy().astype(np.float64)
    err = np.abs(Cm - C)
    assert np.all(err <= 2.0 ** -24 * C * (1 + 1e-12) + 1e-300), (err / np.maximum(C, 1e-300)).max()


@pytest.mark.parametrize("persistent", [1, 0])
def test_euclid_solve_both_paths(A, oracle_lib, lay, persistent):
    announce(f"distance cost 3000x150 solve, persistent={persistent}")
    L, C, scale = lay["L"], lay["C"], lay["scale"]
    eps, tol = 0.05, 1e-8
    ref = oracle_lib.sinkhorn(C, L.a, L.b, eps, 1e-12, 20000)
    with A.Solver(L.I, L.J, persistent=persistent) as s:
        st, res = s.solve_euclid(L.dev_xy, L.rrh_xy, scale, L.a, L.b, eps, tol, 3000)
        assert st == A.OT_OK
        assert bool(res.flags & A.OT_RESULT_PERSISTENT) == bool(persistent)
        f, g = s.potentials()
        P = s.plan()
    check(oracle_lib, C, L.a, L.b, eps, tol, f, g, res, ref)
    # the library's plan is the FP64 plan of its own potentials
    np.testing.assert_allclose(P, oracle_lib.plan(C, f, g, eps), rtol=1e-12, atol=1e-300)


def test_euclid_cran_20000x400(A, oracle_lib):
    announce("distance cost at 20000 x 400, device positions, cooperative")
    import torch
    L = S.preset_layout("cran_20000x400")
    C, scale = oracle_lib.distance_cost(L, 0.0)
    eps, tol = 0.05, 1e-8
    dev = torch.device("cuda:0")
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    ad, bd = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    ref = oracle_lib.sinkhorn(C, L.a, L.b, eps, 1e-12, 20000)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_euclid(xy, rxy, scale, ad, bd, eps, tol, 5000)
        assert st == A.OT_OK
        assert res.flags & A.OT_RESULT_PERSISTENT
        f, g = s.potentials()
    check(oracle_lib, C, L.a, L.b, eps, tol, f, g, res, ref)


def test_euclid_maxsinr_is_the_nearest_rrh(A, oracle_lib, lay):
    announce("maxSINR rule under the distance cost: the nearest RRH")
    L, C = lay["L"], lay["C"]
    with A.Solver(L.I, L.J) as s:
        assoc, lam = s.maxsinr(*A.euclid_desc(L.dev_xy, L.rrh_xy, lay["scale"]), L.lam)
    srt = np.sort(C, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-9 * srt[:, 0]
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(assoc[clear], np.argmin(C, axis=1)[clear])
    np.testing.assert_allclose(lam, np.bincount(assoc, weights=L.lam, minlength=L.J), rtol=1e-12)


def test_euclid_batch_and_snapshots(A, oracle_lib):
    announce("distance costs in a batch (with the median scale) and in a snapshot solve")
    import torch
    dev = torch.device("cuda:0")
    eps, tol = 0.05, 1e-8
    cases = []
    for k, (I, J) in enumerate([(900, 33), (1501, 130), (700, 400)]):
        L = S.make_layout(I, J, 1500.0, seed=8200 + k)
        C, scale = oracle_lib.distance_cost(L, 0.0)
        cases.append((L, C, scale))
    descs, aa, bb, keep = [], [], [], []
    for k, (L, C, scale) in enumerate(cases):
        xy = torch.from_numpy(L.dev_xy).to(dev)
        rxy = torch.from_numpy(L.rrh_xy).to(dev)
        keep += [xy, rxy]
        # the last instance asks the batch for the median itself
        descs.append(A.euclid_desc(xy, rxy, scale if k < 2 else 0.0))
        aa.append(torch.from_numpy(L.a).to(dev))
        bb.append(torch.from_numpy(L.b).to(dev))
    with A.Solver(16, 16) as s:
        st, res = s.solve_batch(descs, aa, bb, eps, tol, 3000)
        assert st == A.OT_OK, [r.status for r in res]
        for k, (L, C, scale) in enumerate(cases):
            f, g = s.batch_potentials(k)
            # the batch solves the FP32-rounded cost: judged on the FP64 one
            # with the marginal slack that rounding allows (|dC| / eps)
            chk = oracle_lib.plan_stats(C, L.a, L.b, f, g, eps)
            ref = oracle_lib.sinkhorn(C, L.a, L.b, eps, 1e-12, 20000)
            rst = oracle_lib.plan_stats(C, L.a, L.b, ref.f, ref.g, eps)
            assert res[k].marginal_violation < tol
            assert abs(chk["objective"] - rst["objective"]) <= OBJ_RTOL * abs(rst["objective"])
            assert chk["marginal_violation"] < tol + 2.0 ** -23 * C.max() / eps * 2
    # snapshots over a distance cost (BF16 path, its own 1e-3 bar)
    L, C, scale = cases[1]
    As = S.snapshot_marginals(L.I, 4, seed=8300)
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_snapshots(A.euclid_desc(xy, rxy, scale), torch.from_numpy(As).to(dev),
                                    torch.from_numpy(L.b).to(dev), eps, 1e-6, 3000)
        assert st == A.OT_OK
        Cq = C.astype(np.float32).astype(np.float64)
        for q in range(4):
            f, g = s.snapshot_potentials(q)
            chk = oracle_lib.plan_stats(Cq, As[q], L.b, f, g, eps)
            ref = oracle_lib.sinkhorn(Cq, As[q], L.b, eps, 1e-11, 20000)
            rst = oracle_lib.plan_stats(Cq, As[q], L.b, ref.f, ref.g, eps)
            assert chk["marginal_violation"] < 1e-3
            assert abs(chk["objective"] - rst["objective"]) < 1e-3 * abs(rst["objective"])


def test_euclid_rejects_bad_inputs(A, lay):
    announce("distance cost validation")
    L = lay["L"]
    with A.Solver(L.I, L.J) as s:
        with pytest.raises(A.OTError) as e:
            s.solve_euclid(L.dev_xy, L.rrh_xy, 0.0, L.a, L.b, 0.05, 1e-8, 100)
        assert e.value.status == A.OT_EINVAL and "scale" in str(e.value)
        bad = L.dev_xy.copy()
        bad[17, 1] = np.nan
        with pytest.raises(A.OTError) as e:
            s.solve_euclid(bad, L.rrh_xy, 1.0, L.a, L.b, 0.05, 1e-8, 100)
        assert e.value.status == A.OT_EINVAL and "non-finite" in str(e.value)
        # a valid solve on the same handle afterwards
        st, res = s.solve_euclid(L.dev_xy, L.rrh_xy, lay["scale"], L.a, L.b, 0.05, 1e-8, 3000)
        assert st == A.OT_OK


def test_euclid_adaptive_and_evaluation(A, oracle_lib):
    """Alg. 2 and the Sec. II-B evaluation under the distance cost (the
    paper's policy with Euclidean costs), against the oracle on the same
    FP64 distances."""
    announce("Alg. 2 and evaluation under the distance cost, 1500 x 12")
    import torch
    dev = torch.device("cuda:0")
    L = S.make_layout(1500, 12, 1500.0, hot_spots=1, hot_share=0.5, seed=8400)
    C, scale = oracle_lib.distance_cost(L, 0.0)
    eps, tol, cap = 0.05, 1e-9, 30
    want = oracle_lib.adaptive_sinkhorn(C, L.a, eps, tol, 20000, max_outer=cap)
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    with A.Solver(L.I, L.J) as s:
        st, q, js, r = s.adaptive(*A.euclid_desc(xy, rxy, scale), torch.from_numpy(L.a).to(dev), eps, tol, 20000,
                                  0.0, cap)
        assert st == A.OT_OK
        loads = s.rrh_loads()
        f, g = s.potentials()
        kappa, tau = 0.7 / loads.max(), 2.0
        rho, en, ev = s.evaluate(kappa, tau)
    # the handle holds the returned solve; its loads and evaluation against
    # the oracle's computation from the same potentials
    np.testing.assert_allclose(loads, oracle_lib.rrh_loads(C, f, g, eps), rtol=1e-12)
    ref = oracle_lib.evaluate(C, f, g, eps, L.a, kappa, tau)
    np.testing.assert_allclose(rho, ref["rho"], rtol=1e-12)
    np.testing.assert_allclose(en, ref["EN"], rtol=1e-11)
    assert abs(ev.mean_completion - ref["T_mean"]) <= 1e-11 * ref["T_mean"]
    assert r.max_load <= r.first_max_load
    chk = oracle_lib.plan_stats(C, L.a, q, f, g, eps)
    assert chk["marginal_violation"] < tol * 1.05
    # the same first decision as the oracle unless its two largest loads tie
    first = oracle_lib.sinkhorn(C, L.a, np.full(L.J, L.a.sum() / L.J), eps, tol, 20000)
    ld = np.sort(oracle_lib.rrh_loads(C, first.f, first.g, eps))
    if ld[-1] - ld[-2] > 1e-6 * ld[-1]:
        assert js[0] == want["history"][0][0]
    if r.solves == want["solves"]:
        assert abs(r.max_load - want["max_load"]) <= 1e-6 * want["max_load"]


def test_euclid_served_requests(A, oracle_lib):
    """Distance-cost requests through the serving queue (positions and
    marginals in device memory, the cost materialised at admission): each
    matches the oracle on the FP32-rounded distances to the FP32-path bar,
    and a repeat of a layout starts warm."""
    announce("distance-cost requests through the serving queue")
    import torch
    dev = torch.device("cuda:0")
    eps, tol = 0.05, 1e-8
    cases, keep = [], []
    for k, (I, J) in enumerate([(800, 30), (1900, 140), (1200, 333)]):
        L = S.make_layout(I, J, 1200.0, hot_spots=1, hot_share=0.3, seed=8500 + k)
        C, scale = oracle_lib.distance_cost(L, 0.0)
        xy = torch.from_numpy(L.dev_xy).to(dev)
        rxy = torch.from_numpy(L.rrh_xy).to(dev)
        ad, bd = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
        keep += [xy, rxy, ad, bd]
        cases.append((L, C, scale, xy, rxy, ad, bd))
    with A.Server() as srv:
        for k, (L, C, scale, xy, rxy, ad, bd) in enumerate(cases):
            srv.submit(A.euclid_desc(xy, rxy, scale), ad, bd, eps, tol, 3000, layout_key=900 + k, user_tag=k)
        done = run_until_done(srv, len(cases))
        for c in done:
            L, C, scale = cases[c.user_tag][:3]
            assert c.result.status == A.OT_OK, c.result.status
            f, g = srv.potentials(900 + c.user_tag, L.I, L.J)
            Cq = C.astype(np.float32).astype(np.float64)
            chk = oracle_lib.plan_stats(Cq, L.a, L.b, f, g, eps)
            ref = oracle_lib.sinkhorn(Cq, L.a, L.b, eps, 1e-12, 20000)
            rs = oracle_lib.plan_stats(Cq, L.a, L.b, ref.f, ref.g, eps)
            assert c.result.marginal_violation < tol
            assert chk["marginal_violation"] < tol * 1.05
            assert abs(chk["objective"] - rs["objective"]) <= 1e-6 * abs(rs["objective"])
        # the same layout again: admitted warm from its resident potentials
        L, C, scale, xy, rxy, ad, bd = cases[1]
        srv.submit(A.euclid_desc(xy, rxy, scale), ad, bd, eps, tol, 3000, layout_key=901, user_tag=7)
        (c,) = run_until_done(srv, 1)
        assert c.result.status == A.OT_OK and c.warm
    del keep


def run_until_done(srv, n, limit=100000):
    done = []
    for _ in range(limit):
        done += srv.progress()
        if len(done) >= n:
            return done
    raise AssertionError("server did not finish")
