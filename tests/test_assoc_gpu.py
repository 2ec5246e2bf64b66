"""GPU tests of the association-quality entry points against the FP64 oracle:
RRH loads and the processor-sharing evaluation of Sec. II-B, the maxSINR
rule and its traffic Lambda (Sec. II-A / IV), Lemma 1 at the 20000 x 400
workload, and the Adaptive Sinkhorn Association (Sec. IV, Alg. 2).

Bars: loads and evaluation computed by the library from its own potentials
agree with the oracle's computation from the same potentials to 1e-12
relative (both FP64); against the oracle's converged solution within 1e-6.
maxSINR associations: identical wherever the oracle's best and second-best
costs differ by more than 1e-9 relative (a closer pair may go either way
when the two sides evaluate the cost along different FP64 paths); Lambda
to 1e-12. Alg. 2: the same sequence of RRHs j* as the oracle up to the
first step whose two largest loads lie within 1e-6 relative (a near tie,
where either choice is valid), and with no such step the same q (to 1e-14)
and the same number of solves.
"""

import numpy as np
import pytest

import scenario as S

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def hot(oracle_lib):
    # 3000 devices, 60 RRHs, 2 km with two hot spots: an uneven load
    L = S.make_layout(3000, 60, 2000.0, hot_spots=2, hot_share=0.5, seed=6060)
    C64, scale = oracle_lib.cost(L)
    return dict(L=L, C64=C64, scale=scale, C32=C64.astype(np.float32))


def test_loads_and_evaluation(A, oracle_lib, hot):
    announce("RRH loads and processor-sharing evaluation, 3000 x 60")
    L, C32 = hot["L"], hot["C32"]
    Cq = C32.astype(np.float64)
    eps, tol = 0.05, 1e-9
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(C32, L.a, L.b, eps, tol, 5000)
        assert st == A.OT_OK
        f, g = s.potentials()
        loads = s.rrh_loads()
        np.testing.assert_allclose(loads, oracle_lib.rrh_loads(Cq, f, g, eps), rtol=1e-12)
        ref = oracle_lib.sinkhorn(Cq, L.a, L.b, eps, 1e-12, 20000)
        np.testing.assert_allclose(loads, oracle_lib.rrh_loads(Cq, ref.f, ref.g, eps), rtol=1e-6)
        # kappa below 1 / max load: no RRH overloaded
        kappa = 0.8 / loads.max()
        tau = 3.0
        rho, en, ev = s.evaluate(kappa, tau)
        want = oracle_lib.evaluate(Cq, f, g, eps, L.a, kappa, tau)
        np.testing.assert_allclose(rho, want["rho"], rtol=1e-12)
        np.testing.assert_allclose(en, want["EN"], rtol=1e-11)
        assert abs(ev.mean_completion - want["T_mean"]) <= 1e-11 * want["T_mean"]
        assert abs(ev.objective - want["objective"]) <= 1e-11 * want["objective"]
        assert ev.overloaded_rrhs == 0 and ev.devices_overloaded == 0
        assert abs(ev.max_rho - want["rho"].max()) <= 1e-12
        # overloaded: infinite queues and completion times
        rho2, en2, ev2 = s.evaluate(2.0 / loads.max(), tau)
        assert ev2.overloaded_rrhs == int((rho2 >= 1).sum()) > 0
        assert np.all(np.isinf(en2[rho2 >= 1])) and np.isinf(ev2.mean_completion)
        assert ev2.devices_overloaded > 0


def test_evaluation_needs_a_solve(A):
    announce("loads / evaluate before a solve")
    with A.Solver(10, 3) as s:
        with pytest.raises(A.OTError) as e:
            s._J = 3
            s.rrh_loads()
        assert e.value.status == A.OT_ESTATE


def _best_two(C):
    srt = np.sort(C, axis=1)
    return srt[:, 0], srt[:, 1]


def test_maxsinr_dense_and_geometry(A, oracle_lib, hot):
    announce("maxSINR association and traffic, dense FP32 and geometry")
    L, C32, scale = hot["L"], hot["C32"], hot["scale"]
    with A.Solver(L.I, L.J) as s:
        assoc, lam = s.maxsinr(*A.matrix_desc(C32, A.OT_COST_DENSE), L.lam)
    # dense: the same FP32 costs on both sides, so the decisions are exact
    Rq = 1.0 / C32.astype(np.float64)
    np.testing.assert_array_equal(assoc, oracle_lib.maxsinr_association(Rq))
    np.testing.assert_allclose(lam, oracle_lib.maxsinr_traffic(Rq, L.lam), rtol=1e-12)
    assert abs(lam.sum() - L.lam.sum()) <= 1e-12 * L.lam.sum()
    # geometry: the FP64 functor against the oracle's FP64 rates
    with A.Solver(L.I, L.J) as s:
        d, keep = A.geometry_desc(L.dev_xy, L.rrh_xy, L.radio, L.shadow_key, scale)
        assoc_g, lam_g = s.maxsinr(d, keep, L.lam)
    R = oracle_lib.rates(L)
    want = oracle_lib.maxsinr_association(R)
    c1, c2 = _best_two(1.0 / R)
    clear = (c2 - c1) > 1e-9 * c1
    assert clear.mean() > 0.99
    np.testing.assert_array_equal(assoc_g[clear], want[clear])
    np.testing.assert_allclose(lam_g, np.bincount(assoc_g, weights=L.lam, minlength=L.J), rtol=1e-12)


def test_lemma1_on_the_cran_workload(A, oracle_lib):
    """Lemma 1 at 20000 x 400: with q = Lambda from the GPU's maxSINR rule the
    entropic plan's transport cost sits between sum_i a_i min_j C_ij (any
    coupling pays at least that) and that bound plus eps min(H(a), H(q))."""
    announce("Lemma 1 with the maxSINR marginal, cran_20000x400")
    import torch
    L = S.preset_layout("cran_20000x400")
    C64, scale = oracle_lib.cost(L)
    C32 = C64.astype(np.float32)
    Cq = C32.astype(np.float64)
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(C32).to(dev)
    a = L.lam / L.lam.sum()
    with A.Solver(L.I, L.J) as s:
        assoc, lam = s.maxsinr(*A.matrix_desc(Cd, A.OT_COST_DENSE), torch.from_numpy(a).to(dev))
        keep = lam > 0  # RRHs nobody picks carry no mass
        Ck = np.ascontiguousarray(C32[:, keep])
        q = lam[keep]
        q = q / q.sum() * a.sum()
        eps = 0.01
        with A.Solver(L.I, int(keep.sum())) as s2:
            st, res = s2.solve_dense(Ck, a, q, eps, 1e-6, 20000)
            assert st in (A.OT_OK, A.OT_WARN_MAXITER)
            f, g = s2.potentials()
    Ckq = Ck.astype(np.float64)
    stt = oracle_lib.plan_stats(Ckq, a, q, f, g, eps)
    lb = oracle_lib.lemma1_lower_bound(Ckq, a)
    assert stt["objective"] >= (stt["row_sums"] * Ckq.min(axis=1)).sum() * (1 - 1e-12)
    assert stt["objective"] <= lb + eps * min(oracle_lib.entropy(a), oracle_lib.entropy(q)) + 1e-4
    # the same decisions as the oracle's argmax over these FP32 costs
    np.testing.assert_array_equal(assoc, oracle_lib.maxsinr_association(1.0 / Cq))


@pytest.mark.parametrize("I,J,seed", [(2000, 16, 6161), (800, 5, 6262)])
def test_adaptive_sinkhorn_against_oracle(A, oracle_lib, I, J, seed):
    announce(f"Adaptive Sinkhorn (Alg. 2), {I} x {J}")
    L = S.make_layout(I, J, 1500.0, hot_spots=1, hot_share=0.5, seed=seed)
    C64, scale = oracle_lib.cost(L)
    C32 = C64.astype(np.float32)
    Cq = C32.astype(np.float64)
    eps, tol, cap = 0.05, 1e-9, 40
    want = oracle_lib.adaptive_sinkhorn(Cq, L.a, eps, tol, 20000, max_outer=cap)
    with A.Solver(I, J) as s:
        st, q, js, r = s.adaptive(*A.matrix_desc(C32, A.OT_COST_DENSE), L.a, eps, tol, 20000, 0.0, cap)
        assert st == A.OT_OK
        loads = s.rrh_loads()
        f, g = s.potentials()
    # the decisions up to the first near tie of the oracle's two largest loads
    hist = want["history"]
    tie = None
    for k in range(min(len(js), len(hist))):
        if js[k] != hist[k][0]:
            qq = np.full(J, L.a.sum() / J)
            for jj, _ in hist[:k]:
                n = qq + r.delta / (J - 1)
                n[jj] = qq[jj] - r.delta
                qq = n
            sol = oracle_lib.sinkhorn(Cq, L.a, qq, eps, tol, 20000)
            ld = np.sort(oracle_lib.rrh_loads(Cq, sol.f, sol.g, eps))
            assert ld[-1] - ld[-2] <= 1e-6 * ld[-1], (k, js[k], hist[k])
            tie = k
            break
    if tie is None:
        assert r.solves == want["solves"] and r.best == want["outer"]
        np.testing.assert_allclose(q, want["q"], rtol=1e-14)
        assert abs(r.max_load - want["max_load"]) <= 1e-6 * want["max_load"]
    assert abs(r.delta - 0.01 * L.a.sum() / J) <= 1e-15
    # the handle holds the returned solve: its loads and potentials
    assert abs(loads.max() - r.max_load) <= 1e-12 * r.max_load
    np.testing.assert_allclose(loads, oracle_lib.rrh_loads(Cq, f, g, eps), rtol=1e-12)
    chk = oracle_lib.plan_stats(Cq, L.a, q, f, g, eps)
    assert chk["marginal_violation"] < tol * 1.05
    assert r.max_load <= r.first_max_load


@pytest.mark.parametrize("I,J,seed,persistent,kind", [(3000, 400, 6363, 1, "dense"), (2500, 600, 6464, 1, "dense"),
                                                       (3000, 400, 6565, 0, "dense"), (20000, 100, 6666, 1, "dense"),
                                                       (3000, 400, 6767, 1, "geometry")])
def test_adaptive_loads_from_the_final_check(A, oracle_lib, I, J, seed, persistent, kind):
    """Alg. 2's RRH loads: at J <= 512 the solves' final exact checks sum
    them beside the marginals (the second case, J = 600, takes a pass of
    their own). The returned loads against the oracle's loads of the handle's
    potentials (1e-12), the reported maximum load equal to their maximum,
    and rho_j = kappa load_j exactly. The chunked path (persistent 0) checks
    through the same kernels; at 20000 rows the check's grid is capped at
    half of the partial rows so that the load partials fit beside them. A
    geometry cost sums its loads from the FP64 functor's costs, against the
    oracle's own FP64 costs."""
    announce(f"Alg. 2 loads from the final check, {kind} {I} x {J}, persistent={persistent}")
    L = S.make_layout(I, J, 3000.0, hot_spots=2, hot_share=0.4, seed=seed)
    C64, scale = oracle_lib.cost(L)
    C32 = C64.astype(np.float32)
    Cq = C32.astype(np.float64) if kind == "dense" else C64
    eps, tol, cap = 0.05, 1e-9, (3 if I < 10000 else 2)
    with A.Solver(I, J, persistent=persistent) as s:
        if kind == "dense":
            desc, a_in = A.matrix_desc(C32, A.OT_COST_DENSE), L.a
        else:  # (Alg. 2 takes positions in device memory)
            import torch
            dev = torch.device("cuda:0")
            xy, rxy = torch.from_numpy(L.dev_xy).to(dev), torch.from_numpy(L.rrh_xy).to(dev)
            desc, a_in = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, scale), torch.from_numpy(L.a).to(dev)
        st, q, js, r = s.adaptive(*desc, a_in, eps, tol, 20000, 0.0, cap)
        assert st == A.OT_OK
        loads = s.rrh_loads()
        f, g = s.potentials()
        kappa = 0.5 / loads.max()
        rho, en, ev = s.evaluate(kappa, 1.0)
    np.testing.assert_allclose(loads, oracle_lib.rrh_loads(Cq, f, g, eps), rtol=1e-12)
    assert loads.max() == r.max_load
    np.testing.assert_array_equal(rho, kappa * loads)
    assert 1 <= r.solves <= cap and (js[:r.solves] >= 0).all() and (js[:r.solves] < J).all()

