"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (targets of the FP32 path: FP32 exponentials feed FP64 sums and
an FP64 polish, so what remains is the stop rule's tol):
* marginal violation of the returned plan < tol (1e-8 / 1e-9 here), both as
  the library reports it and as the oracle recomputes it from the library's
  potentials with its own cost;
* relative error of the transport cost <C, pi> against the oracle run to
  1e-12: <= 1e-6;
* plan L1 distance to the oracle's plan: <= 1e-6 (total mass 1).
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


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    return torch


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def oracle_ref(O, C, a, b, eps):
    r = O.sinkhorn(C, a, b, eps, 1e-12, 20000)
    st = O.plan_stats(C, a, b, r.f, r.g, eps)
    return r, st


# Cell by cell: on every cell that carries mass (pi_ref above 1e-12 of the
# largest entry) the plan of the library's potentials is within 100 tol
# relative of the oracle's plan run to 1e-12, i.e. the gauge-invariant
# f_i + g_j agree to 100 tol eps. The oracle's own tol-run reaches up to 13 tol
# on these instances (a row's relative error is bounded by the residual
# times sum(a) / a_i, far above the typical cell).
ELEM_FACTOR = 100.0


def check_cells(O, C, f, g, ref, eps, tol):
    P = O.plan(C, f, g, eps)
    P0 = O.plan(C, ref.f, ref.g, eps)
    m = P0 > 1e-12 * P0.max()
    rel = np.abs(P - P0)[m] / P0[m]
    assert rel.max() <= ELEM_FACTOR * tol, rel.max()
    dfg = np.abs((f[:, None] + g[None, :]) - (ref.f[:, None] + ref.g[None, :]))[m]
    assert dfg.max() <= ELEM_FACTOR * tol * eps * 1.0001 + 1e-15, dfg.max()
    return np.abs(P - P0).sum()


def check_against(O, C, a, b, eps, tol, f, g, res, ref_stats, ref=None, plan_l1=PLAN_L1):
    chk = O.plan_stats(C, a, b, f, g, eps)
    assert res.marginal_violation < tol, res.marginal_violation
    assert chk["marginal_violation"] < tol * 1.05, chk["marginal_violation"]
    rel = abs(chk["objective"] - ref_stats["objective"]) / abs(ref_stats["objective"])
    assert rel <= OBJ_RTOL, rel
    # the library's own statistics agree with the oracle's recomputation
    assert abs(res.objective - chk["objective"]) <= 1e-9 * abs(chk["objective"])
    assert abs(res.marginal_violation - chk["marginal_violation"]) <= 1e-10 + 1e-6 * chk["marginal_violation"]
    if ref is not None:
        l1 = check_cells(O, C, f, g, ref, eps, tol)
        assert l1 <= plan_l1, l1
    return chk


@pytest.fixture(scope="module")
def small_cfg(oracle_lib):
    L = S.preset_layout("small_1000x50")
    C64, scale = oracle_lib.cost(L)
    C32 = C64.astype(np.float32)
    Cd = C32.astype(np.float64)
    ref, ref_stats = oracle_ref(oracle_lib, Cd, L.a, L.b, 0.05)
    return dict(L=L, C64=C64, C32=C32, Cd=Cd, scale=scale, ref=ref, ref_stats=ref_stats)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_dense_small_workload(A, oracle_lib, small_cfg, precision):
    announce(f"dense 1000x50 eps=0.05 tol=1e-9 precision={precision}")
    L = small_cfg["L"]
    prec = A.OT_PREC_FP32 if precision == "fp32" else A.OT_PREC_FP64
    with A.Solver(L.I, L.J, precision=prec) as s:
        st, res = s.solve_dense(small_cfg["C32"], L.a, L.b, 0.05, 1e-9, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
    check_against(oracle_lib, small_cfg["Cd"], L.a, L.b, 0.05, 1e-9, f, g, res, small_cfg["ref_stats"], small_cfg["ref"])
    # iteration count near the oracle's at the same tol (reading: +-2 plus the polish)
    r = oracle_lib.sinkhorn(small_cfg["Cd"], L.a, L.b, 0.05, 1e-9, 2000)
    assert abs(res.iterations - r.iters) <= 4


def test_dense_device_tensors_and_plan(A, oracle_lib, small_cfg, torch_mod):
    announce("dense 1000x50 device tensors + plan fp32/fp64")
    torch = torch_mod
    L = small_cfg["L"]
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(small_cfg["C32"]).to(dev)
    a = torch.from_numpy(L.a).to(dev)
    b = torch.from_numpy(L.b).to(dev)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(Cd, a, b, 0.05, 1e-9, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
        P64 = s.plan(torch.empty((L.I, L.J), dtype=torch.float64, device=dev)).cpu().numpy()
        P32 = s.plan(np.empty((L.I, L.J), dtype=np.float32))
    check_against(oracle_lib, small_cfg["Cd"], L.a, L.b, 0.05, 1e-9, f, g, res, small_cfg["ref_stats"], small_cfg["ref"])
    expect = oracle_lib.plan(small_cfg["Cd"], f, g, 0.05)
    np.testing.assert_allclose(P64, expect, rtol=1e-12, atol=1e-300)
    np.testing.assert_allclose(P32, expect.astype(np.float32), rtol=2e-7, atol=1e-44)
    assert np.abs(P64 - oracle_lib.plan(small_cfg["Cd"], small_cfg["ref"].f, small_cfg["ref"].g, 0.05)).sum() <= PLAN_L1


@pytest.mark.parametrize("I,J", [(1, 7), (9, 1), (37, 5), (129, 67), (513, 130), (1000, 256), (3001, 400), (777, 1031)])
def test_dense_ragged_shapes(A, oracle_lib, I, J):
    announce(f"dense random {I}x{J}")
    rng = np.random.default_rng(1000 * I + J)
    C = rng.uniform(0.0, 1.0, size=(I, J)).astype(np.float32)
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = rng.uniform(0.5, 1.5, J)
    b = b / b.sum() * a.sum()
    Cd = C.astype(np.float64)
    eps, tol = 0.05, 1e-8
    ref, ref_stats = oracle_ref(oracle_lib, Cd, a, b, eps)
    with A.Solver(I, J) as s:
        st, res = s.solve_dense(C, a, b, eps, tol, 5000)
        assert st == A.OT_OK
        f, g = s.potentials()
    check_against(oracle_lib, Cd, a, b, eps, tol, f, g, res, ref_stats, ref)


@pytest.mark.parametrize("blocks,waves,lanes,I,J", [(5, 4, 16, 1000, 52), (37, 8, 32, 3001, 400), (64, 8, 64, 2500, 1031),
                                                   (3, 8, 0, 700, 2048), (11, 4, 16, 999, 17), (7, 8, 32, 513, 300)])
def test_dense_launch_shapes(A, oracle_lib, blocks, waves, lanes, I, J):
    # few workgroups: many rows per wave, so the row slots refill across batches
    announce(f"dense random {I}x{J} with {blocks} workgroups x {waves} waves, {lanes} lanes per row")
    rng = np.random.default_rng(7 * I + J)
    C = rng.uniform(0.0, 2.0, size=(I, J)).astype(np.float32)
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = np.full(J, a.sum() / J)
    Cd = C.astype(np.float64)
    eps, tol = 0.08, 1e-8
    ref, ref_stats = oracle_ref(oracle_lib, Cd, a, b, eps)
    with A.Solver(I, J, sweep_blocks=blocks, sweep_waves=waves, sweep_lanes=lanes) as s:
        st, res = s.solve_dense(C, a, b, eps, tol, 5000)
        assert st == A.OT_OK
        f, g = s.potentials()
    check_against(oracle_lib, Cd, a, b, eps, tol, f, g, res, ref_stats, ref)


def test_dense_fp64_matrix(A, oracle_lib, small_cfg):
    announce("dense 1000x50 float64 matrix")
    L = small_cfg["L"]
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(small_cfg["C64"], L.a, L.b, 0.05, 1e-9, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
    ref, ref_stats = oracle_ref(oracle_lib, small_cfg["C64"], L.a, L.b, 0.05)
    check_against(oracle_lib, small_cfg["C64"], L.a, L.b, 0.05, 1e-9, f, g, res, ref_stats, ref)


def test_rates_matrix(A, oracle_lib, small_cfg):
    announce("rates 1000x50 float64, oracle scale")
    L = small_cfg["L"]
    R = oracle_lib.rates(L)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_rates(R, small_cfg["scale"], L.a, L.b, 0.05, 1e-9, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
    ref, ref_stats = oracle_ref(oracle_lib, small_cfg["C64"], L.a, L.b, 0.05)
    check_against(oracle_lib, small_cfg["C64"], L.a, L.b, 0.05, 1e-9, f, g, res, ref_stats, ref)


def test_geometry_cost_functor_median_and_solve(A, oracle_lib, small_cfg, torch_mod):
    announce("geometry 1000x50: materialised cost, median, on-the-fly solve")
    torch = torch_mod
    L = small_cfg["L"]
    dev = torch.device("cuda:0")
    with A.Solver(L.I, L.J) as s:
        d, keep = A.geometry_desc(L.dev_xy, L.rrh_xy, L.radio, L.shadow_key, small_cfg["scale"])
        med = s.cost_median(d)
        # the FP32 median of 1/R against the oracle's FP64 median
        assert abs(med - small_cfg["scale"]) <= 2e-6 * small_cfg["scale"], (med, small_cfg["scale"])
        Cdev = torch.empty((L.I, L.J), dtype=torch.float32, device=dev)
        s.materialize_cost(d, Cdev)
        Cm = Cdev.cpu().numpy().astype(np.float64)
        # FP64 functor rounded once to FP32
        rel = np.abs(Cm - small_cfg["C64"]) / small_cfg["C64"]
        assert rel.max() <= 2.0 ** -23, rel.max()
        st, res = s.solve_geometry(L.dev_xy, L.rrh_xy, L.radio, L.shadow_key, small_cfg["scale"], L.a, L.b, 0.05,
                                   1e-9, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
    ref, ref_stats = oracle_ref(oracle_lib, small_cfg["C64"], L.a, L.b, 0.05)
    check_against(oracle_lib, small_cfg["C64"], L.a, L.b, 0.05, 1e-9, f, g, res, ref_stats, ref)


def test_invalid_inputs_rejected(A, small_cfg):
    announce("validation errors")
    L = small_cfg["L"]
    C = small_cfg["C32"].copy()
    with A.Solver(L.I, L.J) as s:
        def status(C=C, a=L.a, b=L.b, eps=0.05, max_iter=100):
            try:
                return s.solve_dense(C, a, b, eps, 1e-6, max_iter)[0]
            except A.OTError as e:
                return e.status
        Cn = C.copy()
        Cn[5, 7] = np.nan
        assert status(C=Cn) == A.OT_EINVAL
        Ci = C.copy()
        Ci[0, 0] = np.inf
        assert status(C=Ci) == A.OT_EINVAL
        a0 = L.a.copy()
        a0[3] = 0.0
        assert status(a=a0) == A.OT_EINVAL
        assert status(a=L.a * 2) == A.OT_EINVAL
        assert status(eps=0.0) == A.OT_EINVAL
        assert status(eps=np.nan) == A.OT_EINVAL
        assert status(max_iter=0) == A.OT_EINVAL
        big = np.zeros((L.I + 1, L.J), dtype=np.float32)
        assert status(C=big, a=np.full(L.I + 1, 1.0 / (L.I + 1))) == A.OT_EINVAL
        # plan before a successful solve
        with pytest.raises(A.OTError) as e:
            s.plan()
        assert e.value.status == A.OT_ESTATE
        # after the failures the handle still solves
        st, res = s.solve_dense(C, L.a, L.b, 0.05, 1e-8, 2000)
        assert st == A.OT_OK and res.marginal_violation < 1e-8


def test_max_iter_warning(A, small_cfg):
    announce("max_iter warning")
    L = small_cfg["L"]
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(small_cfg["C32"], L.a, L.b, 0.05, 1e-12, 3)
        assert st == A.OT_WARN_MAXITER
        assert res.iterations == 3 and res.marginal_violation > 1e-12
        s.plan()  # the result is valid


def test_warm_start_and_determinism(A, oracle_lib, small_cfg):
    announce("warm start, bitwise determinism")
    L = small_cfg["L"]
    with A.Solver(L.I, L.J) as s:
        st, r1 = s.solve_dense(small_cfg["C32"], L.a, L.b, 0.05, 1e-9, 2000)
        f1, g1 = s.potentials()
        st, r2 = s.solve_dense(small_cfg["C32"], L.a, L.b, 0.05, 1e-9, 2000)
        f2, g2 = s.potentials()
        assert np.array_equal(f1, f2) and np.array_equal(g1, g2)
        assert r1.iterations == r2.iterations
        st, r3 = s.solve_dense(small_cfg["C32"], L.a, L.b, 0.05, 1e-9, 2000, warm_start=True)
        # from a converged start the FP32 sweeps only walk to their noise
        # floor (a few iterations) before the FP64 polish
        assert st == A.OT_OK and r3.iterations <= max(6, r1.iterations // 4)
        f3, g3 = s.potentials()
    check_against(oracle_lib, small_cfg["Cd"], L.a, L.b, 0.05, 1e-9, f3, g3, r3, small_cfg["ref_stats"], small_cfg["ref"])


def test_closed_forms(A):
    announce("closed forms: constant cost, J=1, I=1")
    rng = np.random.default_rng(3)
    I, J = 300, 40
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = rng.uniform(0.5, 1.5, J)
    b = b / b.sum() * a.sum()
    with A.Solver(I, J) as s:
        st, res = s.solve_dense(np.full((I, J), 0.7, dtype=np.float32), a, b, 0.03, 1e-12, 50)
        P = s.plan()
        np.testing.assert_allclose(P, np.outer(a, b) / a.sum(), rtol=1e-12)
        st, res = s.solve_dense(rng.uniform(size=(I, 1)).astype(np.float32), a, np.array([a.sum()]), 0.03, 1e-12, 50)
        np.testing.assert_allclose(s.plan().ravel(), a, rtol=1e-13)
        st, res = s.solve_dense(rng.uniform(size=(1, J)).astype(np.float32), np.array([b.sum()]), b, 0.03, 1e-12, 50)
        np.testing.assert_allclose(s.plan().ravel(), b, rtol=1e-13)


@pytest.fixture(scope="module")
def cran_cfg(oracle_lib):
    L = S.preset_layout("cran_20000x400")
    C64, scale = oracle_lib.cost(L)
    return dict(L=L, C64=C64, scale=scale, refs={})


@pytest.mark.parametrize("eps", [0.1, 0.02, 0.005])
def test_cran_20000x400_dense_and_geometry(A, oracle_lib, cran_cfg, eps, torch_mod):
    announce(f"20000x400 eps={eps}: dense fp32 matrix and on-the-fly geometry")
    torch = torch_mod
    L, C64 = cran_cfg["L"], cran_cfg["C64"]
    C32 = C64.astype(np.float32)
    Cd = C32.astype(np.float64)
    dev = torch.device("cuda:0")
    a, b = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(torch.from_numpy(C32).to(dev), a, b, eps, 1e-8, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
        ref, ref_stats = oracle_ref(oracle_lib, Cd, L.a, L.b, eps)
        check_against(oracle_lib, Cd, L.a, L.b, eps, 1e-8, f, g, res, ref_stats, ref)
        xy, rxy = torch.from_numpy(L.dev_xy).to(dev), torch.from_numpy(L.rrh_xy).to(dev)
        st, res = s.solve_geometry(xy, rxy, L.radio, L.shadow_key, cran_cfg["scale"], a, b, eps, 1e-8, 2000)
        assert st == A.OT_OK
        f, g = s.potentials()
    ref, ref_stats = oracle_ref(oracle_lib, C64, L.a, L.b, eps)
    check_against(oracle_lib, C64, L.a, L.b, eps, 1e-8, f, g, res, ref_stats, ref)


@pytest.mark.parametrize("where", ["host", "device"])
def test_dense_row_padded_matrix(A, oracle_lib, torch_mod, where):
    announce(f"row-padded FP32 matrix (ld = J + 5, NaN padding) in {where} memory")
    L = S.make_layout(1500, 130, 1000.0, seed=77)
    C64, _ = oracle_lib.cost(L)
    C32 = C64.astype(np.float32)
    I, J = C32.shape
    for ld in (J + 2, J + 6):  # ld % 4 == 0 (vector loads) and not
        buf = np.full((I, ld), np.nan, np.float32)
        buf[:, :J] = C32
        M = buf if where == "host" else torch_mod.from_numpy(buf).to("cuda:0")
        a = L.a if where == "host" else torch_mod.from_numpy(L.a).to("cuda:0")
        b = L.b if where == "host" else torch_mod.from_numpy(L.b).to("cuda:0")
        d, keep = A.matrix_desc(M, A.OT_COST_DENSE, J=J)
        with A.Solver(I, J) as s:
            st, res = s.solve(d, keep, a, b, 0.05, 1e-9, 2000)
            assert st == A.OT_OK
            f, g = s.potentials()
            P = s.plan()
        Cq = C32.astype(np.float64)
        ref, ref_stats = oracle_ref(oracle_lib, Cq, L.a, L.b, 0.05)
        check_against(oracle_lib, Cq, L.a, L.b, 0.05, 1e-9, f, g, res, ref_stats, ref)
        assert np.allclose(P, oracle_lib.plan(Cq, f, g, 0.05), rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("kind,I,J,persistent,tol", [
    ("dense", 1000, 50, 1, 1e-9), ("dense", 1000, 50, 0, 1e-11), ("dense", 777, 1031, 1, 1e-8),
    ("geometry", 2000, 120, 1, 1e-9), ("geometry", 1500, 600, 0, 1e-8), ("euclid", 1800, 90, 1, 1e-9)])
def test_plan_written_by_the_final_check(A, oracle_lib, torch_mod, kind, I, J, persistent, tol):
    """A plan asked for before the solve (ot_assoc_set_plan_output) is written
    by the final exact check from the cells it computes: against the plan
    pass over the same potentials (FP64 within a few ulps of its FP64
    exponentials, FP32 equal up to one ulp) and against the oracle's plan of
    those potentials (1e-12; for costs regenerated from positions, geometry
    and distance, on the entries above 1e-12 of the largest, as the two
    sides' FP64 costs differ by ulps that an exponent of a few hundred
    amplifies in the tiny ones). tol 1e-11 makes the check
    miss on the FP32 path and run the FP64 phase and a second check, whose
    plan must be the one left. A buffer smaller than I x J is not written."""
    torch = torch_mod
    announce(f"plan from the final check, {kind} {I}x{J}, persistent={persistent}, tol={tol}")
    dev = torch.device("cuda:0")
    eps = 0.05
    L = S.make_layout(I, J, 2000.0, hot_spots=2, hot_share=0.4, seed=7100 + I + J)
    a = torch.from_numpy(L.a).to(dev)
    b = torch.from_numpy(L.b).to(dev)
    with A.Solver(I, J, persistent=persistent) as s:
        if kind == "dense":
            C64, _ = oracle_lib.cost(L)
            C32 = C64.astype(np.float32)
            Cq = C32.astype(np.float64)
            Cd = torch.from_numpy(C32).to(dev)
            solve = lambda: s.solve_dense(Cd, a, b, eps, tol, 20000)
        elif kind == "euclid":
            xy = torch.from_numpy(L.dev_xy).to(dev)
            rxy = torch.from_numpy(L.rrh_xy).to(dev)
            Cq, scale = oracle_lib.distance_cost(L, 0.0)
            solve = lambda: s.solve_euclid(xy, rxy, scale, a, b, eps, tol, 20000)
        else:
            xy = torch.from_numpy(L.dev_xy).to(dev)
            rxy = torch.from_numpy(L.rrh_xy).to(dev)
            d, keep = A.geometry_desc(xy, rxy, L.radio, L.shadow_key, 1.0)
            scale = s.cost_median(d)
            Cq, _ = oracle_lib.cost(L, scale=scale)
            solve = lambda: s.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, a, b, eps, tol, 20000)
        for dt in (torch.float64, torch.float32):
            fused = torch.full((I, J), float("nan"), dtype=dt, device=dev)
            s.set_plan_output(fused)
            st, res = solve()
            assert st == A.OT_OK
            back = s.plan(fused)  # returns at once: written by the check
            assert back is fused
            s.set_plan_output(None)
            sep = s.plan(torch.empty((I, J), dtype=dt, device=dev))
            P, Q = fused.cpu().numpy(), sep.cpu().numpy()
            assert np.isfinite(P).all()
            if dt == torch.float64:
                np.testing.assert_allclose(P, Q, rtol=4e-15, atol=1e-300)
                f, g = s.potentials()
                R = oracle_lib.plan(Cq, f, g, eps)
                # (costs regenerated from positions: the two sides' FP64 costs
                # differ by ulps, which an exponent of a few hundred carries
                # into the tiny entries; the entries that carry mass are held
                # to 1e-12)
                m = R > 1e-12 * R.max() if kind != "dense" else np.ones(R.shape, bool)
                np.testing.assert_allclose(P[m], R[m], rtol=1e-12, atol=1e-300)
            else:
                assert (np.abs(P - Q) <= np.spacing(np.maximum(np.abs(P), np.abs(Q))) * 1.0 + 1e-45).all()
        # a buffer too small for I x J is left alone
        small = torch.full((I * J - 1,), float("nan"), dtype=torch.float32, device=dev)
        s.set_plan_output(small)
        st, res = solve()
        assert st == A.OT_OK and bool(torch.isnan(small).all())
        s.set_plan_output(None)
