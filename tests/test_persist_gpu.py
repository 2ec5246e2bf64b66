"""GPU tests of the cooperative FP32 phase (ot_assoc_options.persistent): one
launch that keeps the instance's FP32 cost in LDS and exchanges the column
partials and the new g between workgroups through polled exchange slots
(agent-scope atomic loads and stores).

Every case is solved with the cooperative launch and with the chunked graph
launches, and both are held to the same bar against the FP64 oracle as the
other parity tests (marginal violation < tol as reported and as recomputed by
the oracle; transport cost within 1e-6 relative of the oracle's converged
solution; plan L1 distance <= 1e-6). The result flag says which path ran;
the LDS capacity boundary is tested on both sides.
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


# cell by cell: the plan of the library's potentials within 100 tol relative
# of the oracle's (1e-12) plan on every cell with mass, i.e. f_i + g_j within
# 100 tol eps (the oracle's own tol-run reaches up to 13 tol on such instances)
ELEM_FACTOR = 100.0


def check(O, C, a, b, eps, tol, f, g, res, ref):
    chk = O.plan_stats(C, a, b, f, g, eps)
    rst = O.plan_stats(C, a, b, ref.f, ref.g, eps)
    assert res.marginal_violation < tol, res.marginal_violation
    assert chk["marginal_violation"] < tol * 1.05, chk["marginal_violation"]
    assert abs(chk["objective"] - rst["objective"]) <= OBJ_RTOL * abs(rst["objective"])
    assert abs(res.objective - chk["objective"]) <= 1e-9 * abs(chk["objective"])
    P, P0 = O.plan(C, f, g, eps), O.plan(C, ref.f, ref.g, eps)
    l1 = np.abs(P - P0).sum()
    assert l1 <= PLAN_L1, l1
    m = P0 > 1e-12 * P0.max()
    assert (np.abs(P - P0)[m] / P0[m]).max() <= ELEM_FACTOR * tol
    dfg = np.abs((f[:, None] + g[None, :]) - (ref.f[:, None] + ref.g[None, :]))[m]
    assert dfg.max() <= ELEM_FACTOR * tol * eps * 1.0001 + 1e-15, dfg.max()


def random_case(I, J, seed):
    rng = np.random.default_rng(seed)
    C = rng.uniform(0.0, 1.0, size=(I, J)).astype(np.float32)
    a = rng.uniform(0.5, 1.5, I)
    a /= a.sum()
    b = rng.uniform(0.5, 1.5, J)
    b = b / b.sum() * a.sum()
    return C, a, b


def solve_both(A, I, J, fn):
    out = {}
    for pers in (1, 0):
        with A.Solver(I, J, persistent=pers) as s:
            st, res = fn(s)
            f, g = s.potentials()
            out[pers] = (st, res, f, g)
    return out


@pytest.mark.parametrize("I,J", [(1, 1), (2, 3), (50, 7), (1000, 50), (4097, 130), (6000, 400), (1200, 512), (1200, 516),
                                 (3000, 513), (900, 2048)])
def test_dense_both_paths(A, oracle_lib, I, J):
    # (512 and 516 columns sit on either side of the width at which the exact
    # check changes from its narrow kernel instantiation to its wide one)
    announce(f"dense random {I}x{J}, cooperative and chunked")
    C, a, b = random_case(I, J, 77 * I + J)
    Cd = C.astype(np.float64)
    eps, tol = 0.05, 1e-8
    ref = oracle_lib.sinkhorn(Cd, a, b, eps, 1e-12, 20000)
    out = solve_both(A, I, J, lambda s: s.solve_dense(C, a, b, eps, tol, 2000))
    for pers, (st, res, f, g) in out.items():
        assert st == A.OT_OK, (pers, st)
        assert bool(res.flags & A.OT_RESULT_PERSISTENT) == bool(pers), (pers, res.flags)
        check(oracle_lib, Cd, a, b, eps, tol, f, g, res, ref)
    # the two paths run the same iteration with different summation orders
    # and row shifts; the FP32 phase ends at the first stall (a residual
    # below 1e-7 that is not 5 % below the least of the last four), which
    # each path reaches within the few iterations after its residual enters
    # the FP32 noise band: the two stops can differ by that band's width on
    # either side (observed up to 5 on the 50 x 7 case)
    print(f"[case] iterations: cooperative {out[1][1].iterations} ({out[1][1].fp64_iterations} FP64), "
          f"chunked {out[0][1].iterations} ({out[0][1].fp64_iterations} FP64)", flush=True)
    assert abs(out[1][1].iterations - out[0][1].iterations) <= 8


def test_lds_capacity_boundary(A):
    """20480 x 400 is the largest FP32 instance of 400 RRHs whose rows fit in
    the LDS of 256 CUs (80 rows of 1600 bytes per workgroup); one more device
    needs 96-row blocks, which do not fit, and the solve falls back to the
    chunked launches."""
    announce("LDS capacity boundary at J=400")
    import torch
    props = torch.cuda.get_device_properties(0)
    if props.multi_processor_count != 256:
        pytest.skip("boundary computed for 256 CUs")
    for I, expect in ((20480, 1), (20481, 0)):
        C, a, b = random_case(I, 400, I)
        with A.Solver(I, 400) as s:
            st, res = s.solve_dense(C, a, b, 0.05, 1e-8, 2000)
            assert st == A.OT_OK and res.marginal_violation < 1e-8
            assert (res.flags & A.OT_RESULT_PERSISTENT) == expect, (I, res.flags)


def test_cran_20000x400_cooperative(A, oracle_lib):
    announce("cran_20000x400 dense, cooperative path against the oracle")
    L = S.preset_layout("cran_20000x400")
    C64, scale = oracle_lib.cost(L)
    C32 = C64.astype(np.float32)
    Cd = C32.astype(np.float64)
    eps, tol = 0.02, 1e-8
    ref = oracle_lib.sinkhorn(Cd, L.a, L.b, eps, 1e-11, 20000)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(C32, L.a, L.b, eps, tol, 2000)
        assert st == A.OT_OK and res.flags & A.OT_RESULT_PERSISTENT
        f, g = s.potentials()
    check(oracle_lib, Cd, L.a, L.b, eps, tol, f, g, res, ref)


def test_geometry_and_rates_both_paths(A, oracle_lib):
    announce("geometry 3000x150 and FP32 rates, cooperative and chunked")
    L = S.make_layout(3000, 150, 2000.0, hot_spots=2, hot_share=0.4, seed=5150)
    C64, scale = oracle_lib.cost(L)
    eps, tol = 0.05, 1e-8
    ref = oracle_lib.sinkhorn(C64, L.a, L.b, eps, 1e-12, 20000)
    out = solve_both(A, L.I, L.J, lambda s: s.solve_geometry(L.dev_xy, L.rrh_xy, L.radio, L.shadow_key, scale,
                                                              L.a, L.b, eps, tol, 2000))
    for pers, (st, res, f, g) in out.items():
        assert st == A.OT_OK
        assert bool(res.flags & A.OT_RESULT_PERSISTENT) == bool(pers)
        check(oracle_lib, C64, L.a, L.b, eps, tol, f, g, res, ref)
    # rates: C = (1 / R) / scale with R given in FP32
    R = (1.0 / (C64 * scale)).astype(np.float32)
    Cr = (1.0 / R.astype(np.float64)) / scale
    ref_r = oracle_lib.sinkhorn(Cr, L.a, L.b, eps, 1e-12, 20000)
    out = solve_both(A, L.I, L.J, lambda s: s.solve_rates(R, scale, L.a, L.b, eps, tol, 2000))
    for pers, (st, res, f, g) in out.items():
        assert st == A.OT_OK
        assert bool(res.flags & A.OT_RESULT_PERSISTENT) == bool(pers)
        check(oracle_lib, Cr, L.a, L.b, eps, tol, f, g, res, ref_r)


def test_fp64_costs_take_the_chunked_path(A, oracle_lib):
    announce("FP64 dense cost: no cooperative launch")
    C, a, b = random_case(2000, 60, 9)
    Cd = C.astype(np.float64) + 1e-3 * np.arange(60)[None, :]
    ref = oracle_lib.sinkhorn(Cd, a, b, 0.05, 1e-12, 20000)
    with A.Solver(2000, 60) as s:
        st, res = s.solve_dense(Cd, a, b, 0.05, 1e-8, 2000)
        assert st == A.OT_OK and not (res.flags & A.OT_RESULT_PERSISTENT)
        f, g = s.potentials()
    check(oracle_lib, Cd, a, b, 0.05, 1e-8, f, g, res, ref)


def test_cooperative_max_iter_warm_start_and_determinism(A, oracle_lib):
    announce("cooperative path: max_iter stop, warm start, bitwise determinism")
    C, a, b = random_case(5000, 200, 21)
    Cd = C.astype(np.float64)
    eps = 0.05
    with A.Solver(5000, 200) as s:
        st, res = s.solve_dense(C, a, b, eps, 1e-12, 3)
        assert st == A.OT_WARN_MAXITER and res.iterations == 3 and res.flags & A.OT_RESULT_PERSISTENT
        st, r1 = s.solve_dense(C, a, b, eps, 1e-9, 2000)
        f1, g1 = s.potentials()
        st, r2 = s.solve_dense(C, a, b, eps, 1e-9, 2000)
        f2, g2 = s.potentials()
        assert np.array_equal(f1, f2) and np.array_equal(g1, g2) and r1.iterations == r2.iterations
        st, r3 = s.solve_dense(C, a, b, eps, 1e-9, 2000, warm_start=True)
        assert st == A.OT_OK and r3.iterations <= max(6, r1.iterations // 4)
        assert r3.flags & A.OT_RESULT_PERSISTENT
        f3, g3 = s.potentials()
    ref = oracle_lib.sinkhorn(Cd, a, b, eps, 1e-12, 20000)
    check(oracle_lib, Cd, a, b, eps, 1e-9, f3, g3, r3, ref)


def test_cooperative_rejects_bad_inputs(A):
    announce("cooperative path: inputs rejected on the device")
    C, a, b = random_case(3000, 100, 4)
    with A.Solver(3000, 100) as s:
        bad = C.copy()
        bad[1234, 56] = np.nan
        with pytest.raises(A.OTError) as e:
            s.solve_dense(bad, a, b, 0.05, 1e-8, 100)
        assert e.value.status == A.OT_EINVAL and "non-finite" in str(e.value)
        a2 = a.copy()
        a2[7] = -a2[7]
        with pytest.raises(A.OTError) as e:
            s.solve_dense(C, a2, b, 0.05, 1e-8, 100)
        assert e.value.status == A.OT_EINVAL and "marginal a" in str(e.value)
        with pytest.raises(A.OTError) as e:
            s.solve_dense(C, a, b * 1.5, 0.05, 1e-8, 100)
        assert e.value.status == A.OT_EINVAL and "unbalanced" in str(e.value)
        st, res = s.solve_dense(C, a, b, 0.05, 1e-8, 2000)
        assert st == A.OT_OK and res.flags & A.OT_RESULT_PERSISTENT


@pytest.mark.parametrize("offset", [20.0, -20.0])
def test_row_shift_far_from_the_row_sums(A, oracle_lib, offset):
    """Warm start from potentials f = offset (far from the solution): the row
    shift recovered from the previous iterate (log2(e) ln a_i - kk f_i) then
    puts every row sum far outside [2^-100, 2^100], and both the cooperative
    and the streaming sweeps must redo those rows with the row maximum and
    converge to the oracle's solution as from a cold start."""
    announce(f"warm start from f = {offset:+g}: row shifts far off, both paths")
    C, a, b = random_case(2000, 100, 9191)
    Cd = C.astype(np.float64)
    eps, tol = 0.05, 1e-8
    ref = oracle_lib.sinkhorn(Cd, a, b, eps, 1e-12, 20000)

    def warm(s):
        s.set_potentials(np.full(2000, offset), np.zeros(100))
        return s.solve_dense(C, a, b, eps, tol, 3000, warm_start=True)

    out = solve_both(A, 2000, 100, warm)
    for pers, (st, res, f, g) in out.items():
        assert st == A.OT_OK, (pers, st)
        assert bool(res.flags & A.OT_RESULT_PERSISTENT) == bool(pers)
        check(oracle_lib, Cd, a, b, eps, tol, f, g, res, ref)


@pytest.mark.parametrize("I,J,seed", [(997, 37, 9301), (1501, 150, 9302), (2003, 300, 9303), (3001, 400, 9304)])
def test_streaming_geometry_rows_past_the_range(A, oracle_lib, I, J, seed):
    """Geometry costs on the streaming path with row counts that leave rows
    of the last wave step past the range: those lanes re-read the job's last
    row (its positions, interference sums and index alike), so every term
    stays finite and the solve matches the oracle."""
    announce(f"geometry {I}x{J} on the streaming path, ragged last step")
    L = S.make_layout(I, J, 1500.0, hot_spots=2, hot_share=0.4, seed=seed)
    C64, scale = oracle_lib.cost(L)
    eps, tol = 0.05, 1e-8
    ref = oracle_lib.sinkhorn(C64, L.a, L.b, eps, 1e-12, 20000)
    with A.Solver(I, J, persistent=0) as s:
        st, res = s.solve_geometry(L.dev_xy, L.rrh_xy, L.radio, L.shadow_key, scale, L.a, L.b, eps, tol, 3000)
        assert st == A.OT_OK
        assert not (res.flags & A.OT_RESULT_PERSISTENT)
        f, g = s.potentials()
    check(oracle_lib, C64, L.a, L.b, eps, tol, f, g, res, ref)


def test_cooperative_wait_gives_up_and_recovers(A):
    """The bounded waits of the cooperative FP32 phase, forced from the host:
    the launch withholds g at its third iteration, every later wait gives up,
    all workgroups leave the kernel normally and the solve returns OT_EDEVICE;
    the next solve on the same handle runs as usual, bitwise as on a fresh
    handle."""
    import time
    announce("cooperative phase: withheld exchange at iteration 3 -> give-up, then recovery")
    C, a, b = random_case(20000, 400, 77)
    eps, tol = 0.05, 1e-8
    with A.Solver(20000, 400) as s:
        assert A.ot_assoc_test_hold_exchange(3) == A.OT_OK
        t0 = time.perf_counter()
        with pytest.raises(A.OTError) as e:
            s.solve_dense(C, a, b, eps, tol, 2000)
        dt = time.perf_counter() - t0
        print(f"[case] gave up after {dt * 1e3:.1f} ms: {e.value}", flush=True)
        assert e.value.status == A.OT_EDEVICE
        assert "gave up" in str(e.value)
        assert dt < 5.0
        st, res = s.solve_dense(C, a, b, eps, tol, 2000)
        assert st == A.OT_OK and res.flags & A.OT_RESULT_PERSISTENT
        f, g = s.potentials()
    with A.Solver(20000, 400) as s:
        st0, res0 = s.solve_dense(C, a, b, eps, tol, 2000)
        f0, g0 = s.potentials()
    assert res.iterations == res0.iterations
    np.testing.assert_array_equal(f, f0)
    np.testing.assert_array_equal(g, g0)
    assert A.ot_assoc_test_hold_exchange(-1) == A.OT_EINVAL


@pytest.mark.parametrize("I,J", [(1000, 50), (4097, 130), (6000, 400)])
def test_iteration_counts_against_oracle(A, oracle_lib, I, J):
    """Iteration counts near tol, anchored on the oracle run to the same tol
    with the same stop rule: the all-FP64 path within 2 iterations of it; the
    FP32 paths (cooperative and chunked) no earlier than 2 before it and at
    most 8 after it: their FP32 phase stops at the first stall once the FP32
    residual is in its noise band (r < 1e-7 and not 5 % below the least of
    the last four), which can lie a few iterations past the iterate where the
    FP64 residual would have met tol, before the FP64 polish and check."""
    announce(f"iteration counts against the oracle at tol, {I}x{J}")
    C, a, b = random_case(I, J, 991 * I + J)
    Cd = C.astype(np.float64)
    eps, tol = 0.05, 1e-8
    ref = oracle_lib.sinkhorn(Cd, a, b, eps, tol, 20000)
    with A.Solver(I, J, precision=A.OT_PREC_FP64) as s:
        st, r64 = s.solve_dense(C, a, b, eps, tol, 2000)
        assert st == A.OT_OK
    out = solve_both(A, I, J, lambda s: s.solve_dense(C, a, b, eps, tol, 2000))
    k32 = {p: out[p][1].iterations for p in out}
    print(f"[case] oracle {ref.iters}, FP64 path {r64.iterations}, FP32 cooperative {k32[1]}, chunked {k32[0]}",
          flush=True)
    assert abs(r64.iterations - ref.iters) <= 2
    for p in (1, 0):
        assert ref.iters - 2 <= k32[p] <= ref.iters + 8, (p, k32[p], ref.iters)


@pytest.mark.parametrize("pers", [1, 0])
def test_reported_device_time_covers_the_solve(A, pers):
    """The result's device time runs from the solve's first launch to its last
    control-block copy: positive, within the call's wall-clock time, and (on
    the cooperative path) at least the cooperative launch it contains; the
    same on a second solve of the handle, when the exchange block is zeroed by
    the init launch again."""
    import time

    import torch
    announce(f"device time of a 4000 x 130 solve, persistent={pers}")
    C, a, b = random_case(4000, 130, 4130)
    dev = torch.device("cuda:0")
    Cd, ad, bd = (torch.from_numpy(x).to(dev) for x in (C, a, b))
    with A.Solver(4000, 130, persistent=pers) as s:
        for rep in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st, res = s.solve_dense(Cd, ad, bd, 0.05, 1e-8, 2000)
            wall = time.perf_counter() - t0
            assert st == A.OT_OK
            assert bool(res.flags & A.OT_RESULT_PERSISTENT) == bool(pers)
            assert 0.0 < res.seconds <= wall, (rep, res.seconds, wall)
            if pers:
                ms, it = s.fast_phase_time()
                assert 0.0 < ms * 1e-3 <= res.seconds and it >= 1, (rep, ms, res.seconds)
            if rep == 0:
                f0, g0 = s.potentials()
            else:
                f1, g1 = s.potentials()
                assert np.array_equal(f0, f1) and np.array_equal(g0, g1)
