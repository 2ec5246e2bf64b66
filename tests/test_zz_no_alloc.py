"""GPU test of the no-allocation entry point ot_assoc_solve_static (for
callers that cannot allocate device memory): through the C ABI, against the
handle-based ot_assoc_solve on the same inputs (the same kernels and launch
shapes, so the potentials must agree bitwise), on two calls in a row, the
second with a smaller (ragged) instance; the array it keeps its buffers in
is shared between the calls. No device allocation may happen in either
call. Sizes beyond its stated maximum are rejected."""

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


def _instance(oracle_lib, name=None, I=None, J=None, seed=0):
    L = S.preset_layout(name) if name else S.make_layout(I, J, 1000.0, seed=seed)
    C, _ = oracle_lib.cost(L)
    return L, C.astype(np.float32)


def _handle_solve(A, torch, C, L, eps, tol):
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(C).to(dev)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_dense(Cd, torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev), eps, tol, 2000)
        f, g = s.potentials()
    return st, res, f, g


def _static_solve(A, torch, C, L, eps, tol, ld=None):
    dev = torch.device("cuda:0")
    if ld is None:
        Cd = torch.from_numpy(C).to(dev)
    else:  # a padded row stride
        Cd = torch.full((L.I, ld), float("inf"), dtype=torch.float32, device=dev)
        Cd[:, :L.J] = torch.from_numpy(C).to(dev)
    a, b = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    f = torch.empty(L.I, dtype=torch.float64, device=dev)
    g = torch.empty(L.J, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    n0 = A.ot_assoc_device_allocations()
    st, res = A.ot_assoc_solve_static(Cd, a, b, f, g, eps, tol, 2000, J=L.J)
    n1 = A.ot_assoc_device_allocations()
    return st, res, f.cpu().numpy(), g.cpu().numpy(), n1 - n0


def test_static_solve_matches_handle_solve_twice(A, oracle_lib):
    import torch

    eps, tol = 0.02, 1e-8
    L1, C1 = _instance(oracle_lib, "cran_20000x400")
    L2, C2 = _instance(oracle_lib, I=3001, J=257, seed=77)
    # the handle path first (it allocates), then two static calls in a row
    ref1 = _handle_solve(A, torch, C1, L1, eps, tol)
    ref2 = _handle_solve(A, torch, C2, L2, 0.05, tol)
    print("\n[case] static solve 20000x400 eps 0.02, then 3001x257 eps 0.05 (padded stride 260)", flush=True)
    got1 = _static_solve(A, torch, C1, L1, eps, tol)
    got2 = _static_solve(A, torch, C2, L2, 0.05, tol, ld=260)
    for (st, res, f, g), (gst, gres, gf, gg, nalloc), L, C, e in ((ref1, got1, L1, C1, eps), (ref2, got2, L2, C2, 0.05)):
        print(f"[case] {L.I}x{L.J}: {gres.iterations} iterations, violation {gres.marginal_violation:.3e}, "
              f"allocations {nalloc}", flush=True)
        assert nalloc == 0
        assert gst == st == A.OT_OK
        assert gres.iterations == res.iterations and gres.fp64_iterations == res.fp64_iterations
        assert gres.marginal_violation == res.marginal_violation
        np.testing.assert_array_equal(gf, f)
        np.testing.assert_array_equal(gg, g)
        chk = oracle_lib.plan_stats(C.astype(np.float64), L.a, L.b, gf, gg, e)
        assert chk["marginal_violation"] < tol


def test_static_solve_warm_start_and_limits(A, oracle_lib):
    import torch

    dev = torch.device("cuda:0")
    L, C = _instance(oracle_lib, I=1500, J=40, seed=3)
    Cd = torch.from_numpy(C).to(dev)
    a, b = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    f = torch.empty(L.I, dtype=torch.float64, device=dev)
    g = torch.empty(L.J, dtype=torch.float64, device=dev)
    st, cold = A.ot_assoc_solve_static(Cd, a, b, f, g, 0.05, 1e-9, 2000)
    assert st == A.OT_OK
    # a warm start from the converged potentials: a few iterations (the FP32
    # phase has to see its residual stall), the same as the handle's warm start
    with A.Solver(L.I, L.J) as s:
        s.solve_dense(Cd, a, b, 0.05, 1e-9, 2000)
        _, hwarm = s.solve_dense(Cd, a, b, 0.05, 1e-9, 2000, warm_start=True)
        hf, hg = s.potentials()
    st, warm = A.ot_assoc_solve_static(Cd, a, b, f, g, 0.05, 1e-9, 2000, warm_start=1)
    print(f"\n[case] 1500x40 warm start: {warm.iterations} iterations (cold {cold.iterations})", flush=True)
    assert st == A.OT_OK and warm.iterations == hwarm.iterations < cold.iterations // 2
    np.testing.assert_array_equal(f.cpu().numpy(), hf)
    np.testing.assert_array_equal(g.cpu().numpy(), hg)
    chk = oracle_lib.plan_stats(C.astype(np.float64), L.a, L.b, f.cpu().numpy(), g.cpu().numpy(), 0.05)
    assert chk["marginal_violation"] < 1e-9
    # beyond the stated maximum: rejected before anything runs
    big = torch.zeros((4, 513), dtype=torch.float32, device=dev)
    bb = torch.full((513,), 1.0 / 513, dtype=torch.float64, device=dev)
    aa = torch.full((4,), 0.25, dtype=torch.float64, device=dev)
    with pytest.raises(A.OTError) as e:
        A.ot_assoc_solve_static(big, aa, bb, aa.clone(), bb.clone(), 0.1, 1e-6, 10)
    assert e.value.status == A.OT_EINVAL
