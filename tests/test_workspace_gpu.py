"""GPU tests of the handle options around the solve of eq. (5) (Sec. III-B):
a caller-owned (torch) workspace from which every device buffer of the
single-instance calls is carved, the stop-rule cadence `check_every`, and the
read-only streaming ceiling used beside the sweeps' HBM figures.

Results with a workspace are compared bitwise with a handle that allocates
its own (the same kernels run on the same inputs), and both against the
FP64 oracle."""

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


@pytest.fixture(scope="module")
def cran(oracle_lib):
    L = S.preset_layout("cran_20000x400")
    C64, _ = oracle_lib.cost(L)
    return L, C64.astype(np.float32)


def test_torch_workspace_solve_allocates_nothing(A, cran, oracle_lib):
    import torch

    L, C32 = cran
    eps, tol = 0.02, 1e-8
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(C32).to(dev)
    ad, bd = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    nbytes = A.ot_assoc_workspace_size(L.I, L.J)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    print(f"\n[case] 20000x400 dense, torch workspace of {nbytes} bytes", flush=True)
    n0 = A.ot_assoc_device_allocations()
    with A.Solver(L.I, L.J, workspace=ws.data_ptr(), workspace_bytes=nbytes) as s:
        assert A.ot_assoc_device_allocations() == n0  # create took its buffers from the workspace
        st, res = s.solve_dense(Cd, ad, bd, eps, tol, 2000)
        f, g = s.potentials()
        Pd = torch.empty((L.I, L.J), dtype=torch.float32, device=dev)
        s.plan(Pd)
        Ph = s.plan(np.empty((L.I, L.J), dtype=np.float64))  # host plan: blocks through the work region
        loads = s.rrh_loads()
        st2, res2 = s.solve_dense(Cd, ad, bd, eps, tol, 2000, warm_start=True)
        assert A.ot_assoc_device_allocations() == n0, "a call on a workspace handle allocated device memory"
    assert st == A.OT_OK and res.marginal_violation < tol
    with A.Solver(L.I, L.J) as s:
        _, ref = s.solve_dense(Cd, ad, bd, eps, tol, 2000)
        f0, g0 = s.potentials()
        P0 = s.plan()
        loads0 = s.rrh_loads()
    # the same kernels on the same inputs: bitwise the same results
    assert res.iterations == ref.iterations
    np.testing.assert_array_equal(f, f0)
    np.testing.assert_array_equal(g, g0)
    np.testing.assert_array_equal(Ph, P0)
    np.testing.assert_array_equal(Pd.cpu().numpy(), P0.astype(np.float32))
    np.testing.assert_array_equal(loads, loads0)
    # and against the oracle
    C = C32.astype(np.float64)
    chk = oracle_lib.plan_stats(C, L.a, L.b, f, g, eps)
    assert chk["marginal_violation"] < tol


def test_workspace_limits(A, cran):
    import torch

    L, C32 = cran
    dev = torch.device("cuda:0")
    nbytes = A.ot_assoc_workspace_size(1000, 50)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    with pytest.raises(A.OTError) as e:  # too small
        A.Solver(1000, 50, workspace=ws.data_ptr(), workspace_bytes=nbytes - 256)
    assert e.value.status == A.OT_EINVAL
    with pytest.raises(A.OTError) as e:  # misaligned
        A.Solver(1000, 50, workspace=ws.data_ptr() + 8, workspace_bytes=nbytes)
    assert e.value.status == A.OT_EINVAL
    # a host-memory matrix needs staging room beyond the fixed buffers
    Ls = S.preset_layout("small_1000x50")
    C = np.ascontiguousarray(np.random.default_rng(0).uniform(0.1, 2.0, (Ls.I, Ls.J)))
    with A.Solver(Ls.I, Ls.J, workspace=ws.data_ptr(), workspace_bytes=nbytes) as s:
        with pytest.raises(A.OTError) as e:
            s.solve_dense(C, Ls.a, Ls.b, 0.05, 1e-8, 2000)
        assert e.value.status == A.OT_ENOMEM
    big = torch.empty(nbytes + C.nbytes, dtype=torch.uint8, device=dev)
    n0 = A.ot_assoc_device_allocations()
    with A.Solver(Ls.I, Ls.J, workspace=big.data_ptr(), workspace_bytes=big.numel()) as s:
        st, res = s.solve_dense(C, Ls.a, Ls.b, 0.05, 1e-8, 2000)
    assert A.ot_assoc_device_allocations() == n0
    assert st == A.OT_OK and res.marginal_violation < 1e-8


@pytest.mark.parametrize("persistent", [1, 0])
def test_check_every(A, cran, oracle_lib, persistent):
    import torch

    L, C32 = cran
    eps, tol = 0.02, 1e-8
    dev = torch.device("cuda:0")
    Cd = torch.from_numpy(C32).to(dev)
    ad, bd = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    with A.Solver(L.I, L.J, persistent=persistent) as s:
        _, r1 = s.solve_dense(Cd, ad, bd, eps, tol, 2000)
    for ce in (3, 8):
        with A.Solver(L.I, L.J, persistent=persistent, check_every=ce) as s:
            st, r = s.solve_dense(Cd, ad, bd, eps, tol, 2000)
            f, g = s.potentials()
        fast = r.iterations - r.fp64_iterations
        print(f"\n[case] persistent={persistent} check_every={ce}: {r.iterations} iterations "
              f"({fast} FP32), every-iteration run {r1.iterations}", flush=True)
        assert st == A.OT_OK and r.marginal_violation < tol
        # the FP32 phase stops only at a multiple of check_every, no earlier than with every check
        assert fast % ce == 0
        assert fast >= r1.iterations - r1.fp64_iterations
        assert fast < r1.iterations - r1.fp64_iterations + 4 * ce  # (a stall may need a later multiple)
        chk = oracle_lib.plan_stats(C32.astype(np.float64), L.a, L.b, f, g, eps)
        assert chk["marginal_violation"] < tol


def test_read_ceiling(A):
    import torch

    buf = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")  # 1 GiB, above the last-level cache
    with A.Solver(100, 10) as s:
        ms = s.time_read(buf, reps=10)
    gbps = buf.numel() * 4 / (ms * 1e-3) / 1e9
    print(f"\n[case] read-only stream over 1 GiB: {ms * 1e3:.1f} us = {gbps:.0f} GB/s", flush=True)
    assert 1000.0 < gbps < 8000.0 * 1.05  # a real stream, and no faster than the published HBM peak
