"""GPU tests of the request server (ot_serve_*): requests admitted while
others run, results against the FP64 oracle, the same result alone and in the
mix, warm starts across drifting snapshots of a layout, and admission by the
device-memory budget."""

import numpy as np
import pytest

import scenario as S

pytestmark = pytest.mark.gpu

EPS = 0.05
TOL = 1e-8


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


def run_until_done(srv, n, limit=100000):
    done = []
    for _ in range(limit):
        done += srv.progress()
        if len(done) >= n:
            return done
    raise AssertionError("server did not finish")


@pytest.fixture(scope="module")
def reqs(oracle_lib):
    out = []
    for k, (I, J) in enumerate([(900, 40), (2500, 200), (1300, 77), (600, 400), (3100, 130), (1700, 256)]):
        L = S.make_layout(I, J, 1000.0, seed=6000 + k)
        C64, _ = oracle_lib.cost(L)
        C32 = C64.astype(np.float32)
        out.append(dict(L=L, C32=C32, Cq=C32.astype(np.float64)))
    return out


def test_serve_mix_matches_oracle_and_alone(A, oracle_lib, reqs):
    announce("6 requests submitted together; each alone in a fresh server")
    with A.Server() as srv:
        for k, x in enumerate(reqs):
            srv.submit(x["C32"], x["L"].a, x["L"].b, EPS, TOL, 2000, layout_key=100 + k, user_tag=k)
        done = run_until_done(srv, len(reqs))
        mix = {}
        for c in done:
            k = c.user_tag
            x = reqs[k]
            assert c.result.status == A.OT_OK, c.result.status
            assert c.t_submit <= c.t_admit <= c.t_done
            f, g = srv.potentials(100 + k, x["L"].I, x["L"].J)
            chk = oracle_lib.plan_stats(x["Cq"], x["L"].a, x["L"].b, f, g, EPS)
            assert c.result.marginal_violation < TOL
            assert chk["marginal_violation"] < TOL * 1.05
            ref = oracle_lib.sinkhorn(x["Cq"], x["L"].a, x["L"].b, EPS, 1e-12, 20000)
            rs = oracle_lib.plan_stats(x["Cq"], x["L"].a, x["L"].b, ref.f, ref.g, EPS)
            assert abs(chk["objective"] - rs["objective"]) <= 1e-6 * abs(rs["objective"])
            mix[k] = (f, g, c.result.iterations)
    for k in (1, 3):
        x = reqs[k]
        with A.Server() as srv:
            srv.submit(x["C32"], x["L"].a, x["L"].b, EPS, TOL, 2000, layout_key=7)
            (c,) = run_until_done(srv, 1)
            f, g = srv.potentials(7, x["L"].I, x["L"].J)
        assert c.result.iterations == mix[k][2]
        assert np.array_equal(f, mix[k][0]) and np.array_equal(g, mix[k][1])


def test_serve_staggered_arrivals(A, oracle_lib, reqs):
    announce("requests submitted while others are in flight")
    with A.Server() as srv:
        got = []
        for k, x in enumerate(reqs):
            srv.submit(x["C32"], x["L"].a, x["L"].b, EPS, TOL, 2000, user_tag=k)
            got += srv.progress()
            got += srv.progress()
        got += run_until_done(srv, len(reqs) - len(got))
        assert sorted(c.user_tag for c in got) == list(range(len(reqs)))
        for c in got:
            assert c.result.status == A.OT_OK and c.result.marginal_violation < TOL


def test_serve_warm_start_over_drift(A, oracle_lib):
    announce("one layout, 5 snapshots with 5 m drift, warm started")
    L0 = S.make_layout(2000, 100, 1000.0, seed=6100)
    pos = S.drift_positions(L0, 5, 5.0, seed=6101)
    with A.Server() as srv:
        iters = []
        for t, xy in enumerate(pos):
            L = S.with_positions(L0, xy)
            C32 = oracle_lib.cost(L)[0].astype(np.float32)
            srv.submit(C32, L.a, L.b, 0.02, 1e-6, 2000, layout_key=42, user_tag=t)
            (c,) = run_until_done(srv, 1)
            assert c.result.status == A.OT_OK
            assert c.warm == (1 if t > 0 else 0)
            f, g = srv.potentials(42, L.I, L.J)
            chk = oracle_lib.plan_stats(C32.astype(np.float64), L.a, L.b, f, g, 0.02)
            assert chk["marginal_violation"] < 1e-6 * 1.05
            iters.append(c.result.iterations)
    assert max(iters[1:]) < iters[0], iters


def test_serve_budget_admission(A, reqs):
    announce("admission by a small device-memory budget")
    x = reqs[4]
    I, J = x["L"].I, x["L"].J
    one = 4 * I * (J + 3) // 4 * 4 + 8 * 8 * (I + J) + 8 * ((I + 63) // 64) * (J + 6) + 4096
    with A.Server(budget_bytes=float(2.5 * one)) as srv:
        for k in range(5):
            srv.submit(x["C32"], x["L"].a, x["L"].b, EPS, TOL, 2000, user_tag=k)
        seen_running = 0
        done = []
        for _ in range(100000):
            done += srv.progress()
            q, r, _, used = srv.counts()
            seen_running = max(seen_running, r)
            assert used <= 2.5 * one
            if len(done) == 5:
                break
        assert len(done) == 5 and seen_running <= 2
        assert all(c.result.status == A.OT_OK for c in done)
        # a request larger than the whole budget is completed with OT_ENOMEM
        big = np.ones((20000, 400), np.float32)
        srv.submit(big, np.full(20000, 1 / 20000), np.full(400, 1 / 400), EPS, TOL, 10, user_tag=99)
        (c,) = run_until_done(srv, 1)
        assert c.user_tag == 99 and c.result.status == A.OT_ENOMEM
