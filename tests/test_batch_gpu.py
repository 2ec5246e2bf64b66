"""GPU parity of the batched engine (ot_assoc_solve_batch) against the FP64
oracle: uneven instances across every column class and ragged row counts,
every input kind, determinism, independence of an instance from its batch
neighbours, limits and errors.

Each instance is a problem in its own right: the oracle solves it on the same
FP32-rounded cost (rounded on the oracle side from its own FP64 cost) and the
batch must match to the FP32-path bar: marginal violation < tol (as reported
and as the oracle recomputes it from the batch's potentials), transport cost
within 1e-6 relative of the oracle run to 1e-12, plan L1 within 1e-6.
"""

import numpy as np
import pytest

import scenario as S

pytestmark = pytest.mark.gpu

OBJ_RTOL = 1e-6
PLAN_L1 = 1e-6
TOL = 1e-8
EPS = 0.05

# (I, J): every column class (J <= 64, 128, 256, 512), J not a multiple of 4,
# row counts that leave ragged last parts for 64 / 128 / 256 rows per part
SIZES = [(700, 20), (1501, 50), (513, 64), (2000, 101), (999, 130), (3001, 257), (1200, 400), (800, 512)]


@pytest.fixture(scope="module")
def A():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_01559_amd import ot_assoc
    ot_assoc.lib()
    return ot_assoc


@pytest.fixture(scope="module")
def inst(oracle_lib):
    """Instances from the small-workload generator, their oracle FP64 costs
    rounded to FP32, and the oracle's converged solutions of those costs."""
    out = []
    for k, (I, J) in enumerate(SIZES):
        L = S.make_layout(I, J, 1000.0, seed=5000 + k)
        C64, scale = oracle_lib.cost(L)
        C32 = C64.astype(np.float32)
        Cq = C32.astype(np.float64)
        ref = oracle_lib.sinkhorn(Cq, L.a, L.b, EPS, 1e-12, 20000)
        ref_stats = oracle_lib.plan_stats(Cq, L.a, L.b, ref.f, ref.g, EPS)
        out.append(dict(L=L, C64=C64, C32=C32, Cq=Cq, scale=scale, ref=ref, ref_stats=ref_stats))
    return out


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def check(O, x, f, g, res, tol=TOL):
    L = x["L"]
    chk = O.plan_stats(x["Cq"], L.a, L.b, f, g, EPS)
    assert res.marginal_violation < tol, res.marginal_violation
    assert chk["marginal_violation"] < tol * 1.05, chk["marginal_violation"]
    rel = abs(chk["objective"] - x["ref_stats"]["objective"]) / abs(x["ref_stats"]["objective"])
    assert rel <= OBJ_RTOL, rel
    assert abs(res.objective - chk["objective"]) <= 1e-9 * abs(chk["objective"])
    P, P0 = O.plan(x["Cq"], f, g, EPS), O.plan(x["Cq"], x["ref"].f, x["ref"].g, EPS)
    l1 = np.abs(P - P0).sum()
    assert l1 <= PLAN_L1, l1
    # cell by cell (cells with mass): within 100 tol relative, f_i + g_j within 100 tol eps
    m = P0 > 1e-12 * P0.max()
    assert (np.abs(P - P0)[m] / P0[m]).max() <= 100 * tol
    dfg = np.abs((f[:, None] + g[None, :]) - (x["ref"].f[:, None] + x["ref"].g[None, :]))[m]
    assert dfg.max() <= 100 * tol * EPS * 1.0001 + 1e-15


def test_batch_uneven_host_fp32(A, oracle_lib, inst):
    announce(f"batch of {len(inst)} uneven instances, host FP32 costs, tuned")
    with A.Solver(16, 16) as s:
        st, res = s.solve_batch([x["C32"] for x in inst], [x["L"].a for x in inst], [x["L"].b for x in inst],
                                EPS, TOL, 2000)
        assert st == A.OT_OK, [r.status for r in res]
        for k, x in enumerate(inst):
            f, g = s.batch_potentials(k)
            check(oracle_lib, x, f, g, res[k])
            assert res[k].fp64_iterations >= 1


def test_batch_input_kinds(A, oracle_lib, inst):
    announce("batch of every input kind: FP64 host, FP32 device in place / padded, rates, geometry")
    import torch
    dev = torch.device("cuda:0")
    picks = [0, 2, 3, 6, 7]
    costs, aa, bb = [], [], []
    keep = []
    # FP64 host dense
    x = inst[0]
    costs.append(x["Cq"]); aa.append(x["L"].a); bb.append(x["L"].b)
    # FP32 device, J = 64 (referenced in place)
    x = inst[2]
    Cd = torch.from_numpy(x["C32"]).to(dev)
    costs.append(Cd); aa.append(torch.from_numpy(x["L"].a).to(dev)); bb.append(torch.from_numpy(x["L"].b).to(dev))
    # FP32 device, J = 101 (padded copy)
    x = inst[3]
    Cd2 = torch.from_numpy(x["C32"]).to(dev)
    costs.append(Cd2); aa.append(torch.from_numpy(x["L"].a).to(dev)); bb.append(torch.from_numpy(x["L"].b).to(dev))
    # rates, FP64 host, with the oracle's scale
    x = inst[6]
    R = oracle_lib.rates(x["L"])
    costs.append(A.matrix_desc(R, A.OT_COST_RATES, x["scale"])); aa.append(x["L"].a); bb.append(x["L"].b)
    keep.append(R)
    # geometry in device memory, oracle scale
    x = inst[7]
    xy = torch.from_numpy(x["L"].dev_xy).to(dev)
    rxy = torch.from_numpy(x["L"].rrh_xy).to(dev)
    costs.append(A.geometry_desc(xy, rxy, x["L"].radio, x["L"].shadow_key, x["scale"]))
    aa.append(torch.from_numpy(x["L"].a).to(dev)); bb.append(torch.from_numpy(x["L"].b).to(dev))
    with A.Solver(16, 16) as s:
        st, res = s.solve_batch(costs, aa, bb, EPS, TOL, 2000)
        assert st == A.OT_OK, [r.status for r in res]
        for q, k in enumerate(picks):
            f, g = s.batch_potentials(q)
            if k in (6, 7):
                # rates / geometry: the batch rounds its own FP64 cost to FP32;
                # check it against the oracle's FP64 cost at the FP32 bar
                x = inst[k]
                chk = oracle_lib.plan_stats(x["C64"], x["L"].a, x["L"].b, f, g, EPS)
                ref = oracle_lib.sinkhorn(x["C64"], x["L"].a, x["L"].b, EPS, 1e-12, 20000)
                rst = oracle_lib.plan_stats(x["C64"], x["L"].a, x["L"].b, ref.f, ref.g, EPS)
                assert res[q].marginal_violation < TOL
                assert abs(chk["objective"] - rst["objective"]) <= OBJ_RTOL * abs(rst["objective"])
                # FP32 rounding of C moves the marginals by at most |dC|/eps
                assert chk["marginal_violation"] < TOL + 2.0 ** -23 * x["C64"].max() / EPS * 2
            else:
                check(oracle_lib, inst[k], f, g, res[q])
    del keep


def test_batch_deterministic_and_independent_of_neighbours(A, inst):
    announce("batch determinism and neighbour independence (fixed layout)")
    costs = [x["C32"] for x in inst]
    aa = [x["L"].a for x in inst]
    bb = [x["L"].b for x in inst]
    with A.Solver(16, 16, batch_tune=0) as s:
        s.solve_batch(costs, aa, bb, EPS, TOL, 2000)
        full = [s.batch_potentials(k) for k in range(len(inst))]
        s.solve_batch(costs, aa, bb, EPS, TOL, 2000)
        again = [s.batch_potentials(k) for k in range(len(inst))]
        sub = [5, 1]
        s.solve_batch([costs[k] for k in sub], [aa[k] for k in sub], [bb[k] for k in sub], EPS, TOL, 2000)
        alone = [s.batch_potentials(q) for q in range(len(sub))]
    for k in range(len(inst)):
        assert np.array_equal(full[k][0], again[k][0]) and np.array_equal(full[k][1], again[k][1])
    for q, k in enumerate(sub):
        assert np.array_equal(full[k][0], alone[q][0]) and np.array_equal(full[k][1], alone[q][1])


def test_batch_plan(A, oracle_lib, inst):
    announce("batch plan of two instances against the oracle's plan of the same potentials")
    with A.Solver(16, 16) as s:
        s.solve_batch([inst[1]["C32"], inst[5]["C32"]], [inst[1]["L"].a, inst[5]["L"].a],
                      [inst[1]["L"].b, inst[5]["L"].b], EPS, TOL, 2000)
        for q, k in enumerate([1, 5]):
            f, g = s.batch_potentials(q)
            P = s.batch_plan(q)
            Pr = oracle_lib.plan(inst[k]["Cq"], f, g, EPS)
            assert np.allclose(P, Pr, rtol=1e-12, atol=1e-300)
            P32 = s.batch_plan(q, dtype=np.float32)
            assert np.allclose(P32, Pr, rtol=2e-7, atol=1e-38)


def test_batch_single_instance_matches_plain_solver(A, inst):
    announce("one instance through the batch and through ot_assoc_solve")
    x = inst[5]
    with A.Solver(x["L"].I, x["L"].J) as s:
        st, r1 = s.solve_dense(x["C32"], x["L"].a, x["L"].b, EPS, TOL, 2000)
        f1, g1 = s.potentials()
        st, rb = s.solve_batch([x["C32"]], [x["L"].a], [x["L"].b], EPS, TOL, 2000)
        fb, gb = s.batch_potentials(0)
    assert r1.marginal_violation < TOL and rb[0].marginal_violation < TOL
    assert abs(r1.objective - rb[0].objective) <= 1e-9 * abs(r1.objective)
    # both are within tol of the same unique optimum
    P1 = np.exp((f1[:, None] + g1[None, :] - x["Cq"]) / EPS)
    Pb = np.exp((fb[:, None] + gb[None, :] - x["Cq"]) / EPS)
    assert np.abs(P1 - Pb).sum() <= 2 * PLAN_L1


def test_batch_max_iter_and_errors(A, inst):
    announce("batch iteration cap and input errors")
    costs = [inst[0]["C32"], inst[4]["C32"]]
    aa = [inst[0]["L"].a, inst[4]["L"].a]
    bb = [inst[0]["L"].b, inst[4]["L"].b]
    with A.Solver(16, 16) as s:
        st, res = s.solve_batch(costs, aa, bb, 0.002, 1e-12, 3)
        assert st == A.OT_WARN_MAXITER
        for r in res:
            assert r.status == A.OT_WARN_MAXITER and r.iterations <= 3
        with pytest.raises(A.OTError) as e:
            s.solve_batch([np.ones((10, 513), np.float32)], [np.full(10, 0.1)], [np.full(513, 1 / 513 * 1.0)],
                          EPS, TOL, 10)
        assert e.value.status == A.OT_EINVAL
        with pytest.raises(A.OTError) as e:
            s.solve_batch(costs, [aa[0] * 2.0, aa[1]], bb, EPS, TOL, 10)
        assert e.value.status == A.OT_EINVAL
        with pytest.raises(A.OTError) as e:
            s.solve_batch(costs, aa, bb, [EPS, -1.0], TOL, 10)
        assert e.value.status == A.OT_EINVAL
        # the handle still works after rejected batches
        st, res = s.solve_batch(costs, aa, bb, EPS, TOL, 2000)
        assert st == A.OT_OK


def test_batch_constant_cost_closed_form(A):
    announce("batch of constant costs: pi = a b^T / sum(a)")
    rng = np.random.default_rng(7)
    costs, aa, bb = [], [], []
    for I, J in [(37, 5), (300, 33), (129, 128)]:
        a = rng.random(I) + 0.1
        a /= a.sum()
        b = rng.random(J) + 0.1
        b /= b.sum()
        costs.append(np.full((I, J), 0.7, np.float32))
        aa.append(a)
        bb.append(b)
    with A.Solver(16, 16) as s:
        st, res = s.solve_batch(costs, aa, bb, EPS, 1e-10, 2000)
        assert st == A.OT_OK
        for k in range(3):
            P = s.batch_plan(k)
            assert np.allclose(P, np.outer(aa[k], bb[k]), rtol=1e-8, atol=0)


def test_batch_row_padded_inputs_in_place(A, oracle_lib, inst):
    """Row-padded device matrices whose padding holds NaN: those with J a
    multiple of 4 are referenced in place (no 16-byte vector reaches the
    padding), the others copied into the engine's +inf-padded layout; against
    the oracle, and bitwise equal to the same instances copied from the host."""
    announce("batch of row-padded device matrices (NaN padding), and the same costs copied from the host")
    import torch
    dev = torch.device("cuda:0")
    picks = [0, 2, 3, 4, 5]
    costs, aa, bb, keep = [], [], [], []
    for k in picks:
        x = inst[k]
        I, J = x["C32"].shape
        ld = (J + 3) // 4 * 4 + 4
        buf = np.full((I, ld), np.nan, np.float32)
        buf[:, :J] = x["C32"]
        t = torch.from_numpy(buf).to(dev)
        keep.append(t)
        costs.append(A.matrix_desc(t, A.OT_COST_DENSE, J=J))
        aa.append(torch.from_numpy(x["L"].a).to(dev))
        bb.append(torch.from_numpy(x["L"].b).to(dev))
    with A.Solver(16, 16, batch_tune=0) as s:
        st, res = s.solve_batch(costs, aa, bb, EPS, TOL, 2000)
        assert st == A.OT_OK, [r.status for r in res]
        placed = [s.batch_potentials(q) for q in range(len(picks))]
        for q, k in enumerate(picks):
            check(oracle_lib, inst[k], *placed[q], res[q])
        st, res2 = s.solve_batch([inst[k]["C32"] for k in picks], [inst[k]["L"].a for k in picks],
                                 [inst[k]["L"].b for k in picks], EPS, TOL, 2000)
        assert st == A.OT_OK
        for q in range(len(picks)):
            f, g = s.batch_potentials(q)
            assert np.array_equal(f, placed[q][0]) and np.array_equal(g, placed[q][1]), picks[q]
            assert res2[q].iterations == res[q].iterations


def test_batch_256_uneven_tuned_against_oracle(A, oracle_lib):
    """The batched workload itself: 256 instances, I log-uniform in
    [500, 20000], J in [20, 400], 1 km layouts (seeds 3000 + k), eps 0.05,
    tol 1e-6, with the autotuner choosing the launch configuration. Every
    instance must report a violation below tol; a seeded quarter of them (64)
    is checked against the oracle on the same FP32-rounded cost: oracle-side
    violation below tol, transport cost within 1e-6 relative of the oracle run
    to 1e-12, plan L1 within 10 tol (the oracle's own tol-run reaches up to
    2 tol here)."""
    announce("batch of the 256 uneven instances, tuned, a seeded quarter against the oracle")
    eps, tol = 0.05, 1e-6
    Ls = S.batch_layouts(256, 3000)
    costs = [oracle_lib.cost(L)[0].astype(np.float32) for L in Ls]
    with A.Solver(16, 16) as s:
        st, res = s.solve_batch(costs, [L.a for L in Ls], [L.b for L in Ls], eps, tol, 2000)
        assert st == A.OT_OK, [r.status for r in res]
        waves, rpp = s.batch_config()
        picks = np.sort(np.random.default_rng(2027).choice(256, 64, replace=False))
        pots = {int(k): s.batch_potentials(int(k)) for k in picks}
    print(f"[case] tuned configuration: {waves} waves, {rpp} rows per part", flush=True)
    assert all(r.marginal_violation < tol for r in res)
    worst = [0.0, 0.0, 0.0]
    for k in picks:
        L, Cq = Ls[k], costs[k].astype(np.float64)
        f, g = pots[int(k)]
        ref = oracle_lib.sinkhorn(Cq, L.a, L.b, eps, 1e-12, 20000)
        rst = oracle_lib.plan_stats(Cq, L.a, L.b, ref.f, ref.g, eps)
        chk = oracle_lib.plan_stats(Cq, L.a, L.b, f, g, eps)
        rel = abs(chk["objective"] - rst["objective"]) / abs(rst["objective"])
        l1 = float(np.abs(oracle_lib.plan(Cq, f, g, eps) - oracle_lib.plan(Cq, ref.f, ref.g, eps)).sum())
        worst = [max(worst[0], chk["marginal_violation"]), max(worst[1], rel), max(worst[2], l1)]
        assert chk["marginal_violation"] < tol * 1.05, (int(k), chk["marginal_violation"])
        assert rel <= OBJ_RTOL, (int(k), rel)
        assert l1 <= 10 * tol, (int(k), l1)
    print(f"[case] worst of 64: violation {worst[0]:.2e}, objective {worst[1]:.2e}, plan L1 {worst[2]:.2e}",
          flush=True)


CHILD = r'''
import hashlib, json, sys
import numpy as np
import torch
from paper_1805_01559_amd import ot_assoc as A
d = np.load(sys.argv[1])
n = int(d["n"])
costs = [np.ascontiguousarray(d[f"C{k}"]) for k in range(n)]
aa = [d[f"a{k}"] for k in range(n)]
bb = [d[f"b{k}"] for k in range(n)]
with A.Solver(16, 16) as s:
    st, res = s.solve_batch(costs, aa, bb, 0.05, 1e-6, 2000)
    w, r = s.batch_config()
    h = hashlib.sha256()
    for k in range(n):
        f, g = s.batch_potentials(k)
        h.update(f.tobytes()); h.update(g.tobytes())
print(json.dumps(dict(status=int(st), waves=int(w), rpp=int(r), digest=h.hexdigest(),
                      viol=max(x.marginal_violation for x in res))), flush=True)
'''


def test_batch_tune_cache_persists_choice(A, oracle_lib, tmp_path):
    """The autotuner's choice is written to OT_ASSOC_TUNE_CACHE and a later
    process takes it from there: two fresh processes on the same batch report
    the same configuration and bitwise the same potentials; a process given an
    edited cache runs the edited configuration (it times nothing)."""
    import json, os, subprocess, sys
    announce("autotuner cache across processes (48 uneven instances)")
    Ls = S.batch_layouts(48, 3100)
    arrs = {"n": np.array(len(Ls))}
    for k, L in enumerate(Ls):
        arrs[f"C{k}"] = oracle_lib.cost(L)[0].astype(np.float32)
        arrs[f"a{k}"], arrs[f"b{k}"] = L.a, L.b
    data = tmp_path / "batch.npz"
    np.savez(data, **arrs)
    child = tmp_path / "child.py"
    child.write_text(CHILD)
    cache = tmp_path / "tune.txt"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, OT_ASSOC_TUNE_CACHE=str(cache),
               PYTHONPATH=os.pathsep.join([root, os.environ.get("PYTHONPATH", "")]))

    def run():
        out = subprocess.run([sys.executable, "-u", str(child), str(data)], env=env, cwd=root, capture_output=True,
                             text=True, timeout=240)
        assert out.returncode == 0, out.stderr[-2000:]
        return json.loads(out.stdout.strip().splitlines()[-1])

    first = run()
    lines = [ln.split() for ln in cache.read_text().splitlines() if ln.strip()]
    print(f"[case] first process: {first}; cache: {lines}", flush=True)
    assert first["status"] == A.OT_OK and first["viol"] < 1e-6
    assert len(lines) == 1 and int(lines[0][1]) == first["waves"] and int(lines[0][2]) == first["rpp"]
    second = run()
    assert second == first
    assert len(cache.read_text().splitlines()) == 1  # nothing new was tuned
    # an edited entry is honoured as it stands
    other = (4 if first["waves"] == 8 else 8, 256 if first["rpp"] != 256 else 64)
    cache.write_text(f"{lines[0][0]} {other[0]} {other[1]}\n")
    third = run()
    print(f"[case] edited cache -> {third}", flush=True)
    assert (third["waves"], third["rpp"]) == other
    assert third["status"] == A.OT_OK and third["viol"] < 1e-6
