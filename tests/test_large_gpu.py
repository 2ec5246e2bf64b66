"""GPU parity of the large workload: 200000 devices x 2000 RRHs over a 15 km
square with 16 hot spots, the rate cost of Sec. II-A / Sec. IV choice (ii)
regenerated on the fly from positions (never materialised), eps 0.01,
tol 1e-8 (Alg. 1 of Sec. III-B at the "thousands of users" scale).

The reference is the FP64 oracle's solution of the same instance to a
residual below 1e-12, stored in tests/golden/large_200000x2000_reference.txt
by its committed script (scale = the oracle's lower median of all 4e8 values
of 1/R; <C, pi>; f on a seeded 1 % of the rows; every g). The test then
* recomputes, with the oracle's own FP64 costs regenerated row by row, both
  marginals and <C, pi> of the GPU's potentials over all 4e8 cells: the
  oracle-side marginal violation must meet tol and the transport cost must be
  within 1e-6 relative of the reference's;
* compares the GPU's own plan (ot_assoc_plan, FP64) with the reference plan
  on the sampled rows: L1 distance relative to the sample's mass <= 1e-6.
"""

import os

import numpy as np
import pytest

import scenario as S

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "large_200000x2000_reference.txt")


def load_reference():
    ref, rows, f = {}, [], []
    for ln in open(GOLD):
        if ln.startswith("#") or not ln.strip():
            continue
        t = ln.split()
        if t[0] == "g":
            ref["g"] = np.array([float(v) for v in t[1:]])
        elif t[0][0].isdigit():
            rows.append(int(t[0]))
            f.append(float(t[1]))
        else:
            ref[t[0]] = float(t[1])
    ref["rows"] = np.array(rows, dtype=np.int64)
    ref["f_rows"] = np.array(f)
    return ref


@pytest.fixture(scope="module")
def A():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1805_01559_amd import ot_assoc
    ot_assoc.lib()
    return ot_assoc


def test_large_200000x2000_against_oracle_reference(A, oracle_lib):
    import torch

    ref = load_reference()
    L = S.preset_layout("large_200000x2000")
    assert ref["g"].size == L.J and ref["rows"].size == L.I // 100
    eps, tol, scale = ref["eps"], 1e-8, ref["scale"]
    print(f"\n[case] large_200000x2000, geometry cost on the fly, eps {eps}, tol {tol}, scale {scale!r}", flush=True)
    dev = torch.device("cuda:0")
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    ad, bd = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    rows = ref["rows"]
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, ad, bd, eps, tol, 2000)
        f, g = s.potentials()
        print(f"[case] {res.iterations} iterations ({res.fp64_iterations} FP64), {res.seconds:.3f} s, "
              f"violation {res.marginal_violation:.3e}", flush=True)
        P = torch.empty((L.I, L.J), dtype=torch.float64, device=dev)
        s.plan(P)
        P_rows = P[torch.from_numpy(rows).to(dev)].cpu().numpy()
        del P
    assert st == A.OT_OK
    assert res.marginal_violation < tol
    # oracle-side statistics of the GPU's potentials over every cell
    chk = oracle_lib.geometry_plan_stats(L, scale, f, g, eps)
    obj_rel = abs(chk["objective"] - ref["objective"]) / ref["objective"]
    print(f"[case] oracle-side violation {chk['marginal_violation']:.3e}, objective rel err {obj_rel:.3e} "
          f"(GPU's own {abs(res.objective - ref['objective']) / ref['objective']:.3e})", flush=True)
    assert chk["marginal_violation"] < tol
    assert obj_rel <= 1e-6
    assert abs(res.marginal_violation - chk["marginal_violation"]) <= 1e-3 * chk["marginal_violation"] + 1e-12
    # plans on the sampled rows: the GPU's own against the reference's
    C_rows = oracle_lib.cost_rows(L, rows, scale)
    P_ref = oracle_lib.plan(C_rows, ref["f_rows"], ref["g"], eps)
    l1 = float(np.abs(P_rows - P_ref).sum())
    mass = float(P_ref.sum())
    print(f"[case] plan L1 on {rows.size} sampled rows: {l1:.3e} of mass {mass:.4e} ({l1 / mass:.3e} relative)",
          flush=True)
    assert np.all(np.isfinite(P_rows))
    assert l1 / mass <= 1e-6
