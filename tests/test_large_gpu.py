"""GPU test of the large workload: 200000 devices x 2000 RRHs over a 15 km
square with 16 hot spots, the cost regenerated on the fly from the positions
(it is never materialised), eps 0.01, tol 1e-8.

The oracle cannot hold this instance's cost (4e8 FP64 rates), so it checks
sampled rows: the scale of the cost is the oracle's lower median of 1/R over
2000 random devices (any positive scale defines a valid problem), and for 64
sampled devices the oracle recomputes their costs and their row sums
sum_j exp((f_i + g_j - C_ij) / eps) from the GPU's potentials. Those rows'
deviations from a_i are terms of the marginal violation the library reports,
so their total cannot exceed that violation times sum(a); and the library's
own violation must meet tol.
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


def test_large_200000x2000_on_the_fly(A, oracle_lib):
    print("\n[case] large_200000x2000, geometry cost on the fly, eps 0.01, tol 1e-8", flush=True)
    import torch
    L = S.preset_layout("large_200000x2000")
    rng = np.random.default_rng(2024)
    scale = oracle_lib.lower_median(1.0 / oracle_lib.rates_rows(L, np.sort(rng.choice(L.I, 2000, replace=False))))
    eps, tol = 0.01, 1e-8
    dev = torch.device("cuda:0")
    xy = torch.from_numpy(L.dev_xy).to(dev)
    rxy = torch.from_numpy(L.rrh_xy).to(dev)
    ad, bd = torch.from_numpy(L.a).to(dev), torch.from_numpy(L.b).to(dev)
    with A.Solver(L.I, L.J) as s:
        st, res = s.solve_geometry(xy, rxy, L.radio, L.shadow_key, scale, ad, bd, eps, tol, 20000)
        f, g = s.potentials()
    print(f"[case] {res.iterations} iterations ({res.fp64_iterations} FP64), {res.seconds:.2f} s, "
          f"violation {res.marginal_violation:.3e}", flush=True)
    assert st == A.OT_OK
    assert res.marginal_violation < tol
    assert np.all(np.isfinite(f)) and np.all(np.isfinite(g))
    rows = np.sort(rng.choice(L.I, 64, replace=False))
    C = oracle_lib.cost_rows(L, rows, scale)
    logp = (f[rows][:, None] + g[None, :] - C) / eps
    P = np.exp(logp)
    rs = P.sum(axis=1)
    dev_rows = np.abs(rs - L.a[rows])
    assert dev_rows.sum() <= res.marginal_violation * L.a.sum() * (1 + 1e-9) + 1e-18
    assert np.all(np.isfinite(P)) and rs.min() > 0
