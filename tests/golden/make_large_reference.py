"""Writes large_200000x2000_reference.txt: the FP64 oracle's solution of the
large workload (200000 devices x 2000 RRHs over a 15 km square with 16 hot
spots, the rate cost C = (1/R) / median(1/R) of Sec. II-A / Sec. IV cost
choice (ii), eps = 0.01), run to a total marginal residual below 1e-12 with
the Sinkhorn iteration of Sec. III-B. It calls only the oracle and the seeded
scenario generator.

Recorded: the scale (the lower median of all 4e8 values of 1/R), the
iteration count and residual, <C, pi>, the regularised objective of eq. (5)
and the mass; a seeded 1 % sample of device rows with their potentials f_i;
every g_j. The plan of a sampled row is exp((f_i + g_j - C_ij) / eps) with the
oracle's cost of that row, so the GPU parity test can compare plans on the
sample without the full cost.

Needs about 14 GB of host memory (C, its transpose and a sorted copy for the
median) and a few minutes on 8 cores.

Usage: python tests/golden/make_large_reference.py
"""

import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import scenario as S  # noqa: E402
from oracle import oracle as O  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "large_200000x2000_reference.txt")
EPS, TOL, MAX_ITER = 0.01, 1e-12, 2000
SAMPLE_SEED, SAMPLE_FRAC = 2026, 0.01


def sample_rows(I):
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(I, int(round(SAMPLE_FRAC * I)), replace=False))


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def main():
    O.build(force=False)
    t0 = time.time()
    L = S.preset_layout("large_200000x2000")
    C, scale = O.cost(L)
    t1 = time.time()
    print(f"cost and median: {t1 - t0:.1f} s, scale {scale!r}", flush=True)
    res = O.sinkhorn(C, L.a, L.b, EPS, TOL, MAX_ITER)
    t2 = time.time()
    print(f"sinkhorn: {res.iters} iterations, residual {res.residual:.3e}, {t2 - t1:.1f} s", flush=True)
    if res.status != 0:
        raise SystemExit(f"oracle did not reach tol: status {res.status}")
    st = O.plan_stats(C, L.a, L.b, res.f, res.g, EPS)
    rows = sample_rows(L.I)
    lines = [
        "# FP64 oracle solution of the large workload 200000 x 2000 (15 km, 16 hot spots, seed 2000), rate cost",
        "# C = (1/R) / scale, eps = 0.01, Sinkhorn to a total marginal residual below 1e-12.",
        "# Written by make_large_reference.py (oracle and scenario generator only).",
        f"# host: {cpu_model()}, {os.cpu_count()} threads; cost {t1 - t0:.0f} s, solve {t2 - t1:.0f} s",
        f"scale {float(scale)!r}",
        f"eps {EPS!r}",
        f"tol {TOL!r}",
        f"iterations {res.iters}",
        f"residual {float(st['marginal_violation'])!r}",
        f"objective {float(st['objective'])!r}",
        f"reg_objective {float(st['reg_objective'])!r}",
        f"mass {float(st['mass'])!r}",
        f"sample_seed {SAMPLE_SEED}",
        f"g {' '.join(repr(float(v)) for v in res.g)}",
        "# sampled rows: i f_i",
    ]
    lines += [f"{int(i)} {float(res.f[i])!r}" for i in rows]
    with open(OUT, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {OUT} ({len(rows)} sampled rows)", flush=True)


if __name__ == "__main__":
    main()
