"""Python face of the FP64 CPU oracle (``ot_oracle.c``) plus small helpers.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by the
benchmark's CPU-baseline leg; never by the product library, which must fail
loudly rather than fall back to anything here. The oracle shares no code with
the HIP path.

What it computes (paper sections in parentheses):
* ``rates`` / ``rates_rows``: R_ij = W log2(1 + SINR_ji) with full-power
  interference from all other RRHs (Sec. II-A);
* ``cost``: C_ij = (1/R_ij) / median(1/R), the load-per-unit-traffic cost of
  Sec. IV choice (ii), median-normalised;
* ``distance_cost``: C_ij = ||x_i - X_j|| / scale, the Euclidean cost of
  Sec. IV choice (i) (scale = 1 is the paper's form);
* ``sinkhorn``: FP64 log-domain Sinkhorn (Sec. III-B, Sinkhorn algorithm),
  stopping on the total absolute marginal residual (Sec. III, "Sinkhorn vs LP");
* ``plan`` / ``plan_stats``: pi = exp((f + g - C)/eps) (the KKT form of
  Sec. III-B), its marginals, <C, pi>, the objective of eq. (5) and the dual;
  ``geometry_plan_stats``: the marginals and <C, pi> with the rate cost
  regenerated row by row, for instances whose cost is too large to hold;
* ``brute_force_ot``: the unregularised OT of eqs. (2)-(4) on tiny square
  instances with uniform marginals, by enumeration of permutations;
* ``maxsinr_traffic`` and ``lemma1_lower_bound``: the maxSINR rule and the
  RRH traffic it induces (Sec. IV), and the total-load bound behind Lemma 1;
* ``rrh_loads`` and ``evaluate``: the RRH load rho_j, the mean number of jobs
  E[N_j] = rho_j / (1 - rho_j) under processor sharing and the devices'
  average completion times (Sec. II-B);
* ``adaptive_sinkhorn``: the Adaptive Sinkhorn Association of Sec. IV
  (Alg. 2), with the readings stated at the function.
"""

from __future__ import annotations

import ctypes as ct
import itertools
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libot_oracle.so")
SRC_PATH = os.path.join(HERE, "ot_oracle.c")

OK, WARN_MAXITER, EINVAL, ENOMEM, ENUMERIC = 0, 1, -1, -2, -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (strict IEEE: no fast-math, no contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.run(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
                        "-shared", "-std=c11", "-D_DEFAULT_SOURCE", "-o", tmp, SRC_PATH, "-lm"],
                       check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _Radio(ct.Structure):
    _fields_ = [("tx_power_w", ct.c_double), ("ref_gain", ct.c_double), ("pathloss_exp", ct.c_double),
                ("min_dist_m", ct.c_double), ("shadow_sigma_db", ct.c_double), ("noise_w", ct.c_double),
                ("bandwidth_hz", ct.c_double), ("shadow_key", ct.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ct.CDLL(LIB_PATH)
        dp, fp, i64, i64p = ct.POINTER(ct.c_double), ct.POINTER(ct.c_float), ct.c_int64, ct.POINTER(ct.c_int64)
        L.ora_splitmix64.restype = ct.c_uint64
        L.ora_splitmix64.argtypes = [ct.c_uint64]
        L.ora_shadow_normal.restype = ct.c_double
        L.ora_shadow_normal.argtypes = [ct.c_uint64, i64, i64]
        L.ora_rates_rows.argtypes = [fp, fp, i64, ct.POINTER(_Radio), i64p, i64, dp]
        L.ora_rates.argtypes = [fp, fp, i64, i64, ct.POINTER(_Radio), dp]
        L.ora_lower_median.restype = ct.c_double
        L.ora_lower_median.argtypes = [dp, i64]
        L.ora_cost_from_rates.argtypes = [dp, i64, dp, dp]
        L.ora_sinkhorn.argtypes = [dp, i64, i64, dp, dp, ct.c_double, ct.c_double, ct.c_int32, dp, dp, dp, dp,
                                   ct.POINTER(ct.c_int32), dp]
        L.ora_plan.argtypes = [dp, i64, i64, dp, dp, ct.c_double, dp]
        L.ora_plan_stats.argtypes = [dp, i64, i64, dp, dp, dp, dp, ct.c_double, dp, dp, dp]
        L.ora_geometry_plan_stats.argtypes = [fp, fp, i64, i64, ct.POINTER(_Radio), ct.c_double, dp, dp, dp, dp,
                                              ct.c_double, dp, dp, dp]
        L.ora_sum.restype = ct.c_double
        L.ora_sum.argtypes = [dp, i64]
        _lib = L
    return _lib


def _d(x):
    return x.ctypes.data_as(ct.POINTER(ct.c_double)) if x is not None else None


def _c64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def radio_struct(layout) -> _Radio:
    r = layout.radio
    return _Radio(r["tx_power_w"], r["ref_gain"], r["pathloss_exp"], r["min_dist_m"], r["shadow_sigma_db"],
                  r["noise_w"], r["bandwidth_hz"], ct.c_uint64(layout.shadow_key & (2**64 - 1)))


def splitmix64(x: int) -> int:
    return int(lib().ora_splitmix64(ct.c_uint64(x & (2**64 - 1))))


def shadow_normal(key: int, i: int, j: int) -> float:
    return float(lib().ora_shadow_normal(ct.c_uint64(key & (2**64 - 1)), i, j))


def rates_rows(layout, rows) -> np.ndarray:
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    dev = np.ascontiguousarray(layout.dev_xy, dtype=np.float32)
    rrh = np.ascontiguousarray(layout.rrh_xy, dtype=np.float32)
    out = np.empty((rows.size, layout.J))
    rad = radio_struct(layout)
    st = lib().ora_rates_rows(dev.ctypes.data_as(ct.POINTER(ct.c_float)), rrh.ctypes.data_as(ct.POINTER(ct.c_float)),
                              layout.J, ct.byref(rad), rows.ctypes.data_as(ct.POINTER(ct.c_int64)), rows.size, _d(out))
    if st != OK:
        raise RuntimeError(f"ora_rates_rows failed: {st}")
    return out


def rates(layout) -> np.ndarray:
    return rates_rows(layout, np.arange(layout.I))


def lower_median(x) -> float:
    x = _c64(x).ravel()
    return float(lib().ora_lower_median(_d(x), x.size))


def cost(layout, scale: float = 0.0, R=None):
    """Returns (C, scale). scale <= 0 means: the lower median of 1/R."""
    R = _c64(rates(layout) if R is None else R)
    C = np.empty_like(R)
    s = ct.c_double(scale)
    st = lib().ora_cost_from_rates(_d(R), R.size, ct.byref(s), _d(C))
    if st != OK:
        raise RuntimeError(f"ora_cost_from_rates failed: {st}")
    return C, float(s.value)


def cost_rows(layout, rows, scale: float) -> np.ndarray:
    """Cost rows for a given (already known) scale, e.g. a sample of a large instance."""
    if not scale > 0:
        raise ValueError("cost_rows needs the scale")
    return (1.0 / rates_rows(layout, rows)) / scale


def distance_cost(layout, scale: float = 1.0):
    """Returns (C, scale) with C_ij = ||x_i - X_j|| / scale, the distance
    between device i and RRH j (Sec. IV, cost choice (i)). The positions are
    the layout's FP32 coordinates, taken exactly into FP64; the distance is
    the plain FP64 square root of the summed squared differences. scale <= 0
    means: the lower median of the distances."""
    dev = np.asarray(layout.dev_xy, dtype=np.float32).astype(np.float64)
    rrh = np.asarray(layout.rrh_xy, dtype=np.float32).astype(np.float64)
    dx = dev[:, 0][:, None] - rrh[:, 0][None, :]
    dy = dev[:, 1][:, None] - rrh[:, 1][None, :]
    D = np.sqrt(dx * dx + dy * dy)
    if not scale > 0:
        scale = lower_median(D)
    return D / scale, float(scale)


class SinkhornResult:
    def __init__(self, status, f, g, iters, residual, hist):
        self.status, self.f, self.g, self.iters, self.residual, self.hist = status, f, g, iters, residual, hist

    def __repr__(self):
        return f"SinkhornResult(status={self.status}, iters={self.iters}, residual={self.residual:.3e})"


def sinkhorn(C, a, b, eps, tol, max_iter, g0=None, history=False) -> SinkhornResult:
    C, a, b = _c64(C), _c64(a), _c64(b)
    I, J = C.shape
    f, g = np.empty(I), np.empty(J)
    r, it = ct.c_double(0.0), ct.c_int32(0)
    hist = np.full(max_iter, np.nan) if history else None
    g0 = None if g0 is None else _c64(g0)
    st = lib().ora_sinkhorn(_d(C), I, J, _d(a), _d(b), eps, tol, max_iter, _d(g0), _d(f), _d(g), ct.byref(r),
                            ct.byref(it), _d(hist))
    if st < 0:
        raise ValueError(f"ora_sinkhorn rejected its inputs (status {st})")
    if hist is not None:
        hist = hist[: it.value]
    return SinkhornResult(st, f, g, it.value, r.value, hist)


def plan(C, f, g, eps) -> np.ndarray:
    C, f, g = _c64(C), _c64(f), _c64(g)
    pi = np.empty_like(C)
    st = lib().ora_plan(_d(C), C.shape[0], C.shape[1], _d(f), _d(g), eps, _d(pi))
    if st != OK:
        raise ValueError(f"ora_plan failed: {st}")
    return pi


def plan_stats(C, a, b, f, g, eps) -> dict:
    C, a, b, f, g = _c64(C), _c64(a), _c64(b), _c64(f), _c64(g)
    I, J = C.shape
    out, rs, cs = np.empty(5), np.empty(I), np.empty(J)
    st = lib().ora_plan_stats(_d(C), I, J, _d(a), _d(b), _d(f), _d(g), eps, _d(out), _d(rs), _d(cs))
    if st != OK:
        raise ValueError(f"ora_plan_stats failed: {st}")
    return dict(marginal_violation=out[0], objective=out[1], reg_objective=out[2], dual_objective=out[3],
                mass=out[4], row_sums=rs, col_sums=cs)


def geometry_plan_stats(layout, scale, f, g, eps) -> dict:
    """Statistics of pi = exp((f + g - C)/eps) for the rate cost
    C = (1/R) / scale of a layout, regenerated row by row (the cost is never
    held whole, so this also serves instances too large for ``cost``):
    marginal violation, transport cost <C, pi>, mass, row and column sums."""
    dev = np.ascontiguousarray(layout.dev_xy, dtype=np.float32)
    rrh = np.ascontiguousarray(layout.rrh_xy, dtype=np.float32)
    a, b, f, g = _c64(layout.a), _c64(layout.b), _c64(f), _c64(g)
    out, rs, cs = np.empty(3), np.empty(layout.I), np.empty(layout.J)
    rad = radio_struct(layout)
    st = lib().ora_geometry_plan_stats(dev.ctypes.data_as(ct.POINTER(ct.c_float)),
                                       rrh.ctypes.data_as(ct.POINTER(ct.c_float)), layout.I, layout.J, ct.byref(rad),
                                       float(scale), _d(a), _d(b), _d(f), _d(g), float(eps), _d(out), _d(rs), _d(cs))
    if st != OK:
        raise ValueError(f"ora_geometry_plan_stats failed: {st}")
    return dict(marginal_violation=out[0], objective=out[1], mass=out[2], row_sums=rs, col_sums=cs)


def osum(x) -> float:
    x = _c64(x).ravel()
    return float(lib().ora_sum(_d(x), x.size))


# --------------------------------------------------------------- helpers --

def brute_force_ot(C) -> tuple[float, tuple]:
    """Unregularised OT of eqs. (2)-(4) for a square n x n cost with uniform
    marginals 1/n: by Birkhoff's theorem an optimal plan is a permutation
    matrix divided by n, so enumerate all permutations. Returns (value, sigma)."""
    C = np.asarray(C, dtype=np.float64)
    n = C.shape[0]
    if C.shape != (n, n) or n > 9:
        raise ValueError("brute force is for square instances with n <= 9")
    best, arg = np.inf, None
    rows = np.arange(n)
    for perm in itertools.permutations(range(n)):
        v = C[rows, perm].sum() / n
        if v < best:
            best, arg = v, perm
    return float(best), arg


def maxsinr_association(R) -> np.ndarray:
    """maxSINR rule (Sec. II-A / IV): each device to its highest-rate RRH,
    lowest index on ties. Returns the RRH index per device."""
    return np.argmax(np.asarray(R), axis=1)


def maxsinr_traffic(R, lam) -> np.ndarray:
    """Lambda_j = sum_i pi^SINR_ij lambda_i: the RRH traffic under maxSINR."""
    R = np.asarray(R)
    out = np.zeros(R.shape[1])
    np.add.at(out, maxsinr_association(R), np.asarray(lam, dtype=np.float64))
    return out


def lemma1_lower_bound(C, a) -> float:
    """Every coupling with row sums a pays at least sum_i a_i min_j C_ij; with
    q = maxSINR traffic and C = 1/R this bound is attained (Lemma 1)."""
    C = np.asarray(C, dtype=np.float64)
    return osum(np.asarray(a, dtype=np.float64) * C.min(axis=1))


def entropy(x) -> float:
    x = np.asarray(x, dtype=np.float64)
    x = x[x > 0]
    return float(-(x * np.log(x)).sum())


# ------------------------------------------------------ loads (Sec. II-B) --

def rrh_loads(C, f, g, eps) -> np.ndarray:
    """Per-RRH load of the transport plan x = exp((f + g - C)/eps):
    sum_i C_ij x_ij. With C = 1/(mu R) scaled by a constant and the
    association pi_ij = x_ij / a_i (Lemma 1's pi* = x* / lambda), this is
    Sec. II-B's rho_j = sum_i lambda_i pi_ij / (mu R_ij) up to the factor
    sum(lambda) scale / mu. Column sums are compensated (osum)."""
    C = _c64(C)
    P = plan(C, f, g, eps)
    return np.array([osum(C[:, j] * P[:, j]) for j in range(C.shape[1])])


def evaluate(C, f, g, eps, a, kappa, tau) -> dict:
    """Association quality of the plan x = exp((f + g - C)/eps) with row sums
    a (Sec. II-B), for a cost C = (1/R) / scale:
      rho_j   = kappa sum_i C_ij x_ij             (kappa = sum(lambda) scale / mu)
      E[N_j]  = rho_j / (1 - rho_j) if rho_j < 1, else inf   (processor sharing)
      T_i     = (tau / a_i) sum_j C_ij x_ij / (1 - rho_j)    (tau = scale / mu),
    the average completion time of device i (sum over its associations of
    pi_ij / (mu R_ij (1 - rho_j)) with pi_ij = x_ij / a_i); inf if it uses an
    overloaded RRH. Returns rho, EN, T (per device), T_mean and the objective
    of eq. (1), sum_i T_i."""
    C, a = _c64(C), _c64(a)
    P = plan(C, f, g, eps)
    rho = kappa * np.array([osum(C[:, j] * P[:, j]) for j in range(C.shape[1])])
    over = rho >= 1.0
    EN = np.where(over, np.inf, rho / np.where(over, 1.0, 1.0 - rho))
    T = np.empty(C.shape[0])
    for i in range(C.shape[0]):
        if np.any(over & (P[i] > 0)):
            T[i] = np.inf
        else:
            T[i] = tau / a[i] * osum(C[i] * P[i] / (1.0 - rho))
    return dict(rho=rho, EN=EN, T=T, T_mean=osum(T) / T.size if np.all(np.isfinite(T)) else np.inf,
                objective=osum(T) if np.all(np.isfinite(T)) else np.inf)


# ------------------------------------------- Adaptive Sinkhorn (Alg. 2) --

def adaptive_sinkhorn(C, a, eps, tol, max_iter, delta=None, max_outer=100) -> dict:
    """Adaptive Sinkhorn Association (Sec. IV, Alg. 2) on cost C (load per
    unit traffic) with device traffic a:
      q <- sum(a) / J for every RRH;
      repeat: x <- Sinkhorn(C, a, q, eps); j* <- argmax_j rho_j(x);
              q_j* <- q_j* - delta, q_j <- q_j + delta / (J - 1) for j != j*.
    Readings (the paper leaves them open): delta = 0.01 sum(a) / J; each
    Sinkhorn solve runs to the total residual tol; j* is the lowest index
    among equal loads; the loop ends when the maximum load of a new solve
    does not fall below the best one so far, when q_j* - delta would not stay
    positive, or after max_outer solves; the returned association is the one
    with the lowest maximum load (the last one that lowered it), with the q it
    was solved for. J = 1 has nothing to rebalance: one solve.
    Returns q, f, g, max_load, loads, solves (Sinkhorn solves run), outer
    (the index of the returned solve) and the per-solve history of (j*, max load)."""
    C, a = _c64(C), _c64(a)
    J = C.shape[1]
    mass = osum(a)
    d = 0.01 * mass / J if delta is None else float(delta)
    q = np.full(J, mass / J)
    best, hist = None, []
    for k in range(max_outer):
        r = sinkhorn(C, a, q, eps, tol, max_iter)
        loads = rrh_loads(C, r.f, r.g, eps)
        js = int(np.argmax(loads))
        mx = float(loads[js])
        hist.append((js, mx))
        if best is not None and not mx < best["max_load"]:
            break
        best = dict(q=q.copy(), f=r.f, g=r.g, max_load=mx, loads=loads, outer=k, iters=r.iters)
        if J < 2 or not q[js] - d > 0.0:
            break
        step = d / (J - 1)
        nq = q + step
        nq[js] = q[js] - d
        q = nq
    best["solves"] = len(hist)
    best["history"] = hist
    return best
