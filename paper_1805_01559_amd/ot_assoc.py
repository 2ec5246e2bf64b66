"""ctypes binding of the HIP association library (include/ot_assoc.h).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels. The functions keep the C names (ot_assoc_create, ot_assoc_solve,
ot_assoc_plan, ...); ``Solver`` wraps them for numpy arrays and torch tensors.
There is no fallback: if libot_assoc.so is missing or no GPU is present, the
calls raise.
"""

from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libot_assoc.so")

# ot_status
OT_OK, OT_WARN_MAXITER, OT_EINVAL, OT_ENOMEM, OT_EDEVICE, OT_ENUMERIC, OT_ESTATE = 0, 1, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "OT_OK", 1: "OT_WARN_MAXITER", -1: "OT_EINVAL", -2: "OT_ENOMEM", -3: "OT_EDEVICE",
                -4: "OT_ENUMERIC", -5: "OT_ESTATE"}
OT_COST_DENSE, OT_COST_RATES, OT_COST_GEOMETRY, OT_COST_EUCLID = 0, 1, 2, 3
OT_MEM_HOST, OT_MEM_DEVICE = 0, 1
OT_F32, OT_F64 = 0, 1
OT_PREC_FP32, OT_PREC_FP64 = 0, 1
OT_RESULT_PERSISTENT = 1
OT_RESULT_CHECK_ABOVE_TOL = 2

# every symbol include/ot_assoc.h declares
EXPORTS = [
    "ot_assoc_default_options", "ot_assoc_workspace_size", "ot_assoc_device_allocations", "ot_assoc_create",
    "ot_assoc_solve_static", "ot_assoc_solve", "ot_assoc_plan", "ot_assoc_set_plan_output", "ot_assoc_potentials",
    "ot_assoc_set_potentials", "ot_assoc_cost_median", "ot_assoc_materialize_cost", "ot_assoc_time_sweep", "ot_assoc_time_read",
    "ot_assoc_test_hold_exchange",
    "ot_assoc_fast_phase_time", "ot_assoc_rrh_loads", "ot_assoc_evaluate", "ot_assoc_maxsinr", "ot_assoc_adaptive",
    "ot_assoc_destroy", "ot_assoc_last_error", "ot_assoc_solve_batch", "ot_assoc_batch_config",
    "ot_assoc_batch_potentials", "ot_assoc_solve_snapshots", "ot_assoc_snapshot_potentials",
    "ot_assoc_batch_plan", "ot_serve_default_options", "ot_serve_create", "ot_serve_submit", "ot_serve_progress",
    "ot_serve_counts", "ot_serve_potentials", "ot_serve_now", "ot_serve_last_error", "ot_serve_destroy",
]


class ot_geometry(ct.Structure):
    _fields_ = [("dev_xy", ct.c_void_p), ("rrh_xy", ct.c_void_p), ("tx_power_w", ct.c_double),
                ("ref_gain", ct.c_double), ("pathloss_exp", ct.c_double), ("min_dist_m", ct.c_double),
                ("shadow_sigma_db", ct.c_double), ("noise_w", ct.c_double), ("bandwidth_hz", ct.c_double),
                ("shadow_key", ct.c_uint64)]


class ot_cost_desc(ct.Structure):
    _fields_ = [("kind", ct.c_int), ("I", ct.c_int64), ("J", ct.c_int64), ("mem", ct.c_int), ("dtype", ct.c_int),
                ("data", ct.c_void_p), ("scale", ct.c_double), ("geom", ot_geometry), ("ld", ct.c_int64)]


class ot_assoc_options(ct.Structure):
    _fields_ = [("device", ct.c_int), ("stream", ct.c_void_p), ("precision", ct.c_int), ("polish_iters", ct.c_int),
                ("chunk", ct.c_int), ("use_graphs", ct.c_int), ("sweep_blocks", ct.c_int), ("sweep_waves", ct.c_int),
                ("sweep_rows", ct.c_int), ("sweep_lanes", ct.c_int), ("batch_tune", ct.c_int),
                ("persistent", ct.c_int), ("check_every", ct.c_int), ("workspace", ct.c_void_p),
                ("workspace_bytes", ct.c_size_t), ("snapshot_k_split", ct.c_int)]


class ot_assoc_result(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("fp64_iterations", ct.c_int32), ("status", ct.c_int32),
                ("flags", ct.c_int32), ("marginal_violation", ct.c_double), ("objective", ct.c_double),
                ("reg_objective", ct.c_double), ("dual_objective", ct.c_double), ("seconds", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ot_eval_result(ct.Structure):
    _fields_ = [("max_rho", ct.c_double), ("mean_completion", ct.c_double), ("objective", ct.c_double),
                ("overloaded_rrhs", ct.c_int32), ("devices_overloaded", ct.c_int32)]


class ot_adaptive_result(ct.Structure):
    _fields_ = [("solves", ct.c_int32), ("best", ct.c_int32), ("iterations", ct.c_int32), ("status", ct.c_int32),
                ("max_load", ct.c_double), ("first_max_load", ct.c_double), ("delta", ct.c_double)]


class ot_serve_options(ct.Structure):
    _fields_ = [("device", ct.c_int), ("stream", ct.c_void_p), ("budget_bytes", ct.c_double), ("max_slots", ct.c_int),
                ("max_items", ct.c_int), ("polish_iters", ct.c_int), ("sweep_waves", ct.c_int),
                ("rows_per_part", ct.c_int), ("keep_layouts", ct.c_int)]


class ot_request(ct.Structure):
    _fields_ = [("cost", ot_cost_desc), ("a", ct.c_void_p), ("b", ct.c_void_p), ("eps", ct.c_double),
                ("tol", ct.c_double), ("max_iter", ct.c_int32), ("reserved", ct.c_int32),
                ("layout_key", ct.c_uint64), ("user_tag", ct.c_uint64)]


class ot_completion(ct.Structure):
    _fields_ = [("ticket", ct.c_uint64), ("user_tag", ct.c_uint64), ("layout_key", ct.c_uint64),
                ("warm", ct.c_int32), ("reserved", ct.c_int32), ("t_submit", ct.c_double),
                ("t_admit", ct.c_double), ("t_done", ct.c_double), ("result", ot_assoc_result)]


_lib = None


def lib():
    """The loaded library. Raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_1805_01559_amd.build.build()")
        L = ct.CDLL(LIB_PATH)
        vp, i64, d = ct.c_void_p, ct.c_int64, ct.c_double
        L.ot_assoc_default_options.argtypes = [ct.POINTER(ot_assoc_options)]
        L.ot_assoc_create.argtypes = [ct.POINTER(vp), i64, i64, ct.POINTER(ot_assoc_options)]
        L.ot_assoc_workspace_size.argtypes = [i64, i64, ct.POINTER(ct.c_size_t)]
        L.ot_assoc_device_allocations.argtypes = []
        L.ot_assoc_solve.argtypes = [vp, ct.POINTER(ot_cost_desc), vp, vp, d, d, ct.c_int32, ct.c_int,
                                     ct.POINTER(ot_assoc_result)]
        L.ot_assoc_solve_static.argtypes = [ct.c_int, vp, vp, i64, i64, i64, vp, vp, d, d, ct.c_int32, ct.c_int, vp,
                                            vp, ct.POINTER(ot_assoc_result)]
        L.ot_assoc_plan.argtypes = [vp, vp, ct.c_int, ct.c_int]
        L.ot_assoc_set_plan_output.argtypes = [vp, vp, ct.c_int, ct.c_int64]
        L.ot_assoc_potentials.argtypes = [vp, vp, vp, ct.c_int]
        L.ot_assoc_set_potentials.argtypes = [vp, vp, vp, i64, i64, ct.c_int]
        L.ot_assoc_cost_median.argtypes = [vp, ct.POINTER(ot_cost_desc), ct.POINTER(d)]
        L.ot_assoc_materialize_cost.argtypes = [vp, ct.POINTER(ot_cost_desc), vp]
        L.ot_assoc_time_sweep.argtypes = [vp, ct.c_int32, ct.c_int, ct.POINTER(d)]
        L.ot_assoc_time_read.argtypes = [vp, vp, ct.c_size_t, ct.c_int32, ct.POINTER(d)]
        L.ot_assoc_test_hold_exchange.argtypes = [ct.c_int32]
        L.ot_assoc_fast_phase_time.argtypes = [vp, ct.POINTER(d), ct.POINTER(ct.c_int32)]
        L.ot_assoc_rrh_loads.argtypes = [vp, vp, ct.c_int]
        L.ot_assoc_evaluate.argtypes = [vp, d, d, vp, vp, ct.c_int, ct.POINTER(ot_eval_result)]
        L.ot_assoc_maxsinr.argtypes = [vp, ct.POINTER(ot_cost_desc), vp, vp, vp]
        L.ot_assoc_adaptive.argtypes = [vp, ct.POINTER(ot_cost_desc), vp, d, d, ct.c_int32, d, ct.c_int32, vp, vp,
                                        ct.POINTER(ot_adaptive_result)]
        L.ot_assoc_destroy.argtypes = [vp]
        L.ot_assoc_destroy.restype = None
        L.ot_assoc_last_error.argtypes = [vp]
        L.ot_assoc_last_error.restype = ct.c_char_p
        PP = ct.POINTER(ct.c_void_p)
        L.ot_assoc_solve_batch.argtypes = [vp, ct.c_int, ct.POINTER(ot_cost_desc), PP, PP, ct.POINTER(d), d,
                                           ct.c_int32, ct.POINTER(ot_assoc_result)]
        L.ot_assoc_batch_config.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int)]
        L.ot_assoc_batch_potentials.argtypes = [vp, ct.c_int, vp, vp, ct.c_int]
        L.ot_assoc_solve_snapshots.argtypes = [vp, ct.POINTER(ot_cost_desc), ct.c_int, vp, vp, d, d, ct.c_int32,
                                               ct.POINTER(ot_assoc_result)]
        L.ot_assoc_snapshot_potentials.argtypes = [vp, ct.c_int, vp, vp, ct.c_int]
        L.ot_assoc_batch_plan.argtypes = [vp, ct.c_int, vp, ct.c_int, ct.c_int]
        L.ot_serve_default_options.argtypes = [ct.POINTER(ot_serve_options)]
        L.ot_serve_create.argtypes = [ct.POINTER(vp), ct.POINTER(ot_serve_options)]
        L.ot_serve_submit.argtypes = [vp, ct.POINTER(ot_request), ct.POINTER(ct.c_uint64)]
        L.ot_serve_progress.argtypes = [vp, ct.POINTER(ot_completion), ct.c_int, ct.POINTER(ct.c_int)]
        L.ot_serve_counts.argtypes = [vp, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), ct.POINTER(ct.c_int),
                                      ct.POINTER(d)]
        L.ot_serve_potentials.argtypes = [vp, ct.c_uint64, vp, vp, ct.c_int]
        L.ot_serve_now.argtypes = []
        L.ot_serve_now.restype = d
        L.ot_serve_last_error.argtypes = [vp]
        L.ot_serve_last_error.restype = ct.c_char_p
        L.ot_serve_destroy.argtypes = [vp]
        L.ot_serve_destroy.restype = None
        for name in EXPORTS:
            if name not in ("ot_assoc_destroy", "ot_assoc_last_error", "ot_serve_now", "ot_serve_last_error",
                            "ot_serve_destroy", "ot_assoc_device_allocations"):
                getattr(L, name).restype = ct.c_int
        L.ot_assoc_device_allocations.restype = ct.c_int64
        _lib = L
    return _lib


class OTError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


# ------------------------------------------------------------- C names ----

def ot_assoc_default_options() -> ot_assoc_options:
    o = ot_assoc_options()
    lib().ot_assoc_default_options(ct.byref(o))
    return o


def ot_assoc_last_error(h) -> str:
    s = lib().ot_assoc_last_error(h)
    return s.decode() if s else ""


def _check(h, st):
    if st < 0:
        raise OTError(st, ot_assoc_last_error(h))
    return st


def ot_assoc_create(I_max: int, J_max: int, options: ot_assoc_options | None = None):
    h = ct.c_void_p()
    st = lib().ot_assoc_create(ct.byref(h), I_max, J_max, ct.byref(options) if options is not None else None)
    _check(None, st)
    return h


def ot_assoc_workspace_size(I_max: int, J_max: int) -> int:
    n = ct.c_size_t()
    _check(None, lib().ot_assoc_workspace_size(I_max, J_max, ct.byref(n)))
    return n.value


def ot_assoc_device_allocations() -> int:
    return int(lib().ot_assoc_device_allocations())


def ot_assoc_test_hold_exchange(iteration: int) -> int:
    """Test hook: the calling thread's next cooperative FP32 launch withholds
    g at that iteration so its waits give up (the solve returns OT_EDEVICE)."""
    return int(lib().ot_assoc_test_hold_exchange(int(iteration)))


def ot_assoc_solve(h, desc: ot_cost_desc, a_ptr, b_ptr, eps, tol, max_iter, warm_start=0):
    res = ot_assoc_result()
    st = lib().ot_assoc_solve(h, ct.byref(desc), a_ptr, b_ptr, float(eps), float(tol), int(max_iter), int(warm_start),
                              ct.byref(res))
    _check(h, st)
    return st, res


def ot_assoc_solve_static(C, a, b, f, g, eps, tol, max_iter, warm_start=0, device=0, stream=None, J=None):
    """The no-allocation solve. C is an (I, ld) FP32 torch device tensor whose
    first J columns (default: all) are the cost; a, b, f, g are FP64 device
    tensors of I, J, I, J elements; f and g receive the potentials (and hold
    the starting ones when warm_start). Returns (status, result)."""
    I, ld = int(C.shape[0]), int(C.shape[1])
    J = ld if J is None else int(J)
    res = ot_assoc_result()
    st = lib().ot_assoc_solve_static(int(device), stream, ct.c_void_p(C.data_ptr()), I, J, ld,
                                     ct.c_void_p(a.data_ptr()), ct.c_void_p(b.data_ptr()), float(eps), float(tol),
                                     int(max_iter), int(warm_start), ct.c_void_p(f.data_ptr()),
                                     ct.c_void_p(g.data_ptr()), ct.byref(res))
    _check(None, st)
    return st, res


def ot_assoc_plan(h, pi_ptr, mem, dtype):
    return _check(h, lib().ot_assoc_plan(h, pi_ptr, mem, dtype))


def ot_assoc_potentials(h, f_ptr, g_ptr, mem):
    return _check(h, lib().ot_assoc_potentials(h, f_ptr, g_ptr, mem))


def ot_assoc_set_potentials(h, f_ptr, g_ptr, I, J, mem):
    return _check(h, lib().ot_assoc_set_potentials(h, f_ptr, g_ptr, I, J, mem))


def ot_assoc_cost_median(h, desc: ot_cost_desc) -> float:
    m = ct.c_double()
    _check(h, lib().ot_assoc_cost_median(h, ct.byref(desc), ct.byref(m)))
    return m.value


def ot_assoc_materialize_cost(h, desc: ot_cost_desc, C_ptr):
    return _check(h, lib().ot_assoc_materialize_cost(h, ct.byref(desc), C_ptr))


def ot_assoc_time_sweep(h, reps: int, fp64: bool = False) -> float:
    ms = ct.c_double()
    _check(h, lib().ot_assoc_time_sweep(h, int(reps), int(bool(fp64)), ct.byref(ms)))
    return ms.value


def ot_assoc_fast_phase_time(h):
    """(ms, iterations) of the last solve's cooperative FP32 launch."""
    ms, it = ct.c_double(), ct.c_int32()
    _check(h, lib().ot_assoc_fast_phase_time(h, ct.byref(ms), ct.byref(it)))
    return ms.value, it.value


def ot_assoc_destroy(h):
    if h:
        lib().ot_assoc_destroy(h)


def ot_assoc_solve_batch(h, descs, a_ptrs, b_ptrs, eps, tol, max_iter):
    n = len(descs)
    D = (ot_cost_desc * n)(*descs)
    A = (ct.c_void_p * n)(*a_ptrs)
    B = (ct.c_void_p * n)(*b_ptrs)
    E = (ct.c_double * n)(*[float(e) for e in eps])
    R = (ot_assoc_result * n)()
    st = lib().ot_assoc_solve_batch(h, n, D, A, B, E, float(tol), int(max_iter), R)
    _check(h, st)
    return st, list(R)


def ot_assoc_batch_config(h):
    w, r = ct.c_int(), ct.c_int()
    _check(h, lib().ot_assoc_batch_config(h, ct.byref(w), ct.byref(r)))
    return w.value, r.value


def ot_assoc_batch_potentials(h, k, f_ptr, g_ptr, mem):
    return _check(h, lib().ot_assoc_batch_potentials(h, int(k), f_ptr, g_ptr, mem))


def ot_assoc_batch_plan(h, k, pi_ptr, mem, dtype):
    return _check(h, lib().ot_assoc_batch_plan(h, int(k), pi_ptr, mem, dtype))


def ot_assoc_solve_snapshots(h, desc, B, A_ptr, b_ptr, eps, tol, max_iter):
    R = (ot_assoc_result * B)()
    st = lib().ot_assoc_solve_snapshots(h, ct.byref(desc), int(B), A_ptr, b_ptr, float(eps), float(tol),
                                        int(max_iter), R)
    _check(h, st)
    return st, list(R)


def ot_assoc_snapshot_potentials(h, s, f_ptr, g_ptr, mem):
    return _check(h, lib().ot_assoc_snapshot_potentials(h, int(s), f_ptr, g_ptr, mem))


def ot_serve_default_options() -> ot_serve_options:
    o = ot_serve_options()
    lib().ot_serve_default_options(ct.byref(o))
    return o


def ot_serve_last_error(s) -> str:
    m = lib().ot_serve_last_error(s)
    return m.decode() if m else ""


def _scheck(s, st):
    if st < 0:
        raise OTError(st, ot_serve_last_error(s))
    return st


def ot_serve_create(options: ot_serve_options | None = None):
    s = ct.c_void_p()
    st = lib().ot_serve_create(ct.byref(s), ct.byref(options) if options is not None else None)
    if st < 0:
        raise OTError(st, "ot_serve_create failed")
    return s


def ot_serve_submit(s, req: ot_request) -> int:
    t = ct.c_uint64()
    _scheck(s, lib().ot_serve_submit(s, ct.byref(req), ct.byref(t)))
    return t.value


def ot_serve_progress(s, max_out: int = 256):
    out = (ot_completion * max_out)()
    n = ct.c_int()
    _scheck(s, lib().ot_serve_progress(s, out, max_out, ct.byref(n)))
    return [out[q] for q in range(n.value)]


def ot_serve_counts(s):
    q, r, k, b = ct.c_int(), ct.c_int(), ct.c_int(), ct.c_double()
    _scheck(s, lib().ot_serve_counts(s, ct.byref(q), ct.byref(r), ct.byref(k), ct.byref(b)))
    return q.value, r.value, k.value, b.value


def ot_serve_potentials(s, key, f_ptr, g_ptr, mem):
    return _scheck(s, lib().ot_serve_potentials(s, int(key), f_ptr, g_ptr, mem))


def ot_serve_now() -> float:
    return lib().ot_serve_now()


def ot_serve_destroy(s):
    if s:
        lib().ot_serve_destroy(s)


# ---------------------------------------------------------- marshalling ----

def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr_mem(x, dtype):
    """(pointer, memory space, keepalive) for a numpy array or torch tensor."""
    if _is_torch(x):
        if not x.is_contiguous():
            raise ValueError("tensors must be contiguous")
        want = {np.float32: "torch.float32", np.float64: "torch.float64"}[dtype]
        if str(x.dtype) != want:
            raise TypeError(f"expected {want}, got {x.dtype}")
        return x.data_ptr(), (OT_MEM_DEVICE if x.is_cuda else OT_MEM_HOST), x
    arr = np.ascontiguousarray(x, dtype=dtype)
    return arr.ctypes.data, OT_MEM_HOST, arr


@dataclass
class Radio:
    tx_power_w: float
    ref_gain: float
    pathloss_exp: float
    min_dist_m: float
    shadow_sigma_db: float
    noise_w: float
    bandwidth_hz: float


def geometry_desc(dev_xy, rrh_xy, radio: dict, shadow_key: int, scale: float = 1.0):
    """Descriptor of an on-the-fly geometry cost (Sec. II-A rates, Sec. IV cost (ii))."""
    pd, md, kd = _ptr_mem(dev_xy, np.float32)
    pr, mr, kr = _ptr_mem(rrh_xy, np.float32)
    if md != mr:
        raise ValueError("device and RRH positions must live in the same memory space")
    d = ot_cost_desc()
    d.kind, d.mem, d.dtype = OT_COST_GEOMETRY, md, OT_F32
    d.I, d.J = int(dev_xy.shape[0]), int(rrh_xy.shape[0])
    d.scale = float(scale)
    g = d.geom
    g.dev_xy, g.rrh_xy = pd, pr
    for k in ("tx_power_w", "ref_gain", "pathloss_exp", "min_dist_m", "shadow_sigma_db", "noise_w", "bandwidth_hz"):
        setattr(g, k, float(radio[k]))
    g.shadow_key = int(shadow_key) & (2**64 - 1)
    return d, (kd, kr)


def euclid_desc(dev_xy, rrh_xy, scale: float = 1.0):
    """Descriptor of an on-the-fly distance cost C_ij = ||x_i - X_j|| / scale
    (Sec. IV, cost choice (i))."""
    pd, md, kd = _ptr_mem(dev_xy, np.float32)
    pr, mr, kr = _ptr_mem(rrh_xy, np.float32)
    if md != mr:
        raise ValueError("device and RRH positions must live in the same memory space")
    d = ot_cost_desc()
    d.kind, d.mem, d.dtype = OT_COST_EUCLID, md, OT_F32
    d.I, d.J = int(dev_xy.shape[0]), int(rrh_xy.shape[0])
    d.scale = float(scale)
    d.geom.dev_xy, d.geom.rrh_xy = pd, pr
    return d, (kd, kr)


def matrix_desc(M, kind=OT_COST_DENSE, scale: float = 1.0, J=None):
    """Descriptor of a dense cost (or rate) matrix. With J given, M is an
    (I, ld) row-padded buffer of which the first J columns are the instance."""
    dt = np.float32 if (str(getattr(M, "dtype", "")) in ("float32", "torch.float32")) else np.float64
    p, m, keep = _ptr_mem(M, dt)
    d = ot_cost_desc()
    d.kind, d.mem, d.dtype = kind, m, (OT_F32 if dt == np.float32 else OT_F64)
    d.I, d.J = int(M.shape[0]), int(M.shape[1] if J is None else J)
    d.ld = 0 if J is None else int(M.shape[1])
    if d.J > int(M.shape[1]):
        raise ValueError("J exceeds the buffer's row length")
    d.data, d.scale = p, float(scale)
    return d, (keep,)


class Solver:
    """One solver handle. Inputs may be numpy arrays (host) or torch tensors
    (host or device); a and b must be in the same memory space as the cost."""

    def __init__(self, I_max, J_max, precision=OT_PREC_FP32, device=0, stream=None, **opts):
        o = ot_assoc_default_options()
        o.device = device
        o.precision = precision
        o.stream = stream
        for k, v in opts.items():
            setattr(o, k, v)
        self.h = ot_assoc_create(I_max, J_max, o)
        self.I_max, self.J_max = I_max, J_max
        self._I = self._J = None
        self._snap_dims = None

    def close(self):
        h = getattr(self, "h", None)
        self.h = None
        if h:
            try:
                ot_assoc_destroy(h)
            except Exception:  # interpreter shutdown: the module may be half torn down
                pass

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def solve(self, desc, keep, a, b, eps, tol, max_iter, warm_start=False):
        pa, ma, ka = _ptr_mem(a, np.float64)
        pb, mb, kb = _ptr_mem(b, np.float64)
        if ma != desc.mem or mb != desc.mem:
            raise ValueError("a and b must be in the cost's memory space")
        st, res = ot_assoc_solve(self.h, desc, pa, pb, eps, tol, max_iter, int(warm_start))
        self._I, self._J = desc.I, desc.J
        del keep, ka, kb
        return st, res

    # ---- association quality (Sec. II-B), maxSINR (Sec. IV), Alg. 2 ----
    def rrh_loads(self):
        """load_j = sum_i C_ij x_ij of the last solve's plan (J doubles, host)."""
        out = np.empty(self._J, np.float64)
        _check(self.h, lib().ot_assoc_rrh_loads(self.h, out.ctypes.data, OT_MEM_HOST))
        return out

    def evaluate(self, kappa, tau):
        """(rho, E[N], ot_eval_result) of the last solve: rho = kappa load,
        E[N] = rho / (1 - rho), device completion times with tau."""
        rho = np.empty(self._J, np.float64)
        en = np.empty(self._J, np.float64)
        r = ot_eval_result()
        _check(self.h, lib().ot_assoc_evaluate(self.h, float(kappa), float(tau), rho.ctypes.data, en.ctypes.data,
                                               OT_MEM_HOST, ct.byref(r)))
        return rho, en, r

    def maxsinr(self, desc, keep, a):
        """(association per device, Lambda per RRH) of the maxSINR rule; a in
        the cost's memory space; host numpy results."""
        pa, ma, ka = _ptr_mem(a, np.float64)
        if ma != desc.mem:
            raise ValueError("a must be in the cost's memory space")
        if desc.mem == OT_MEM_HOST:
            assoc = np.empty(desc.I, np.int32)
            lam = np.empty(desc.J, np.float64)
            _check(self.h, lib().ot_assoc_maxsinr(self.h, ct.byref(desc), pa, assoc.ctypes.data, lam.ctypes.data))
            return assoc, lam
        import torch
        assoc = torch.empty(desc.I, dtype=torch.int32, device=a.device)
        lam = torch.empty(desc.J, dtype=torch.float64, device=a.device)
        _check(self.h, lib().ot_assoc_maxsinr(self.h, ct.byref(desc), pa, assoc.data_ptr(), lam.data_ptr()))
        del keep, ka
        return assoc.cpu().numpy(), lam.cpu().numpy()

    def adaptive(self, desc, keep, a, eps, tol=1e-8, max_iter=2000, delta=0.0, max_outer=100):
        """Adaptive Sinkhorn Association (Alg. 2). Returns (status, q, j* per
        solve, ot_adaptive_result); the handle then holds the best solve."""
        pa, ma, ka = _ptr_mem(a, np.float64)
        if ma != desc.mem:
            raise ValueError("a must be in the cost's memory space")
        q = np.empty(desc.J, np.float64)
        js = np.full(max_outer, -1, np.int32)
        r = ot_adaptive_result()
        st = lib().ot_assoc_adaptive(self.h, ct.byref(desc), pa, float(eps), float(tol), int(max_iter), float(delta),
                                     int(max_outer), q.ctypes.data, js.ctypes.data, ct.byref(r))
        _check(self.h, st)
        self._I, self._J = desc.I, desc.J
        del keep, ka
        return st, q, js[: r.solves], r

    def solve_dense(self, C, a, b, eps, tol=1e-8, max_iter=2000, warm_start=False):
        d, keep = matrix_desc(C, OT_COST_DENSE)
        return self.solve(d, keep, a, b, eps, tol, max_iter, warm_start)

    def solve_rates(self, R, scale, a, b, eps, tol=1e-8, max_iter=2000, warm_start=False):
        d, keep = matrix_desc(R, OT_COST_RATES, scale)
        return self.solve(d, keep, a, b, eps, tol, max_iter, warm_start)

    def solve_geometry(self, dev_xy, rrh_xy, radio, shadow_key, scale, a, b, eps, tol=1e-8, max_iter=2000,
                       warm_start=False):
        d, keep = geometry_desc(dev_xy, rrh_xy, radio, shadow_key, scale)
        return self.solve(d, keep, a, b, eps, tol, max_iter, warm_start)

    def solve_euclid(self, dev_xy, rrh_xy, scale, a, b, eps, tol=1e-8, max_iter=2000, warm_start=False):
        d, keep = euclid_desc(dev_xy, rrh_xy, scale)
        return self.solve(d, keep, a, b, eps, tol, max_iter, warm_start)

    def plan(self, out=None, dtype=np.float64):
        """The plan of the last solve: into `out` (numpy or torch), else a new numpy array."""
        if self._I is None:  # let the library report the state error
            ot_assoc_plan(self.h, None, OT_MEM_HOST, OT_F64)
        if out is None:
            out = np.empty((self._I, self._J), dtype=dtype)
        dt = np.float32 if str(out.dtype) in ("float32", "torch.float32") else np.float64
        p, m, keep = _ptr_mem(out, dt)
        if not _is_torch(out) and keep is not out:
            raise ValueError("numpy plan buffer must be contiguous")
        ot_assoc_plan(self.h, p, m, OT_F32 if dt == np.float32 else OT_F64)
        return out

    def set_plan_output(self, out):
        """Have the following solves write their plan into the device tensor
        `out` (float32 or float64, at least I x J elements) from their final
        check; plan(out) then returns at once. None stops it."""
        if out is None:
            _check(self.h, lib().ot_assoc_set_plan_output(self.h, None, OT_F32, 0))
            self._plan_keep = None
            return
        if not _is_torch(out) or not out.is_cuda or not out.is_contiguous():
            raise ValueError("the plan output must be a contiguous device tensor")
        dt = OT_F32 if str(out.dtype) == "torch.float32" else OT_F64 if str(out.dtype) == "torch.float64" else None
        if dt is None:
            raise ValueError("the plan output must be float32 or float64")
        _check(self.h, lib().ot_assoc_set_plan_output(self.h, ct.c_void_p(out.data_ptr()), dt, out.numel()))
        self._plan_keep = out

    def potentials(self):
        f = np.empty(self._I)
        g = np.empty(self._J)
        ot_assoc_potentials(self.h, f.ctypes.data, g.ctypes.data, OT_MEM_HOST)
        return f, g

    def set_potentials(self, f, g):
        f = np.ascontiguousarray(f, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        ot_assoc_set_potentials(self.h, f.ctypes.data, g.ctypes.data, f.size, g.size, OT_MEM_HOST)
        self._I, self._J = f.size, g.size

    def fast_phase_time(self):
        return ot_assoc_fast_phase_time(self.h)

    def time_sweep(self, reps=50, fp64=False):
        """Average ms of one fused-sweep launch of the last solve's shape."""
        return ot_assoc_time_sweep(self.h, reps, fp64)

    def time_read(self, buf, reps=20):
        """Average ms of a read-only streaming pass over a device tensor (the HBM read ceiling)."""
        ms = ct.c_double()
        _check(self.h, lib().ot_assoc_time_read(self.h, ct.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size(),
                                                int(reps), ct.byref(ms)))
        return ms.value

    def cost_median(self, desc):
        return ot_assoc_cost_median(self.h, desc)

    def materialize_cost(self, desc, C_out):
        p, m, keep = _ptr_mem(C_out, np.float32)
        if m != OT_MEM_DEVICE:
            raise ValueError("materialize_cost writes a device buffer")
        return ot_assoc_materialize_cost(self.h, desc, p)

    # ------------------------------------------------------------ batches --
    def solve_batch(self, costs, a_list, b_list, eps, tol=1e-6, max_iter=2000):
        """Solves instances together. costs: list of cost matrices (numpy or
        torch) or (desc, keep) pairs; a_list / b_list in the costs' memory."""
        descs, keep = [], []
        for c in costs:
            if isinstance(c, tuple):
                descs.append(c[0])
                keep.append(c[1])
            else:
                d, k = matrix_desc(c, OT_COST_DENSE)
                descs.append(d)
                keep.append(k)
        pa, pb = [], []
        for d, a, b in zip(descs, a_list, b_list):
            p1, m1, k1 = _ptr_mem(a, np.float64)
            p2, m2, k2 = _ptr_mem(b, np.float64)
            want = OT_MEM_DEVICE if d.kind in (OT_COST_GEOMETRY, OT_COST_EUCLID) else d.mem
            if m1 != want or m2 != want:
                raise ValueError("marginals must be in the cost's memory space")
            pa.append(p1)
            pb.append(p2)
            keep += [k1, k2]
        eps_l = list(eps) if hasattr(eps, "__len__") else [eps] * len(descs)
        st, res = ot_assoc_solve_batch(self.h, descs, pa, pb, eps_l, tol, max_iter)
        self._batch_dims = [(d.I, d.J) for d in descs]
        del keep
        return st, res

    # ---------------------------------------------------------- snapshots --
    def solve_snapshots(self, cost, A, b, eps, tol=1e-6, max_iter=2000):
        """B traffic snapshots (rows of A, B x I) over one cost: a matrix or a
        (desc, keep) pair; A and b in the cost's memory space."""
        d, keep = cost if isinstance(cost, tuple) else matrix_desc(cost, OT_COST_DENSE)
        pa, ma, ka = _ptr_mem(A, np.float64)
        pb, mb, kb = _ptr_mem(b, np.float64)
        want = OT_MEM_DEVICE if d.kind in (OT_COST_GEOMETRY, OT_COST_EUCLID) else d.mem
        if ma != want or mb != want:
            raise ValueError("snapshots and b must be in the cost's memory space")
        st, res = ot_assoc_solve_snapshots(self.h, d, int(A.shape[0]), pa, pb, eps, tol, max_iter)
        self._snap_dims = (d.I, d.J, int(A.shape[0]))
        self._I, self._J = d.I, d.J
        del keep, ka, kb
        return st, res

    def snapshot_potentials(self, s):
        if self._snap_dims is None:  # let the library report the state error
            ot_assoc_snapshot_potentials(self.h, s, None, None, OT_MEM_HOST)
        I, J, _ = self._snap_dims
        f = np.empty(I)
        g = np.empty(J)
        ot_assoc_snapshot_potentials(self.h, s, f.ctypes.data, g.ctypes.data, OT_MEM_HOST)
        return f, g

    def batch_config(self):
        """(waves per FP32 sweep workgroup, rows per work item) of the last batch."""
        return ot_assoc_batch_config(self.h)

    def batch_potentials(self, k):
        I, J = self._batch_dims[k]
        f = np.empty(I)
        g = np.empty(J)
        ot_assoc_batch_potentials(self.h, k, f.ctypes.data, g.ctypes.data, OT_MEM_HOST)
        return f, g

    def batch_plan(self, k, dtype=np.float64):
        I, J = self._batch_dims[k]
        out = np.empty((I, J), dtype=dtype)
        ot_assoc_batch_plan(self.h, k, out.ctypes.data, OT_MEM_HOST, OT_F32 if dtype == np.float32 else OT_F64)
        return out


class Server:
    """Request server over the batched engine (ot_serve_*). Requests keep
    references to their buffers until their completion is returned."""

    def __init__(self, device=0, stream=None, **opts):
        o = ot_serve_default_options()
        o.device = device
        o.stream = stream
        for k, v in opts.items():
            setattr(o, k, v)
        self.s = ot_serve_create(o)
        self._keep = {}

    def close(self):
        s = getattr(self, "s", None)
        self.s = None
        if s:
            try:
                ot_serve_destroy(s)
            except Exception:
                pass

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def submit(self, cost, a, b, eps, tol=1e-6, max_iter=2000, layout_key=0, user_tag=0):
        """cost: a matrix (numpy / torch) or a (desc, keep) pair."""
        if isinstance(cost, tuple):
            d, kc = cost
        else:
            d, kc = matrix_desc(cost, OT_COST_DENSE)
        p1, m1, k1 = _ptr_mem(a, np.float64)
        p2, m2, k2 = _ptr_mem(b, np.float64)
        want = OT_MEM_DEVICE if d.kind in (OT_COST_GEOMETRY, OT_COST_EUCLID) else d.mem
        if m1 != want or m2 != want:
            raise ValueError("marginals must be in the cost's memory space")
        r = ot_request()
        r.cost = d
        r.a, r.b = p1, p2
        r.eps, r.tol, r.max_iter = float(eps), float(tol), int(max_iter)
        r.layout_key, r.user_tag = int(layout_key), int(user_tag)
        t = ot_serve_submit(self.s, r)
        self._keep[t] = (kc, k1, k2, cost)
        return t

    def progress(self, max_out=256):
        done = ot_serve_progress(self.s, max_out)
        for c in done:
            self._keep.pop(c.ticket, None)
        return done

    def counts(self):
        return ot_serve_counts(self.s)

    def potentials(self, key, I, J):
        f = np.empty(I)
        g = np.empty(J)
        ot_serve_potentials(self.s, key, f.ctypes.data, g.ctypes.data, OT_MEM_HOST)
        return f, g

    @staticmethod
    def now():
        return ot_serve_now()
