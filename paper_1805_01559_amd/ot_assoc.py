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
OT_COST_DENSE, OT_COST_RATES, OT_COST_GEOMETRY = 0, 1, 2
OT_MEM_HOST, OT_MEM_DEVICE = 0, 1
OT_F32, OT_F64 = 0, 1
OT_PREC_FP32, OT_PREC_FP64 = 0, 1

# every symbol include/ot_assoc.h declares
EXPORTS = [
    "ot_assoc_default_options", "ot_assoc_create", "ot_assoc_solve", "ot_assoc_plan", "ot_assoc_potentials",
    "ot_assoc_set_potentials", "ot_assoc_cost_median", "ot_assoc_materialize_cost", "ot_assoc_time_sweep",
    "ot_assoc_destroy", "ot_assoc_last_error",
]


class ot_geometry(ct.Structure):
    _fields_ = [("dev_xy", ct.c_void_p), ("rrh_xy", ct.c_void_p), ("tx_power_w", ct.c_double),
                ("ref_gain", ct.c_double), ("pathloss_exp", ct.c_double), ("min_dist_m", ct.c_double),
                ("shadow_sigma_db", ct.c_double), ("noise_w", ct.c_double), ("bandwidth_hz", ct.c_double),
                ("shadow_key", ct.c_uint64)]


class ot_cost_desc(ct.Structure):
    _fields_ = [("kind", ct.c_int), ("I", ct.c_int64), ("J", ct.c_int64), ("mem", ct.c_int), ("dtype", ct.c_int),
                ("data", ct.c_void_p), ("scale", ct.c_double), ("geom", ot_geometry)]


class ot_assoc_options(ct.Structure):
    _fields_ = [("device", ct.c_int), ("stream", ct.c_void_p), ("precision", ct.c_int), ("polish_iters", ct.c_int),
                ("chunk", ct.c_int), ("use_graphs", ct.c_int), ("sweep_blocks", ct.c_int), ("sweep_waves", ct.c_int),
                ("sweep_rows", ct.c_int), ("sweep_lanes", ct.c_int)]


class ot_assoc_result(ct.Structure):
    _fields_ = [("iterations", ct.c_int32), ("fp64_iterations", ct.c_int32), ("status", ct.c_int32),
                ("reserved", ct.c_int32), ("marginal_violation", ct.c_double), ("objective", ct.c_double),
                ("reg_objective", ct.c_double), ("dual_objective", ct.c_double), ("seconds", ct.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


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
        L.ot_assoc_solve.argtypes = [vp, ct.POINTER(ot_cost_desc), vp, vp, d, d, ct.c_int32, ct.c_int,
                                     ct.POINTER(ot_assoc_result)]
        L.ot_assoc_plan.argtypes = [vp, vp, ct.c_int, ct.c_int]
        L.ot_assoc_potentials.argtypes = [vp, vp, vp, ct.c_int]
        L.ot_assoc_set_potentials.argtypes = [vp, vp, vp, i64, i64, ct.c_int]
        L.ot_assoc_cost_median.argtypes = [vp, ct.POINTER(ot_cost_desc), ct.POINTER(d)]
        L.ot_assoc_materialize_cost.argtypes = [vp, ct.POINTER(ot_cost_desc), vp]
        L.ot_assoc_time_sweep.argtypes = [vp, ct.c_int32, ct.c_int, ct.POINTER(d)]
        L.ot_assoc_destroy.argtypes = [vp]
        L.ot_assoc_destroy.restype = None
        L.ot_assoc_last_error.argtypes = [vp]
        L.ot_assoc_last_error.restype = ct.c_char_p
        for name in EXPORTS:
            if name not in ("ot_assoc_destroy", "ot_assoc_last_error"):
                getattr(L, name).restype = ct.c_int
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


def ot_assoc_solve(h, desc: ot_cost_desc, a_ptr, b_ptr, eps, tol, max_iter, warm_start=0):
    res = ot_assoc_result()
    st = lib().ot_assoc_solve(h, ct.byref(desc), a_ptr, b_ptr, float(eps), float(tol), int(max_iter), int(warm_start),
                              ct.byref(res))
    _check(h, st)
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


def ot_assoc_destroy(h):
    if h:
        lib().ot_assoc_destroy(h)


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


def matrix_desc(M, kind=OT_COST_DENSE, scale: float = 1.0):
    dt = np.float32 if (str(getattr(M, "dtype", "")) in ("float32", "torch.float32")) else np.float64
    p, m, keep = _ptr_mem(M, dt)
    d = ot_cost_desc()
    d.kind, d.mem, d.dtype = kind, m, (OT_F32 if dt == np.float32 else OT_F64)
    d.I, d.J = int(M.shape[0]), int(M.shape[1])
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

    def time_sweep(self, reps=50, fp64=False):
        """Average ms of one fused-sweep launch of the last solve's shape."""
        return ot_assoc_time_sweep(self.h, reps, fp64)

    def cost_median(self, desc):
        return ot_assoc_cost_median(self.h, desc)

    def materialize_cost(self, desc, C_out):
        p, m, keep = _ptr_mem(C_out, np.float32)
        if m != OT_MEM_DEVICE:
            raise ValueError("materialize_cost writes a device buffer")
        return ot_assoc_materialize_cost(self.h, desc, p)
