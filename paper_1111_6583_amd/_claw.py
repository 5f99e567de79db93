"""ctypes declarations for libclaw (include/claw.h).  Marshalling only."""

from __future__ import annotations

import ctypes as C
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libclaw.so")
HEADER = os.path.join(_HERE, "..", "include", "claw.h")

CLAW_OK = 0
ERRORS = {-1: "CLAW_E_INVAL", -2: "CLAW_E_NOMEM", -3: "CLAW_E_DEVICE", -4: "CLAW_E_REJECTED",
          -5: "CLAW_E_NONPHYSICAL", -6: "CLAW_E_BUDGET", -7: "CLAW_E_STATE", -8: "CLAW_E_MAXSTEPS",
          -9: "CLAW_E_TOOBIG"}
STATIC_SCRATCH_BYTES = 64 << 20   # CLAW_STATIC_SCRATCH_BYTES
SCHEMES = {"classic": 1, "sharpclaw": 2}
SOLVERS = {"advection": 1, "sw_roe": 2, "euler_hlle": 3, "elastic_vc": 4, "euler_roe": 5,
           "psystem": 6}
SOURCES = {"none": 0, "axisymmetric": 1}
SPLITS = {"none": 0, "godunov": 1, "strang": 2}
LIMITERS = {"none": 0, "minmod": 1, "mc": 2}
BCS = {"extrap": 1, "periodic": 2, "wall": 3, "dirichlet": 4}
PRECISIONS = {"fp64": 1, "fp32_kahan": 2, "fp32": 3}
INTEGRATORS = {"ssp33": 1, "ssp104": 2}
SIDES = ("x_lower", "x_upper", "y_lower", "y_upper")


class ClawConfig(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("num_cells", C.c_int * 2), ("lower", C.c_double * 2),
        ("upper", C.c_double * 2), ("scheme", C.c_int), ("riemann", C.c_int),
        ("limiter", C.c_int), ("transverse", C.c_int), ("entropy_fix", C.c_int),
        ("bc_lower", C.c_int * 2), ("bc_upper", C.c_int * 2), ("bc_state", (C.c_double * 8) * 4),
        ("cfl_desired", C.c_double), ("cfl_max", C.c_double), ("dt_initial", C.c_double),
        ("dt_max", C.c_double), ("weno_eps", C.c_double), ("precision", C.c_int),
        ("problem_data", C.c_double * 8), ("time_integrator", C.c_int), ("weno_order", C.c_int),
        ("tracer", C.c_int), ("source", C.c_int), ("dimensional_split", C.c_int),
    ]


class ClawStats(C.Structure):
    _fields_ = [("accepted", C.c_longlong), ("rejected", C.c_longlong), ("t", C.c_double),
                ("dt_next", C.c_double), ("max_courant", C.c_double), ("gpu_ms", C.c_double)]

    def as_dict(self):
        return dict(accepted=self.accepted, rejected=self.rejected, t=self.t,
                    dt_next=self.dt_next, max_courant=self.max_courant, gpu_ms=self.gpu_ms)


class ClawTuning(C.Structure):
    _fields_ = [("seg_rows", C.c_int), ("seg_rows_x", C.c_int), ("segs", C.c_int),
                ("order", C.c_int)]


class ClawError(RuntimeError):
    def __init__(self, rc, where=""):
        self.rc = rc
        super().__init__(f"{where}: {ERRORS.get(rc, rc)} ({_strerror(rc)})")


_lib = None


def _strerror(rc):
    if _lib is None:
        return ""
    return _lib.claw_strerror(rc).decode()


def load_library():
    """Load libclaw.so from the package directory; fail loudly if absent.

    torch is imported first: its bundled HIP runtime carries the same soname
    as the one libclaw was linked against, so the dynamic loader binds
    libclaw to that single runtime instead of loading a second one (device
    pointers from torch allocations are then valid for libclaw's kernels).
    """
    global _lib
    if _lib is not None:
        return _lib
    import torch  # noqa: F401  (see above: one HIP runtime per process)
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1111_6583_amd.build` "
                           "(hipcc for gfx950) -- there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    vp, dp, ip = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int)
    cfgp = C.POINTER(ClawConfig)
    stp = C.POINTER(ClawStats)
    tnp = C.POINTER(ClawTuning)
    sig = {
        "claw_strerror": ([C.c_int], C.c_char_p),
        "claw_num_eqn": ([cfgp], C.c_int),
        "claw_num_aux": ([cfgp], C.c_int),
        "claw_workspace_bytes": ([cfgp], C.c_size_t),
        "claw_create": ([cfgp, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
        "claw_set_state": ([vp, vp, C.c_int], C.c_int),
        "claw_set_aux": ([vp, vp, C.c_int], C.c_int),
        "claw_get_state": ([vp, vp, C.c_int], C.c_int),
        "claw_step": ([vp, C.c_double, dp], C.c_int),
        "claw_advance": ([vp, C.c_double, C.c_longlong, stp], C.c_int),
        "claw_advance_graph": ([vp, C.c_double, C.c_int, C.c_longlong, stp], C.c_int),
        "claw_totals": ([vp, dp], C.c_int),
        "claw_get_clock": ([vp, stp], C.c_int),
        "claw_set_clock": ([vp, stp], C.c_int),
        "claw_set_tuning": ([vp, tnp], C.c_int),
        "claw_get_tuning": ([vp, tnp], C.c_int),
        "claw_autotune": ([vp, C.c_int, tnp], C.c_int),
        "claw_time_kernel": ([vp, C.c_double, C.c_int, dp], C.c_int),
        "claw_destroy": ([vp], C.c_int),
        "claw_batch_workspace_bytes": ([C.c_int], C.c_size_t),
        "claw_batch_create": ([C.c_int, vp, C.c_size_t, vp, C.POINTER(vp)], C.c_int),
        "claw_batch_add": ([vp, vp, C.c_double], C.c_int),
        "claw_batch_remove": ([vp, vp], C.c_int),
        "claw_batch_advance": ([vp, C.c_int, ip], C.c_int),
        "claw_batch_launch": ([vp, C.c_int], C.c_int),
        "claw_batch_wait": ([vp, ip], C.c_int),
        "claw_batch_member_clock": ([vp, vp, stp], C.c_int),
        "claw_batch_finished": ([vp, C.POINTER(vp), C.c_int, ip], C.c_int),
        "claw_batch_destroy": ([vp], C.c_int),
        "claw_static_bytes": ([cfgp], C.c_size_t),
        "claw_step_static": ([cfgp, vp, vp, vp, C.c_double, vp, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def header_functions():
    """Function names declared in include/claw.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(claw_[a-z_0-9]+)\s*\(", text)))


def check(rc, where=""):
    if rc != CLAW_OK:
        raise ClawError(rc, where)
    return rc


def make_config(spec: dict) -> ClawConfig:
    """Convert a spec dict (same keys the oracle takes) into a claw_config."""
    c = ClawConfig()
    nd = int(spec["ndim"])
    if nd not in (1, 2):
        raise ValueError(f"ndim must be 1 or 2, got {nd}")
    c.ndim = nd
    nc = list(spec["num_cells"])
    lo, hi = list(spec["lower"]), list(spec["upper"])
    for d in range(nd):
        c.num_cells[d] = int(nc[d])
        c.lower[d] = float(lo[d])
        c.upper[d] = float(hi[d])
    c.scheme = SCHEMES[spec.get("scheme", "classic")]
    c.riemann = SOLVERS[spec["riemann"]]
    c.limiter = LIMITERS[spec.get("limiter", "mc")]
    c.transverse = int(spec.get("transverse", 2))
    c.entropy_fix = int(spec.get("entropy_fix", 0))
    bl = list(spec.get("bc_lower", ["extrap"] * nd))
    bu = list(spec.get("bc_upper", ["extrap"] * nd))
    for d in range(nd):
        c.bc_lower[d] = BCS[bl[d]]
        c.bc_upper[d] = BCS[bu[d]]
    for s, name in enumerate(SIDES):
        vals = (spec.get("bc_state") or {}).get(name)
        if vals is not None:
            for k, v in enumerate(vals):
                c.bc_state[s][k] = float(v)
    c.cfl_desired = float(spec.get("cfl_desired", 0.9))
    c.cfl_max = float(spec.get("cfl_max", 1.0))
    c.dt_initial = float(spec.get("dt_initial", 0.0) or 0.0)
    c.dt_max = float(spec.get("dt_max", 0.0) or 0.0)
    c.weno_eps = float(spec.get("weno_eps", 1e-6))
    c.precision = PRECISIONS[spec.get("precision", "fp64")]
    c.time_integrator = INTEGRATORS[spec.get("time_integrator", "ssp33")]
    c.weno_order = int(spec.get("weno_order", 5))
    c.tracer = int(spec.get("tracer", 0))
    c.source = SOURCES[spec.get("source", "none")]
    c.dimensional_split = SPLITS[spec.get("dimensional_split", "none")]
    for k, v in enumerate(spec.get("problem_data", [])):
        c.problem_data[k] = float(v)
    return c
