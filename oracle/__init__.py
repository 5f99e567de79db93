"""FP64 CPU oracle for the finite-volume step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never calls it.

The arithmetic lives in ``claw_oracle.cpp`` (plain C++, FP64,
``-ffp-contract=off``); this module only marshals arguments through ctypes.
The problem is described by a plain ``spec`` dict (the same dict the GPU
binding accepts; each side converts it to its own C struct):

    ndim, num_cells (nx[, ny]), lower, upper, scheme ("classic"|"sharpclaw"),
    riemann ("advection"|"sw_roe"|"euler_hlle"|"elastic_vc"),
    limiter ("none"|"minmod"|"mc"), transverse (0|1|2), entropy_fix (0|1),
    bc_lower, bc_upper (per dimension: "extrap"|"periodic"|"wall"|"dirichlet"),
    bc_state (dict side -> state list; sides "x_lower", "x_upper",
    "y_lower", "y_upper"), weno_eps, problem_data (list),
    cfl_desired, cfl_max, dt_initial, dt_max.

Arrays are numpy float64 of shape (m, ny, nx) (1D: (m, 1, nx)).
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "claw_oracle.cpp")
_LIB = os.path.join(_HERE, "libclaw_oracle.so")
_lock = threading.Lock()
_lib = None

SCHEMES = {"classic": 1, "sharpclaw": 2}
SOLVERS = {"advection": 1, "sw_roe": 2, "euler_hlle": 3, "elastic_vc": 4, "euler_roe": 5,
           "psystem": 6}
SOURCES = {"none": 0, "axisymmetric": 1}
SPLITS = {"none": 0, "godunov": 1, "strang": 2}
LIMITERS = {"none": 0, "minmod": 1, "mc": 2}
BCS = {"extrap": 1, "periodic": 2, "wall": 3, "dirichlet": 4}
SIDES = ("x_lower", "x_upper", "y_lower", "y_upper")
INTEGRATORS = {"ssp33": 1, "ssp104": 2}


class OCfg(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
        ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double), ("yhi", C.c_double),
        ("scheme", C.c_int), ("solver", C.c_int), ("limiter", C.c_int),
        ("transverse", C.c_int), ("efix", C.c_int), ("bc", C.c_int * 4),
        ("bcstate", (C.c_double * 8) * 4), ("weno_eps", C.c_double), ("pd", C.c_double * 8),
        ("integrator", C.c_int), ("weno_order", C.c_int), ("tracer", C.c_int), ("source", C.c_int),
        ("split", C.c_int), ("cfl_max", C.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (OpenMP over rows, no fast-math)."""
    with _lock:
        if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            tmp = _LIB + ".tmp"
            cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-fPIC",
                   "-shared", _SRC, "-o", tmp]
            subprocess.run(cmd, check=True)
            os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = C.CDLL(_LIB)
    dp = C.POINTER(C.c_double)
    ip = C.POINTER(C.c_int)
    lp = C.POINTER(C.c_long)
    cp = C.POINTER(OCfg)
    lib.or_step.argtypes = [cp, dp, dp, dp, C.c_double, dp]
    lib.or_max_cell_speed.argtypes = [cp, dp, dp]
    lib.or_max_cell_speed.restype = C.c_double
    lib.or_advance.argtypes = [cp, dp, dp, dp, C.c_double, dp, C.c_double, C.c_double,
                               C.c_double, C.c_long, dp, ip, C.c_long, lp, lp, dp]
    lib.or_riemann.argtypes = [cp, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
    lib.or_transverse.argtypes = [cp, C.c_int, dp, dp, dp, dp, dp, dp, dp, dp]
    lib.or_num_flux.argtypes = [cp, C.c_int, dp, dp, dp, dp, dp]
    lib.or_source_step.argtypes = [cp, dp, C.c_double]
    lib.or_source_step.restype = C.c_int
    lib.or_num_flux.restype = C.c_double
    lib.or_weno5.argtypes = [dp, C.c_double, dp, dp]
    lib.or_weno_r.argtypes = [C.c_int, dp, C.c_double, dp, dp]
    lib.or_weno_r.restype = C.c_int
    lib.or_weno_smoothness.argtypes = [C.c_int, dp, dp]
    lib.or_weno_smoothness.restype = C.c_int
    lib.or_weno_linear_weights.argtypes = [C.c_int, dp]
    lib.or_weno_linear_weights.restype = C.c_int
    lib.or_ssp_riccati.argtypes = [C.c_int, C.c_double, C.c_double, C.c_int]
    lib.or_ssp_riccati.restype = C.c_double
    lib.or_limiter.argtypes = [C.c_int, C.c_double]
    lib.or_limiter.restype = C.c_double
    lib.or_totals.argtypes = [cp, dp, dp]
    lib.or_num_threads.argtypes = []
    lib.or_num_threads.restype = C.c_int
    lib.or_set_threads.argtypes = [C.c_int]
    lib.or_set_threads.restype = None
    for f in ("or_num_eqn", "or_num_waves", "or_num_aux"):
        getattr(lib, f).argtypes = [cp]
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double)) if a is not None else None


def make_cfg(spec: dict) -> OCfg:
    c = OCfg()
    nd = int(spec["ndim"])
    nc = list(spec["num_cells"])
    lo = list(spec["lower"])
    hi = list(spec["upper"])
    c.ndim = nd
    c.nx = int(nc[0])
    c.ny = int(nc[1]) if nd == 2 else 1
    c.xlo, c.xhi = float(lo[0]), float(hi[0])
    c.ylo, c.yhi = (float(lo[1]), float(hi[1])) if nd == 2 else (0.0, 1.0)
    c.scheme = SCHEMES[spec.get("scheme", "classic")]
    c.solver = SOLVERS[spec["riemann"]]
    c.limiter = LIMITERS[spec.get("limiter", "mc")]
    c.transverse = int(spec.get("transverse", 2))
    c.efix = int(spec.get("entropy_fix", 0))
    bl = list(spec.get("bc_lower", ["extrap"] * nd))
    bu = list(spec.get("bc_upper", ["extrap"] * nd))
    c.bc[0], c.bc[1] = BCS[bl[0]], BCS[bu[0]]
    if nd == 2:
        c.bc[2], c.bc[3] = BCS[bl[1]], BCS[bu[1]]
    else:
        c.bc[2] = c.bc[3] = BCS["extrap"]
    st = spec.get("bc_state", {}) or {}
    for s, name in enumerate(SIDES):
        vals = st.get(name)
        if vals is not None:
            for k, v in enumerate(vals):
                c.bcstate[s][k] = float(v)
    c.weno_eps = float(spec.get("weno_eps", 1e-6))
    c.integrator = INTEGRATORS[spec.get("time_integrator", "ssp33")]
    c.weno_order = int(spec.get("weno_order", 5)) or 5
    if c.weno_order not in (5, 7, 9, 11, 13, 15, 17):
        raise ValueError(f"weno_order {c.weno_order}: the oracle has WENO of odd orders 5..17")
    c.tracer = int(spec.get("tracer", 0))
    c.source = SOURCES[spec.get("source", "none")]
    c.split = SPLITS[spec.get("dimensional_split", "none")]
    c.cfl_max = float(spec.get("cfl_max", 1.0))
    for k, v in enumerate(spec.get("problem_data", [])):
        c.pd[k] = float(v)
    return c


def num_eqn(spec) -> int:
    return _load().or_num_eqn(C.byref(make_cfg(spec)))


def num_waves(spec) -> int:
    return _load().or_num_waves(C.byref(make_cfg(spec)))


def num_aux(spec) -> int:
    return _load().or_num_aux(C.byref(make_cfg(spec)))


def _state(spec, q):
    c = make_cfg(spec)
    m = _load().or_num_eqn(C.byref(c))
    q = np.ascontiguousarray(q, dtype=np.float64).reshape(m, c.ny, c.nx)
    return c, m, q


def _aux(spec, c, aux):
    na = _load().or_num_aux(C.byref(c))
    if na == 0:
        return None
    return np.ascontiguousarray(aux, dtype=np.float64).reshape(na, c.ny, c.nx)


def step(spec, q, dt, aux=None):
    """One step of size dt.  Returns (q_new, speed) with Courant = dt*speed."""
    c, m, q = _state(spec, q)
    a = _aux(spec, c, aux)
    out = np.empty_like(q)
    sp = C.c_double(0.0)
    _load().or_step(C.byref(c), _ptr(q), _ptr(a), _ptr(out), float(dt), C.byref(sp))
    return out, sp.value


def max_cell_speed(spec, q, aux=None) -> float:
    c, m, q = _state(spec, q)
    a = _aux(spec, c, aux)
    return _load().or_max_cell_speed(C.byref(c), _ptr(q), _ptr(a))


def advance(spec, q, t_end, aux=None, t0=0.0, dt=None, max_steps=10_000_000, log_cap=200_000):
    """Run the step controller from t0 to t_end.

    Returns (q, info) where info has t, dt_next, accepted, rejected,
    max_courant, dts (every dt tried) and acc (1 accepted / 0 rejected), rc.
    """
    c, m, q = _state(spec, q)
    a = _aux(spec, c, aux)
    q = q.copy()
    t = C.c_double(float(t0))
    d = C.c_double(float(spec.get("dt_initial", 0.0) if dt is None else dt))
    dmax = float(spec.get("dt_max", 0.0) or 0.0)
    dts = np.zeros(log_cap)
    acc = np.zeros(log_cap, dtype=np.int32)
    na, nr = C.c_long(0), C.c_long(0)
    cm = C.c_double(0.0)
    rc = _load().or_advance(C.byref(c), _ptr(q), _ptr(a), C.byref(t), float(t_end), C.byref(d),
                            float(spec.get("cfl_desired", 0.9)), float(spec.get("cfl_max", 1.0)),
                            dmax, int(max_steps), _ptr(dts),
                            acc.ctypes.data_as(C.POINTER(C.c_int)), int(log_cap), C.byref(na),
                            C.byref(nr), C.byref(cm))
    n = min(na.value + nr.value, log_cap)
    return q, dict(t=t.value, dt_next=d.value, accepted=na.value, rejected=nr.value,
                   max_courant=cm.value, dts=dts[:n].copy(), acc=acc[:n].copy(), rc=rc)


def riemann(spec, d, ql, qr, auxl=None, auxr=None):
    """Per-face Riemann solve: returns (W[mw, m], s[mw], amdq[m], apdq[m])."""
    c = make_cfg(spec)
    lib = _load()
    m, mw = lib.or_num_eqn(C.byref(c)), lib.or_num_waves(C.byref(c))
    ql = np.zeros(5) + np.pad(np.asarray(ql, float), (0, 5 - m))
    qr = np.zeros(5) + np.pad(np.asarray(qr, float), (0, 5 - m))
    al = np.zeros(3) if auxl is None else np.asarray(auxl, float).copy()
    ar = np.zeros(3) if auxr is None else np.asarray(auxr, float).copy()
    W = np.zeros((5, 5))
    s = np.zeros(5)
    am = np.zeros(5)
    ap = np.zeros(5)
    lib.or_riemann(C.byref(c), int(d), _ptr(ql), _ptr(qr), _ptr(al), _ptr(ar), _ptr(W), _ptr(s),
                   _ptr(am), _ptr(ap))
    return W[:mw, :m], s[:mw], am[:m], ap[:m]


def source_step(spec, q, dt):
    """The geometric source fractional step alone on a state (returns a copy)."""
    c, m, q = _state(spec, q)
    out = q.copy()
    if _load().or_source_step(C.byref(c), _ptr(out), float(dt)) != 0:
        raise ValueError("configuration has no source term")
    return out


def transverse(spec, d, ql, qr, asdq, aux_m=None, aux_c=None, aux_p=None):
    """Split a fluctuation from a face normal to d: returns (bm, bp)."""
    c = make_cfg(spec)
    lib = _load()
    m = lib.or_num_eqn(C.byref(c))
    pad = lambda v: np.pad(np.asarray(v, float), (0, 5 - m))
    ql, qr, asdq = pad(ql), pad(qr), pad(asdq)
    z = np.zeros(3)
    am_, ac_, ap_ = [z.copy() if a is None else np.asarray(a, float).copy() for a in (aux_m, aux_c, aux_p)]
    bm = np.zeros(5)
    bp = np.zeros(5)
    lib.or_transverse(C.byref(c), int(d), _ptr(ql), _ptr(qr), _ptr(am_), _ptr(ac_), _ptr(ap_),
                      _ptr(asdq), _ptr(bm), _ptr(bp))
    return bm[:m], bp[:m]


def num_flux(spec, d, ql, qr, auxl=None, auxr=None):
    """SharpClaw interface flux and speed (aux: the two cells' materials)."""
    c = make_cfg(spec)
    lib = _load()
    m = lib.or_num_eqn(C.byref(c))
    ql = np.pad(np.asarray(ql, float), (0, 5 - m))
    qr = np.pad(np.asarray(qr, float), (0, 5 - m))
    al = np.zeros(3) if auxl is None else np.pad(np.asarray(auxl, float), (0, 3 - len(auxl)))
    ar = np.zeros(3) if auxr is None else np.pad(np.asarray(auxr, float), (0, 3 - len(auxr)))
    F = np.zeros(5)
    s = lib.or_num_flux(C.byref(c), int(d), _ptr(ql), _ptr(qr), _ptr(al), _ptr(ar), _ptr(F))
    return F[:m], s


def weno5(v, eps=1e-6):
    v = np.ascontiguousarray(v, dtype=np.float64)
    qL, qR = C.c_double(), C.c_double()
    _load().or_weno5(_ptr(v), float(eps), C.byref(qL), C.byref(qR))
    return qL.value, qR.value


def weno_r(r, v, eps=1e-6):
    """WENO of order 2r-1 from 2r-1 cell averages centred on a cell: (qL, qR)
    at its right and left edges (general construction)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.size == 2 * r - 1
    qL, qR = C.c_double(), C.c_double()
    if _load().or_weno_r(int(r), _ptr(v), float(eps), C.byref(qL), C.byref(qR)) != 0:
        raise ValueError("r out of range")
    return qL.value, qR.value


def weno_smoothness(r, v):
    """Smoothness indicators of the r candidates from 2r-1 averages."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    b = np.zeros(r)
    if _load().or_weno_smoothness(int(r), _ptr(v), _ptr(b)) != 0:
        raise ValueError("r out of range")
    return b


def weno_linear_weights(r):
    d = np.zeros(r)
    if _load().or_weno_linear_weights(int(r), _ptr(d)) != 0:
        raise ValueError("r out of range")
    return d


def ssp_riccati(integrator, y0, T, n):
    """The SharpClaw step's integrator applied to y' = 1 - y^2, n steps to T."""
    return _load().or_ssp_riccati(INTEGRATORS[integrator], float(y0), float(T), int(n))


def limiter(name, theta):
    return _load().or_limiter(LIMITERS[name], float(theta))


def totals(spec, q):
    c, m, q = _state(spec, q)
    tot = np.zeros(m)
    _load().or_totals(C.byref(c), _ptr(q), _ptr(tot))
    return tot


def set_threads(n: int) -> None:
    """Use n OpenMP threads in later oracle calls."""
    _load().or_set_threads(int(n))


def num_threads() -> int:
    """OpenMP threads the oracle uses (all cores of the affinity mask by default)."""
    return int(_load().or_num_threads())


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"
