"""Seeded synthetic workloads (initial data and problem specs).

This module holds only problem set-up: grids, initial conditions, material
layers and request traces.  It contains none of the finite-volume method's
arithmetic, imports nothing else from this package, and is the one module the
GPU tests and the CPU oracle tests share.

Each generator returns a ``spec`` dict (see ``paper_1111_6583_amd.solver``)
and float64 numpy arrays of shape (m, ny, nx) (1D: (m, 1, nx)).

Workloads (the paper's experiments are PDE initial-value problems defined by
formulas; these stand in for them at the sizes the benchmark configurations
name):

* 1D shallow-water dam break (the paper's serial study uses a shallow-water
  Roe solver with an entropy fix, Section 5);
* 2D radial dam break;
* 2D Euler shock-bubble (Section 7.2: planar shock into a low-density bubble;
  here planar geometry, no tracer);
* 2D linear elasticity in a seeded layered medium;
* a Poisson trace of shallow-water solves for the serving loop.
"""

from __future__ import annotations

import math

import numpy as np

GAMMA = 1.4


def _base(ndim, n, lo, hi, riemann, **kw):
    spec = dict(ndim=ndim, num_cells=tuple(n), lower=tuple(lo), upper=tuple(hi),
                scheme="classic", riemann=riemann, limiter="mc", transverse=2, entropy_fix=0,
                bc_lower=("extrap",) * ndim, bc_upper=("extrap",) * ndim, bc_state={},
                weno_eps=1e-6, problem_data=[], cfl_desired=0.9, cfl_max=1.0, dt_initial=0.0,
                dt_max=0.0, precision="fp64")
    spec.update(kw)
    return spec


def centers(spec):
    """Cell-centre coordinates (x[nx], y[ny]) of a spec's grid."""
    nd = spec["ndim"]
    nx = spec["num_cells"][0]
    x = spec["lower"][0] + (np.arange(nx) + 0.5) * (spec["upper"][0] - spec["lower"][0]) / nx
    if nd == 1:
        return x, np.zeros(1)
    ny = spec["num_cells"][1]
    y = spec["lower"][1] + (np.arange(ny) + 0.5) * (spec["upper"][1] - spec["lower"][1]) / ny
    return x, y


# ---------------------------------------------------------------------------
# 1D shallow-water dam break: g=1, x in [-5,5], h=2 for x<0 else 1, hu=0.
# ---------------------------------------------------------------------------
def dam_break_1d(n=1000, hl=2.0, hr=1.0, **kw):
    spec = _base(1, (n,), (-5.0,), (5.0,), "sw_roe", entropy_fix=1, problem_data=[1.0],
                 cfl_desired=0.9, cfl_max=1.0, **kw)
    x, _ = centers(spec)
    q = np.zeros((2, 1, n))
    q[0, 0] = np.where(x < 0.0, hl, hr)
    return spec, q


# ---------------------------------------------------------------------------
# 2D radial dam break: [-2.5,2.5]^2, h=2 where the cell centre has r<0.5 else 1.
# ---------------------------------------------------------------------------
def radial_dam_break(n=1024, ny=None, h_in=2.0, h_out=1.0, **kw):
    """h_in where the cell centre has r < 0.5, h_out elsewhere (2 and 1 in the
    benchmark; a deep column over a thin layer makes the collapse transonic)."""
    ny = n if ny is None else ny
    spec = _base(2, (n, ny), (-2.5, -2.5), (2.5, 2.5), "sw_roe", entropy_fix=1,
                 problem_data=[1.0], transverse=2, cfl_desired=0.9, cfl_max=1.0, **kw)
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    q = np.zeros((3, ny, n))
    q[0] = np.where(X * X + Y * Y < 0.25, h_in, h_out)
    return spec, q


# ---------------------------------------------------------------------------
# Euler: Rankine-Hugoniot state behind a shock of Mach number M moving into
# still gas (rho0, p0).  Returns (rho, u, p, shock speed).
# ---------------------------------------------------------------------------
def rankine_hugoniot(mach, gamma=GAMMA, rho0=1.0, p0=1.0):
    c0 = math.sqrt(gamma * p0 / rho0)
    m2 = mach * mach
    p1 = p0 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    rho1 = rho0 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    S = mach * c0
    u1 = S * (1.0 - rho0 / rho1)
    return rho1, u1, p1, S


def mach_for_pressure_ratio(ratio, gamma=GAMMA):
    """Shock Mach number giving post/pre pressure ratio ``ratio``."""
    return math.sqrt(1.0 + (ratio - 1.0) * (gamma + 1.0) / (2.0 * gamma))


def euler_conserved(rho, u, v, p, gamma=GAMMA):
    return [rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)]


def shock_bubble(nx=2048, ny=1024, mach=2.0, gamma=GAMMA, bubble_rho=0.1, center=(0.5, 0.0),
                 radius=0.2, shock_x=0.2, sub=16, **kw):
    """Planar Mach-`mach` shock at x=shock_x moving +x into still gas (rho=p=1)
    holding a circular bubble of density bubble_rho (p=1).  Domain
    [0,2]x[-0.5,0.5].  Cut cells take the 16x16 sub-cell midpoint fraction.
    Left boundary: Dirichlet post-shock state; others: extrapolation."""
    rho1, u1, p1, _ = rankine_hugoniot(mach, gamma)
    post = euler_conserved(rho1, u1, 0.0, p1, gamma)
    spec = _base(2, (nx, ny), (0.0, -0.5), (2.0, 0.5), "euler_hlle", scheme="sharpclaw",
                 problem_data=[gamma], bc_lower=("dirichlet", "extrap"),
                 bc_upper=("extrap", "extrap"), bc_state={"x_lower": post}, cfl_desired=0.5,
                 cfl_max=0.6, weno_eps=1e-6, limiter="none", transverse=0, **kw)
    x, y = centers(spec)
    dx = (spec["upper"][0] - spec["lower"][0]) / nx
    dy = (spec["upper"][1] - spec["lower"][1]) / ny
    # bubble volume fraction per cell by sub-cell midpoints
    off = (np.arange(sub) + 0.5) / sub - 0.5
    frac = np.zeros((ny, nx))
    X, Y = np.meshgrid(x, y)
    r2 = radius * radius
    near = (np.abs(X - center[0]) < radius + dx) & (np.abs(Y - center[1]) < radius + dy)
    jj, ii = np.nonzero(near)
    for a in off:
        for b in off:
            xs = x[ii] + a * dx
            ys = y[jj] + b * dy
            frac[jj, ii] += ((xs - center[0]) ** 2 + (ys - center[1]) ** 2 < r2)
    frac /= sub * sub
    rho = 1.0 * (1.0 - frac) + bubble_rho * frac
    q = np.zeros((4, ny, nx))
    q[0] = rho
    q[3] = 1.0 / (gamma - 1.0)
    behind = X < shock_x
    for k in range(4):
        q[k] = np.where(behind, post[k], q[k])
    return spec, q


def _bubble_fraction(x, y, dx, dy, center, radius, sub):
    """Per-cell fraction inside a circle by sub x sub sub-cell midpoints."""
    off = (np.arange(sub) + 0.5) / sub - 0.5
    frac = np.zeros((len(y), len(x)))
    X, Y = np.meshgrid(x, y)
    near = (np.abs(X - center[0]) < radius + dx) & (np.abs(Y - center[1]) < radius + dy)
    jj, ii = np.nonzero(near)
    r2 = radius * radius
    for a in off:
        for b in off:
            xs = x[ii] + a * dx
            ys = y[jj] + b * dy
            frac[jj, ii] += ((xs - center[0]) ** 2 + (ys - center[1]) ** 2 < r2)
    return frac / (sub * sub)


# ---------------------------------------------------------------------------
# The paper's classic shock-bubble run (Section 7.2, eq. euler-rz): axisymmetric
# Euler on [0,2] x [0,0.5] (x = axial z, y = radius r), a planar shock moving
# in +z into still gas (rho = p = 1) holding a spherical bubble (rho = 0.1,
# p = 1) centred on the axis; a tracer is 1 in the bubble.  The post-shock
# state printed in the paper (p = 5, rho ~ 2.82, axial velocity ~ 1.61) is the
# Mach-2.1044 shock, imposed at the left edge.  Reflecting axis (bottom),
# outflow top and right.  Classic Clawpack: Roe solver, MC limiter, full
# transverse corrections, maximum CFL 0.8.  Bubble centre (0.5, 0), radius
# 0.2, shock at z = 0.2 (not given in the paper).
# ---------------------------------------------------------------------------
PAPER_MACH = 2.104417123237


def shock_bubble_axisym(nx=1280, ny=320, mach=PAPER_MACH, gamma=GAMMA, bubble_rho=0.1,
                        center=(0.5, 0.0), radius=0.2, shock_x=0.2, sub=16, tracer=1, **kw):
    rho1, u1, p1, _ = rankine_hugoniot(mach, gamma)
    post = list(euler_conserved(rho1, u1, 0.0, p1, gamma)) + ([0.0] if tracer else [])
    spec = _base(2, (nx, ny), (0.0, 0.0), (2.0, 0.5), "euler_roe", problem_data=[gamma],
                 tracer=tracer, source="axisymmetric", entropy_fix=1, limiter="mc", transverse=2,
                 bc_lower=("dirichlet", "wall"), bc_upper=("extrap", "extrap"),
                 bc_state={"x_lower": post}, cfl_desired=0.75, cfl_max=0.8, **kw)
    x, y = centers(spec)
    dx = 2.0 / nx
    dy = 0.5 / ny
    frac = _bubble_fraction(x, y, dx, dy, center, radius, sub)
    X, _ = np.meshgrid(x, y)
    m = 4 + (1 if tracer else 0)
    q = np.zeros((m, ny, nx))
    q[0] = 1.0 * (1.0 - frac) + bubble_rho * frac
    q[3] = 1.0 / (gamma - 1.0)
    if tracer:
        q[4] = frac
    behind = X < shock_x
    for k in range(m):
        q[k] = np.where(behind, post[k], q[k])
    return spec, q


# ---------------------------------------------------------------------------
# The paper's Listing 1: a 2D Euler Riemann problem on [0,1]^2 with four
# quadrant states, extrapolation boundaries, gamma = 1.4, to t = 0.3, classic
# Clawpack with the 4-wave Roe solver.  The initial data follow the listing's
# formulas as printed (its q[1], q[2] enter the energy as given).
# ---------------------------------------------------------------------------
def listing1_riemann(n=100, gamma=GAMMA, **kw):
    spec = _base(2, (n, n), (0.0, 0.0), (1.0, 1.0), "euler_roe", problem_data=[gamma],
                 limiter="mc", transverse=2, **kw)
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    l, r = X < 0.5, X >= 0.5
    b, t = Y < 0.5, Y >= 0.5
    q = np.zeros((4, n, n))
    q[0] = 2.0 * (l & t) + 1.0 * (l & b) + 1.0 * (r & t) + 3.0 * (r & b)
    q[1] = 0.75 * t - 0.75 * b
    q[2] = 0.5 * l - 0.5 * r
    q[3] = 0.5 * q[0] * (q[1] ** 2 + q[2] ** 2) + 1.0 / (gamma - 1.0)
    return spec, q


# ---------------------------------------------------------------------------
# 2D linear elasticity in a layered medium: 16 layers along x with interfaces
# at seeded sorted uniform positions snapped to cell faces; per layer
# rho ~ U[1,4], lambda, mu ~ U[1,10].  Stress pulse s11 = s22 =
# exp(-(x^2 + (y-0.5)^2)/w^2), w=0.05, on the left boundary (a wall).
# ---------------------------------------------------------------------------
def layered_elastic(n=2048, ny=None, layers=16, seed=1, width=0.05, amplitude=1.0, **kw):
    ny = n if ny is None else ny
    spec = _base(2, (n, ny), (0.0, 0.0), (1.0, 1.0), "elastic_vc", transverse=2,
                 bc_lower=("wall", "extrap"), bc_upper=("extrap", "extrap"), cfl_desired=0.9,
                 cfl_max=1.0, **kw)
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.uniform(0.0, 1.0, layers - 1))
    faces = np.unique(np.clip(np.rint(cuts * n).astype(int), 1, n - 1))
    rho_l = rng.uniform(1.0, 4.0, layers)
    lam_l = rng.uniform(1.0, 10.0, layers)
    mu_l = rng.uniform(1.0, 10.0, layers)
    col_layer = np.searchsorted(faces, np.arange(n), side="right")
    aux = np.zeros((3, ny, n))
    aux[0] = rho_l[col_layer][None, :]
    aux[1] = lam_l[col_layer][None, :]
    aux[2] = mu_l[col_layer][None, :]
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    pulse = amplitude * np.exp(-(X ** 2 + (Y - 0.5) ** 2) / width ** 2)
    q = np.zeros((5, ny, n))
    q[0] = pulse
    q[1] = pulse
    return spec, q, aux


# ---------------------------------------------------------------------------
# Shallow-water hump (serving requests and smooth tests):
# h = 1 + A exp(-|x-x0|^2/w^2) on [0,1]^2, hu = hv = 0, g = 1.
# ---------------------------------------------------------------------------
def sw_hump_spec(n, **kw):
    """Problem spec of an N x N shallow-water hump on [0,1]^2 (no state)."""
    return _base(2, (n, n), (0.0, 0.0), (1.0, 1.0), "sw_roe", entropy_fix=1,
                 problem_data=[1.0], transverse=2, cfl_desired=0.9, cfl_max=1.0, **kw)


def sw_hump(n, amplitude=0.5, width=0.1, x0=(0.5, 0.5), **kw):
    spec = sw_hump_spec(n, **kw)
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    q = np.zeros((3, n, n))
    q[0] = 1.0 + amplitude * np.exp(-((X - x0[0]) ** 2 + (Y - x0[1]) ** 2) / width ** 2)
    return spec, q


def serving_trace(n_requests=2000, rate=200.0, seed=0, nmin=64, nmax=1024, t_end=0.5):
    """Poisson arrivals of shallow-water solves: N ~ U{nmin..nmax}, A ~ U[0.1,1],
    w ~ U[0.05,0.3], x0 ~ U[0.25,0.75]^2, each run to t_end."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps)
    out = []
    for r in range(n_requests):
        out.append(dict(id=r, arrival=float(arrivals[r]), n=int(rng.integers(nmin, nmax + 1)),
                        amplitude=float(rng.uniform(0.1, 1.0)), width=float(rng.uniform(0.05, 0.3)),
                        x0=(float(rng.uniform(0.25, 0.75)), float(rng.uniform(0.25, 0.75))),
                        t_end=t_end))
    return out


def request_problem(req, precision="fp32_kahan"):
    return sw_hump(req["n"], amplitude=req["amplitude"], width=req["width"], x0=req["x0"],
                   precision=precision)


# ---------------------------------------------------------------------------
# Smooth data for convergence and conservation tests.
# ---------------------------------------------------------------------------
def random_smooth_sw(n, seed=0, periodic=True, amplitude=0.2):
    """Periodic smooth shallow-water state from a few random Fourier modes."""
    rng = np.random.default_rng(seed)
    bc = "periodic" if periodic else "extrap"
    spec = _base(2, (n, n), (0.0, 0.0), (1.0, 1.0), "sw_roe", entropy_fix=1,
                 problem_data=[1.0], bc_lower=(bc, bc), bc_upper=(bc, bc))
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    q = np.zeros((3, n, n))
    q[0] = 1.0
    for _ in range(3):
        kx, ky = rng.integers(1, 4, 2)
        ph = rng.uniform(0, 2 * np.pi, 3)
        a = rng.uniform(-1, 1, 3) * amplitude
        q[0] += a[0] * np.sin(2 * np.pi * (kx * X + ky * Y) + ph[0]) * 0.5
        q[1] += a[1] * np.sin(2 * np.pi * (kx * X - ky * Y) + ph[1]) * 0.3
        q[2] += a[2] * np.cos(2 * np.pi * (ky * X + kx * Y) + ph[2]) * 0.3
    return spec, q


def random_smooth_euler(n, seed=0):
    rng = np.random.default_rng(seed)
    spec = _base(2, (n, n), (0.0, 0.0), (1.0, 1.0), "euler_hlle", scheme="sharpclaw",
                 problem_data=[GAMMA], bc_lower=("periodic", "periodic"),
                 bc_upper=("periodic", "periodic"), cfl_desired=0.5, cfl_max=0.6, limiter="none",
                 transverse=0)
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    ph = rng.uniform(0, 2 * np.pi, 4)
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * (X + Y) + ph[0])
    u = 0.5 + 0.1 * np.sin(2 * np.pi * X + ph[1])
    v = -0.3 + 0.1 * np.cos(2 * np.pi * Y + ph[2])
    p = 1.0 + 0.1 * np.sin(2 * np.pi * (X - Y) + ph[3])
    q = np.array(euler_conserved(rho, u, v, p))
    return spec, q


# ---------------------------------------------------------------------------
# Nonlinear p-system in a checkerboard medium (the paper's cylindrical
# solitary-wave problem): positive quadrant [0, P]^2 in units of the medium
# period, `cpp` cells per period (the paper: 240 cells, P = 200).  Squares of
# (K, rho) = (1, 1) where (x - floor(x) - 1/2)(y - floor(y) - 1/2) < 0, else
# (5, 5), at the cell centre.  Initial stress a Gaussian of amplitude 5 and
# variance 5 in x and y centred at the origin, zero velocity; the strain is
# the one whose stress sigma = exp(K eps) - 1 equals it.  Reflecting walls
# at x = 0 and y = 0, zero-order extrapolation at the far sides.  SharpClaw,
# WENO5, SSPRK(10,4).  Returns (spec, q, aux).
# ---------------------------------------------------------------------------
def psystem_material(x, y):
    """(K, rho) of the checkerboard at points (x, y)."""
    s = (x - np.floor(x) - 0.5) * (y - np.floor(y) - 0.5)
    K = np.where(s < 0, 1.0, 5.0)
    return K, K.copy()


def psystem_checkerboard(cpp=240, periods=200, ny_periods=None, amplitude=5.0, variance=5.0,
                         **kw):
    py = periods if ny_periods is None else ny_periods
    n, m = cpp * periods, cpp * py
    spec = _base(2, (n, m), (0.0, 0.0), (float(periods), float(py)), "psystem",
                 scheme="sharpclaw", limiter="none", transverse=0,
                 bc_lower=("wall", "wall"), bc_upper=("extrap", "extrap"),
                 time_integrator="ssp104", weno_order=5, cfl_desired=2.45, cfl_max=2.5)
    spec.update(kw)
    x, y = centers(spec)
    X, Y = np.meshgrid(x, y)
    K, rho = psystem_material(X, Y)
    sig = amplitude * np.exp(-(X * X + Y * Y) / (2.0 * variance))
    q = np.zeros((3, m, n))
    q[0] = np.log1p(sig) / K
    return spec, q, np.array([K, rho])


def psystem_layered_1d(n, lo=0.0, hi=1.0, interfaces=(), materials=((1.0, 1.0),), **kw):
    """1D p-system on [lo, hi] with piecewise-constant (K, rho): material
    k between interfaces[k-1] and interfaces[k] (cell centres).  Returns
    (spec, aux); the caller sets q (strain, momentum)."""
    spec = _base(1, (n,), (lo,), (hi,), "psystem", scheme="sharpclaw", limiter="none",
                 transverse=0, time_integrator="ssp104", weno_order=5, cfl_desired=2.45,
                 cfl_max=2.5)
    spec.update(kw)
    x, _ = centers(spec)
    idx = np.searchsorted(np.asarray(interfaces, float), x)
    mat = np.asarray(materials, float)[idx]
    aux = np.zeros((2, 1, n))
    aux[0, 0] = mat[:, 0]
    aux[1, 0] = mat[:, 1]
    return spec, aux
