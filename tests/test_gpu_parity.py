"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

FP64 bar (per cell and component): |g - o| <= 1e-12 * max(|o|, max|o_k|),
the component's own largest magnitude covering cells where it is near zero,
floored at 1e-2 of the largest component sharing its units (a component
that small carries rounding errors on its partners' scale; see UNIT_FLOOR).
FP32+Kahan bar: relative L1 error per component against the FP64 oracle
run with the same dt sequence (1e-5 shallow water, 1e-4 Euler/elasticity).
Integer-like results (step counts, accept/reject sequences) must be equal.
"""

import sys

import numpy as np
import pytest

import oracle
from paper_1111_6583_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def solver(spec, q, aux=None, seg_rows=None):
    from paper_1111_6583_amd import Solver
    s = Solver(spec)
    s.set_state(q)
    if aux is not None:
        s.set_aux(aux)
    if seg_rows:
        s.set_tuning(seg_rows)
    return s


def unit_groups(spec):
    """Components that share physical units.  Used only for a component whose
    exact value is zero everywhere (a transverse momentum of y-uniform data,
    a momentum at rest): its computed values are rounding noise, and it is
    compared on the scale of the components sharing its units."""
    r, nd = spec["riemann"], spec["ndim"]
    if r == "sw_roe":
        return [[0], [1]] if nd == 1 else [[0], [1, 2]]
    if r == "euler_hlle":
        return [[0], [1], [2]] if nd == 1 else [[0], [1, 2], [3]]
    if r == "euler_roe":
        g = [[0], [1], [2]] if nd == 1 else [[0], [1, 2], [3]]
        return g + ([[len(g) + (0 if nd == 1 else 1)]] if spec.get("tracer") else [])
    if r == "elastic_vc":
        return [[0, 1, 2], [3, 4]]
    if r == "psystem":
        return [[0], [1]] if nd == 1 else [[0], [1, 2]]
    return [[0]]


# A component more than 1/UNIT_FLOOR times smaller than the largest component
# sharing its units is compared on UNIT_FLOOR times that one's scale: its
# rounding errors come from arithmetic on the larger components (a small
# transverse momentum is updated by fluxes carrying the pressure and the
# streamwise momentum).  Measured on the oracle itself: SSPRK(10,4) + WENO7
# shock-bubble at t = 0.03, rho v = 1.6e-3 of rho u; a one-ulp perturbation
# of the state before every step moves rho v by 1.8e-12 of its own largest
# value but only 4e-15 of rho u's, as for every other component.  With the
# floor at 1e-2 of the group an honest FP64 difference is amplified at most
# 100 times on the own scale, which stays inside 1e-12.
UNIT_FLOOR = 1e-2


def fp64_scales(o, spec):
    """Per-component scale of the FP64 bar: the component's own largest
    magnitude over the grid (|g - o| <= 1e-12 max(|o|, max|o_k|) per cell),
    floored at UNIT_FLOOR times the largest magnitude among the components
    sharing its units."""
    comp_max = np.max(np.abs(o), axis=tuple(range(1, o.ndim)))
    scale = comp_max.copy()
    for grp in unit_groups(spec):
        gmax = max(comp_max[grp])
        for k in grp:
            scale[k] = max(comp_max[k], UNIT_FLOOR * gmax)
    return np.where(scale > 0, scale, 1.0)


def fp64_err(g, o, spec, scales=None):
    """Largest |g - o| / max(|o|, scale_k) over cells and components k
    (scales: per-component scales to use instead of o's own, e.g. those of
    the whole grid when o is a window of it)."""
    sc = fp64_scales(o, spec) if scales is None else np.asarray(scales, dtype=np.float64)
    scale = np.maximum(np.abs(o), sc.reshape((-1,) + (1,) * (o.ndim - 1)))
    return float(np.max(np.abs(g - o) / scale))


# The kernels' reciprocals and reciprocal square roots carry up to 2.1e-15
# relative error (one Newton step after the hardware estimate; measured over
# 2^20 arguments), against the oracle's correctly rounded divisions.
KERNEL_REL_ERR = 2.1e-15
PERTURBATION = 1e-15


def _stages(spec):
    if spec.get("scheme", "classic") != "sharpclaw":
        return 1
    return 10 if spec.get("time_integrator", "ssp33") == "ssp104" else 3


def rounding_tol(spec, q, dts, aux=None, region=None, scales=None):
    """FP64 parity bar of a case run with the step sizes dts: 1e-12, or,
    where the method itself amplifies rounding more than that, the oracle's
    own response to a relative PERTURBATION of its state before every step,
    scaled to the kernels' rounding: each stage of a step enters the state
    with a relative error up to KERNEL_REL_ERR, and both sides round, so the
    factor is 2 * stages * KERNEL_REL_ERR / PERTURBATION (42 for the ten-stage
    SSPRK(10,4), 12.6 for SSPRK(3,3)).  High-order WENO's nonlinear weights
    are steep functions of the data (alpha ~ 1/(eps + beta)^2 with
    eps = 1e-6), so rounding-level differences grow there; a wrong
    coefficient, index or sign gives differences of 1e-6 and more.  region:
    (rows, columns) slices of the cells compared (the rest, e.g. a window's
    margin next to its artificial boundaries, is not measured); scales: as
    for fp64_err."""
    rng = np.random.default_rng(12345)
    ref = np.array(q, dtype=np.float64)
    x = ref.copy()
    for dt in dts:
        ref, _ = oracle.step(spec, ref, dt, aux=aux)
        x, _ = oracle.step(spec, x * (1.0 + PERTURBATION * rng.standard_normal(x.shape)), dt, aux=aux)
    if region is not None:
        ref, x = ref[(slice(None),) + tuple(region)], x[(slice(None),) + tuple(region)]
    sens = fp64_err(x, ref, spec, scales)
    factor = 2.0 * _stages(spec) * KERNEL_REL_ERR / PERTURBATION
    say("oracle rounding sensitivity", sens, "bar", max(1e-12, factor * sens))
    return max(1e-12, factor * sens)


def l1_rel(g, o):
    return [float(np.sum(np.abs(g[k] - o[k])) / max(np.sum(np.abs(o[k])), 1e-300))
            for k in range(o.shape[0])]


def l1_rel_groups(g, o, spec):
    """L1 error per component relative to its own L1 norm, floored at
    UNIT_FLOOR times the largest L1 norm among the components sharing its
    units (the FP32 counterpart of the FP64 floor)."""
    norms = [float(np.sum(np.abs(o[k]))) for k in range(o.shape[0])]
    floor = list(norms)
    for grp in unit_groups(spec):
        for k in grp:
            floor[k] = max(norms[k], UNIT_FLOOR * max(norms[m] for m in grp))
    return [float(np.sum(np.abs(g[k] - o[k]))) / max(floor[k], 1e-300) for k in range(o.shape[0])]


def replay(spec, q, dts, aux=None, seg_rows=None):
    s = solver(spec, q, aux, seg_rows)
    for dt in dts:
        s.step(dt)
    out = s.get_state()
    s.close()
    return out


def oracle_run(spec, q, t_end, aux=None):
    qf, info = oracle.advance(spec, q, t_end, aux=aux)
    assert info["rc"] == 0
    return qf, info["dts"][info["acc"] == 1], info


def full_size_replay(spec, q, k, aux=None, reps=2):
    """The oracle's controller runs k attempts from the seeded state at full
    size; the GPU replays its step sizes in the tiling the autotuner picks
    (the one the benchmark times).  Returns (gpu state, oracle state, dts)."""
    qo, info = oracle.advance(spec, q, 1e9, aux=aux, max_steps=k)
    dts = info["dts"][info["acc"] == 1]   # k attempts; a rejected one is not replayed
    assert len(dts) >= k - 2
    s = solver(spec, q, aux)
    s.autotune(reps=reps)
    say("tiling: segments", s.get_segs(), "rows per segment", s.get_tuning())
    for dt in dts:
        s.step(dt)
    g = s.get_state()
    s.close()
    return g, qo, dts


def apriori_dt(spec, q, aux=None, frac=0.9):
    """frac times the controller's a-priori first step: cfl_desired times the
    smallest spacing over the largest cell speed of the seeded state."""
    nd = spec["ndim"]
    h = min((spec["upper"][d] - spec["lower"][d]) / spec["num_cells"][d] for d in range(nd))
    return frac * spec["cfl_desired"] * h / oracle.max_cell_speed(spec, q, aux=aux)


def window_spec(spec, lo_i, hi_i, lo_j, hi_j):
    """The sub-grid [lo_i, hi_i) x [lo_j, hi_j) of a 2D spec: the domain's own
    boundary conditions where it touches the domain's edges, extrapolation
    on the artificial sides."""
    nx, ny = spec["num_cells"]
    hx = (spec["upper"][0] - spec["lower"][0]) / nx
    hy = (spec["upper"][1] - spec["lower"][1]) / ny
    bl, bu = spec.get("bc_lower", ("extrap", "extrap")), spec.get("bc_upper", ("extrap", "extrap"))
    return dict(spec, num_cells=(hi_i - lo_i, hi_j - lo_j),
                lower=(spec["lower"][0] + lo_i * hx, spec["lower"][1] + lo_j * hy),
                upper=(spec["lower"][0] + hi_i * hx, spec["lower"][1] + hi_j * hy),
                bc_lower=(bl[0] if lo_i == 0 else "extrap", bl[1] if lo_j == 0 else "extrap"),
                bc_upper=(bu[0] if hi_i == nx else "extrap", bu[1] if hi_j == ny else "extrap"))


def windowed_oracle(spec, q, dts, j0, i0, margin, size=64, aux=None):
    """The oracle's steps dts on the size x size window at (j0, i0) of the
    seeded state q, run on the window plus `margin` cells each way (at least
    the steps' reach, so the window's cells equal the full-grid oracle's bit
    for bit).  Returns (window of the result, window spec, seeded input of
    the padded window, region of the window inside it)."""
    nx, ny = spec["num_cells"]
    lo_j, hi_j = max(j0 - margin, 0), min(j0 + size + margin, ny)
    lo_i, hi_i = max(i0 - margin, 0), min(i0 + size + margin, nx)
    ws = window_spec(spec, lo_i, hi_i, lo_j, hi_j)
    qw = q[:, lo_j:hi_j, lo_i:hi_i]
    aw = None if aux is None else aux[:, lo_j:hi_j, lo_i:hi_i]
    o = qw.copy()
    for dt in dts:
        o, _ = oracle.step(ws, o, dt, aux=aw)
    region = (slice(j0 - lo_j, j0 - lo_j + size), slice(i0 - lo_i, i0 - lo_i + size))
    return o[(slice(None),) + region], ws, qw, aw, region


# --------------------------------------------------------------------------
# 1D classic: the dam break (exact-solution configuration)
# --------------------------------------------------------------------------
def test_dam_break_1d_replayed_dt():
    say("case: 1D dam break, 1000 cells, replayed oracle dt, FP64")
    spec, q = W.dam_break_1d(1000)
    qo, dts, info = oracle_run(spec, q, 2.0)
    g = replay(spec, q, dts)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("graph", [False, True])
def test_dam_break_1d_controller(graph):
    say("case: 1D dam break, controller on", "device" if graph else "host")
    spec, q = W.dam_break_1d(1000)
    qo, dts, info = oracle_run(spec, q, 2.0)
    s = solver(spec, q)
    st = s.advance(2.0, graph=graph)
    assert st["t"] == 2.0
    assert st["accepted"] == info["accepted"] and st["rejected"] == info["rejected"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


def test_dam_break_1d_larger_grid_strips():
    say("case: 1D dam break, 5000 cells (many strips, graph of steps)")
    spec, q = W.dam_break_1d(5000)
    qo, dts, info = oracle_run(spec, q, 0.5)
    s = solver(spec, q)
    st = s.advance(0.5)
    assert st["accepted"] == info["accepted"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


# --------------------------------------------------------------------------
# 2D classic, shallow water
# --------------------------------------------------------------------------
def test_radial_dam_break_ragged_replay():
    say("case: 2D radial dam break 130x77 (ragged strips and segments), 40 steps")
    spec, q = W.radial_dam_break(130, ny=77)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=40)
    dts = info["dts"][info["acc"] == 1]
    assert len(dts) == 40
    g = replay(spec, q, dts)
    assert fp64_err(g, qo, spec) <= 1e-12


BC_CASES = [
    (("periodic", "periodic"), ("periodic", "periodic")),
    (("wall", "wall"), ("wall", "wall")),
    (("extrap", "wall"), ("wall", "extrap")),
    (("wall", "periodic"), ("extrap", "periodic")),
]


@pytest.mark.parametrize("bcl,bcu", BC_CASES)
def test_sw_boundary_conditions(bcl, bcu):
    say("case: SW hump 70x66 bcs", bcl, bcu)
    spec, q = W.sw_hump(70, amplitude=0.6, width=0.15, x0=(0.3, 0.65))
    q = q[:, :66, :].copy()
    spec = dict(spec, num_cells=(70, 66), upper=(1.0, 66 / 70), bc_lower=bcl, bc_upper=bcu)
    q[1] = 0.2 * q[0]
    q[2] = -0.1 * q[0]
    qo, info = oracle.advance(spec, q, 1.0, max_steps=25)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


def test_sw_dirichlet_corners():
    say("case: SW with Dirichlet sides and extrap corners")
    spec, q = W.sw_hump(64, amplitude=0.5, width=0.2)
    spec = dict(spec, bc_lower=("dirichlet", "wall"), bc_upper=("extrap", "dirichlet"),
                bc_state={"x_lower": [1.5, 0.3, 0.0], "y_upper": [1.2, 0.0, -0.2]})
    qo, info = oracle.advance(spec, q, 1.0, max_steps=25)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("trans", [0, 1, 2])
@pytest.mark.parametrize("lim", ["none", "minmod", "mc"])
def test_sw_transverse_and_limiters(trans, lim):
    say("case: SW radial 72x64 transverse", trans, "limiter", lim)
    spec, q = W.radial_dam_break(72, ny=64)
    spec = dict(spec, transverse=trans, limiter=lim, entropy_fix=0 if lim == "minmod" else 1,
                cfl_desired=0.45 if trans == 0 else 0.9)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=20)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


def test_full_size_radial_dam_break_one_step():
    """1024^2 in the tiling the benchmark uses: the oracle's first 10 steps
    from the seeded state, replayed on the GPU, whole grid."""
    say("case: radial dam break 1024^2, 10 replayed steps from the seeded state")
    spec, q = W.radial_dam_break(1024)
    g, o, _ = full_size_replay(spec, q, 10)
    e = fp64_err(g, o, spec)
    say("max rel err", e)
    assert e <= 1e-12


# --------------------------------------------------------------------------
# 2D classic, advection and elasticity
# --------------------------------------------------------------------------
def test_advection_2d_exact_diagonal_shift():
    say("case: advection 2D Courant 1 diagonal shift on the GPU")
    n = 64
    spec = dict(ndim=2, num_cells=(n, n), lower=(0, 0), upper=(1, 1), riemann="advection",
                limiter="mc", transverse=2, bc_lower=("periodic", "periodic"),
                bc_upper=("periodic", "periodic"), problem_data=[1.0, 1.0])
    q0 = np.random.default_rng(11).standard_normal((1, n, n))
    g = replay(spec, q0, [1.0 / n] * 7)
    np.testing.assert_allclose(g, np.roll(q0, (7, 7), axis=(1, 2)), rtol=0, atol=1e-12)


def test_advection_2d_replay():
    say("case: advection 2D smooth + random, u=0.7 v=-0.4, 30 steps")
    n = 97
    spec = dict(ndim=2, num_cells=(n, 83), lower=(0, 0), upper=(1, 83 / 97), riemann="advection",
                limiter="mc", transverse=2, bc_lower=("periodic", "extrap"),
                bc_upper=("periodic", "extrap"), problem_data=[0.7, -0.4])
    q0 = np.random.default_rng(12).standard_normal((1, 83, n))
    qo = q0
    for _ in range(30):
        qo, _ = oracle.step(spec, qo, 0.8 / n)
    g = replay(spec, q0, [0.8 / n] * 30)
    assert fp64_err(g, qo, spec) <= 1e-12


def test_layered_elastic_replay():
    say("case: layered elasticity 96x80, 30 steps")
    spec, q, aux = W.layered_elastic(96, ny=80)
    qo, info = oracle.advance(spec, q, 1.0, aux=aux, max_steps=30)
    g = replay(spec, q, info["dts"][info["acc"] == 1], aux=aux)
    assert fp64_err(g, qo, spec) <= 1e-12


def test_full_size_layered_elastic_one_step():
    say("case: layered elasticity 2048^2, 3 replayed steps from the seeded state")
    spec, q, aux = W.layered_elastic(2048)
    g, o, _ = full_size_replay(spec, q, 3, aux=aux)
    e = fp64_err(g, o, spec)
    say("max rel err", e)
    assert e <= 1e-12


# --------------------------------------------------------------------------
# SharpClaw: WENO5 + HLLE + SSPRK(3,3)
# --------------------------------------------------------------------------
def test_shock_bubble_replay():
    say("case: shock-bubble 128x64 SharpClaw, 30 steps")
    spec, q = W.shock_bubble(128, 64)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=30)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


def test_shock_bubble_ragged_periodic_euler():
    say("case: smooth periodic Euler 77x61 SharpClaw, 20 steps")
    spec, q = W.random_smooth_euler(77, seed=3)
    q = q[:, :61, :].copy()
    spec = dict(spec, num_cells=(77, 61), upper=(1.0, 61 / 77))
    qo, info = oracle.advance(spec, q, 1.0, max_steps=20)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


def test_sharpclaw_1d_planar_shock():
    say("case: SharpClaw 1D Euler planar shock, 400 cells, controller on device")
    rho1, u1, p1, S = W.rankine_hugoniot(2.0)
    n = 400
    post = [rho1, rho1 * u1, p1 / 0.4 + 0.5 * rho1 * u1 * u1]
    spec = dict(ndim=1, num_cells=(n,), lower=(0.0,), upper=(2.0,), scheme="sharpclaw",
                riemann="euler_hlle", problem_data=[1.4], bc_lower=("dirichlet",),
                bc_upper=("extrap",), bc_state={"x_lower": post}, cfl_desired=0.5, cfl_max=0.6)
    x = (np.arange(n) + 0.5) * 2.0 / n
    q = np.zeros((3, 1, n))
    for k in range(3):
        q[k, 0] = np.where(x < 0.3, post[k], [1.0, 0.0, 2.5][k])
    qo, dts, info = oracle_run(spec, q, 0.4)
    s = solver(spec, q)
    st = s.advance(0.4)
    assert st["accepted"] == info["accepted"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


def test_full_size_shock_bubble_one_step():
    say("case: shock-bubble 2048x1024, 6 replayed steps from the seeded state")
    spec, q = W.shock_bubble(2048, 1024)
    g, o, _ = full_size_replay(spec, q, 6)
    e = fp64_err(g, o, spec)
    say("max rel err", e)
    assert e <= 1e-12


# --------------------------------------------------------------------------
# SharpClaw variants: SSPRK(10,4) (the SharpClaw default) and WENO7
# --------------------------------------------------------------------------
VARIANTS = [("ssp104", 5), ("ssp33", 7), ("ssp104", 7)]


@pytest.mark.parametrize("integ,order", VARIANTS)
def test_sharpclaw_variant_shock_bubble_replay(integ, order):
    say("case: shock-bubble 128x64", integ, "WENO", order, "20 steps")
    spec, q = W.shock_bubble(128, 64)
    spec = dict(spec, time_integrator=integ, weno_order=order)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=20)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("integ,order", VARIANTS)
def test_sharpclaw_variant_ragged_periodic(integ, order):
    say("case: smooth periodic Euler 77x61", integ, "WENO", order, "12 steps")
    spec, q = W.random_smooth_euler(77, seed=5)
    q = q[:, :61, :].copy()
    spec = dict(spec, num_cells=(77, 61), upper=(1.0, 61 / 77), time_integrator=integ,
                weno_order=order)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=12)
    g = replay(spec, q, info["dts"][info["acc"] == 1], seg_rows=7)
    assert fp64_err(g, qo, spec) <= 1e-12


def test_sharpclaw_weno7_advection_walls_replay():
    say("case: SharpClaw WENO7 advection 70x50, wall/extrap BCs, 15 steps")
    rng = np.random.default_rng(11)
    spec = dict(ndim=2, num_cells=(70, 50), lower=(0.0, 0.0), upper=(1.4, 1.0),
                scheme="sharpclaw", riemann="advection", problem_data=[0.7, -0.4],
                bc_lower=("wall", "extrap"), bc_upper=("extrap", "wall"), weno_order=7,
                time_integrator="ssp104", cfl_desired=0.7, cfl_max=0.8)
    q = rng.uniform(0.5, 1.5, (1, 50, 70))
    qo, info = oracle.advance(spec, q, 1.0, max_steps=15)
    g = replay(spec, q, info["dts"][info["acc"] == 1], seg_rows=9)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("integ,order", VARIANTS)
def test_sharpclaw_variant_1d_planar_shock_device_controller(integ, order):
    say("case: SharpClaw 1D planar shock, 300 cells,", integ, "WENO", order)
    rho1, u1, p1, S = W.rankine_hugoniot(2.0)
    n = 300
    post = [rho1, rho1 * u1, p1 / 0.4 + 0.5 * rho1 * u1 * u1]
    spec = dict(ndim=1, num_cells=(n,), lower=(0.0,), upper=(2.0,), scheme="sharpclaw",
                riemann="euler_hlle", problem_data=[1.4], bc_lower=("dirichlet",),
                bc_upper=("extrap",), bc_state={"x_lower": post}, cfl_desired=0.5, cfl_max=0.6,
                time_integrator=integ, weno_order=order)
    x = (np.arange(n) + 0.5) * 2.0 / n
    q = np.zeros((3, 1, n))
    for k in range(3):
        q[k, 0] = np.where(x < 0.3, post[k], [1.0, 0.0, 2.5][k])
    qo, dts, info = oracle_run(spec, q, 0.3)
    s = solver(spec, q)
    st = s.advance(0.3, steps_per_graph=4)
    assert st["accepted"] == info["accepted"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


def test_sharpclaw_ssp104_device_vs_host_controller():
    say("case: shock-bubble 96x48 SSPRK(10,4) WENO7, host vs device controller")
    spec, q = W.shock_bubble(96, 48)
    spec = dict(spec, time_integrator="ssp104", weno_order=7, cfl_desired=0.7, cfl_max=0.8)
    qo, dts, info = oracle_run(spec, q, 0.03)
    a = solver(spec, q)
    sa = a.advance(0.03, graph=False)
    b = solver(spec, q)
    sb = b.advance(0.03, graph=True, steps_per_graph=3)
    assert sa["accepted"] == sb["accepted"] == info["accepted"]
    np.testing.assert_array_equal(a.get_state(), b.get_state())
    assert fp64_err(b.get_state(), qo, spec) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_sharpclaw_weno7_tiling_does_not_change_results(prec):
    say("case: WENO7 SSPRK(10,4) seg_rows 3/16/100 bitwise equal", prec)
    spec, q = W.shock_bubble(150, 100)
    spec = dict(spec, precision=prec, time_integrator="ssp104", weno_order=7)
    outs = [replay(spec, q, [1e-3] * 4, seg_rows=sr) for sr in (3, 16, 100)]
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_full_size_shock_bubble_weno7_ssp104_one_step():
    say("case: shock-bubble 2048x1024 WENO7 SSPRK(10,4), one replayed step from the seeded state")
    spec, q = W.shock_bubble(2048, 1024)
    spec = dict(spec, time_integrator="ssp104", weno_order=7, cfl_desired=0.7, cfl_max=0.8)
    g, o, _ = full_size_replay(spec, q, 1, reps=1)
    e = fp64_err(g, o, spec)
    say("max rel err", e)
    assert e <= 1e-12


@pytest.mark.parametrize("integ,order", VARIANTS)
def test_fp32_kahan_sharpclaw_variant_l1(integ, order):
    # 60 steps: the shock has entered the bubble, so rho*v is no longer zero
    # up to rounding (its L1 norm would otherwise be pure noise)
    say("case: FP32+Kahan shock-bubble 256x128,", integ, "WENO", order, "60 steps (replayed dt)")
    spec, q = W.shock_bubble(256, 128)
    spec = dict(spec, time_integrator=integ, weno_order=order)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=60)
    g = replay(dict(spec, precision="fp32_kahan"), q, info["dts"][info["acc"] == 1])
    err = l1_rel(g, qo)
    errg = l1_rel_groups(g, qo, spec)
    say("L1 relative errors", err, "on the unit-group scale", errg)
    assert max(errg) <= 1e-4
    assert max(err[0], err[1], err[3]) <= 1e-5


# --------------------------------------------------------------------------
# WENO of orders 9 to 17 (generated reconstructions; r = 5 .. 9 halo lanes).
# Linear advection meets 1e-12 directly; where the method amplifies rounding
# beyond it (nonlinear data: the shock-bubble, smooth Euler, the planar
# shock) the bar is the case's own rounding sensitivity (rounding_tol).
# --------------------------------------------------------------------------
HIGH_ORDERS = [9, 11, 13, 15, 17]


@pytest.mark.parametrize("order", HIGH_ORDERS)
def test_sharpclaw_high_order_advection_walls_replay(order):
    say("case: SharpClaw advection 70x50, wall/extrap BCs, WENO", order, "10 steps")
    rng = np.random.default_rng(11)
    spec = dict(ndim=2, num_cells=(70, 50), lower=(0.0, 0.0), upper=(1.4, 1.0),
                scheme="sharpclaw", riemann="advection", problem_data=[0.7, -0.4],
                bc_lower=("wall", "extrap"), bc_upper=("extrap", "wall"), weno_order=order,
                time_integrator="ssp104", cfl_desired=0.7, cfl_max=0.8)
    q = rng.uniform(0.5, 1.5, (1, 50, 70))
    qo, info = oracle.advance(spec, q, 1.0, max_steps=10)
    g = replay(spec, q, info["dts"][info["acc"] == 1], seg_rows=9)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("order", HIGH_ORDERS)
def test_sharpclaw_high_order_shock_bubble_replay(order):
    say("case: shock-bubble 128x64, SSPRK(10,4), WENO", order, "12 steps")
    spec, q = W.shock_bubble(128, 64)
    spec = dict(spec, time_integrator="ssp104", weno_order=order)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=12)
    dts = info["dts"][info["acc"] == 1]
    g = replay(spec, q, dts)
    e = fp64_err(g, qo, spec)
    say("max rel err", e)
    assert e <= rounding_tol(spec, q, dts)


@pytest.mark.parametrize("order", HIGH_ORDERS)
def test_sharpclaw_high_order_ragged_periodic(order):
    say("case: smooth periodic Euler 77x61, SSPRK(10,4), WENO", order, "4 steps")
    spec, q = W.random_smooth_euler(77, seed=5)
    q = q[:, :61, :].copy()
    spec = dict(spec, num_cells=(77, 61), upper=(1.0, 61 / 77), time_integrator="ssp104",
                weno_order=order, cfl_desired=2.45, cfl_max=2.5)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=4)
    dts = info["dts"][info["acc"] == 1]
    g = replay(spec, q, dts, seg_rows=7)
    assert fp64_err(g, qo, spec) <= rounding_tol(spec, q, dts)


@pytest.mark.parametrize("order", HIGH_ORDERS)
def test_sharpclaw_high_order_1d_planar_shock_device_controller(order):
    say("case: SharpClaw 1D planar shock, 300 cells, SSPRK(10,4), WENO", order)
    rho1, u1, p1, S = W.rankine_hugoniot(2.0)
    n = 300
    post = [rho1, rho1 * u1, p1 / 0.4 + 0.5 * rho1 * u1 * u1]
    spec = dict(ndim=1, num_cells=(n,), lower=(0.0,), upper=(2.0,), scheme="sharpclaw",
                riemann="euler_hlle", problem_data=[1.4], bc_lower=("dirichlet",),
                bc_upper=("extrap",), bc_state={"x_lower": post}, cfl_desired=1.5, cfl_max=2.0,
                time_integrator="ssp104", weno_order=order)
    x = (np.arange(n) + 0.5) * 2.0 / n
    q = np.zeros((3, 1, n))
    for k in range(3):
        q[k, 0] = np.where(x < 0.3, post[k], [1.0, 0.0, 2.5][k])
    qo, dts, info = oracle_run(spec, q, 0.1)
    s = solver(spec, q)
    st = s.advance(0.1, steps_per_graph=4)
    assert st["accepted"] == info["accepted"]
    assert fp64_err(s.get_state(), qo, spec) <= rounding_tol(spec, q, dts)


@pytest.mark.parametrize("order", [9, 17])
def test_full_size_shock_bubble_high_order_window_one_step(order):
    """The benchmark's grid (2048x1024, SSPRK(10,4), CFL 2.45) in the tiling
    the autotuner picks: one GPU step from the seeded state, and 64x64
    windows of it (the shock front, the inflow corner, the far corner, the
    bubble's edge) against the oracle run on the window plus a margin of
    10 r + 2 cells (one step of ten stages reaches 10 r cells each way).
    Errors are measured on the scales of the whole grid."""
    say("case: shock-bubble 2048x1024 WENO", order, "SSPRK(10,4), windowed parity of one step")
    spec, q = W.shock_bubble(2048, 1024)
    spec = dict(spec, time_integrator="ssp104", weno_order=order, cfl_desired=2.45, cfl_max=2.5)
    dt = apriori_dt(spec, q)
    s = solver(spec, q)
    s.autotune(reps=1)
    s.step(dt)
    g = s.get_state()
    s.close()
    mg = 10 * (order + 1) // 2 + 2
    wins = [(480, 180), (0, 0), (960, 1984), (300, 420)]
    outs = [windowed_oracle(spec, q, [dt], j0, i0, mg) for (j0, i0) in wins]
    scales = np.max([fp64_scales(q, spec)] + [fp64_scales(o[0], spec) for o in outs], axis=0)
    for (j0, i0), (ow, ws, qw, _, region) in zip(wins, outs):
        gw = g[:, j0:j0 + 64, i0:i0 + 64]
        e = fp64_err(gw, ow, spec, scales)
        say("window", (j0, i0), "max rel err", e)
        assert e <= rounding_tol(ws, qw, [dt], region=region, scales=scales), (j0, i0)


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_sharpclaw_weno17_tiling_does_not_change_results(prec):
    say("case: WENO17 SSPRK(10,4) seg_rows 3/16/100 bitwise equal", prec)
    spec, q = W.shock_bubble(150, 100)
    spec = dict(spec, precision=prec, time_integrator="ssp104", weno_order=17)
    outs = [replay(spec, q, [1e-3] * 3, seg_rows=sr) for sr in (3, 16, 100)]
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def fp32_rounding_l1(spec, q, dts):
    """L1 errors (plain and on the unit-group scale) that FP32 rounding alone
    produces in this case: the oracle run with its state perturbed by the
    FP32 unit roundoff (relative 6e-8, seeded) before every step, against the
    unperturbed run."""
    rng = np.random.default_rng(54321)
    ref = np.array(q, dtype=np.float64)
    x = ref.copy()
    for dt in dts:
        ref, _ = oracle.step(spec, ref, dt)
        x, _ = oracle.step(spec, x * (1.0 + 6e-8 * rng.standard_normal(x.shape)), dt)
    return l1_rel(x, ref), l1_rel_groups(x, ref, spec)


@pytest.mark.parametrize("order", [9, 17])
def test_fp32_kahan_sharpclaw_high_order_l1(order):
    # 20 steps at Courant 2.45: the shock has entered the bubble (rho*v is
    # no longer zero up to rounding)
    say("case: FP32+Kahan shock-bubble 256x128, SSPRK(10,4), WENO", order, "20 steps (replayed dt)")
    spec, q = W.shock_bubble(256, 128)
    spec = dict(spec, time_integrator="ssp104", weno_order=order, cfl_desired=2.45, cfl_max=2.5)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=20)
    dts = info["dts"][info["acc"] == 1]
    g = replay(dict(spec, precision="fp32_kahan"), q, dts)
    err = l1_rel(g, qo)
    errg = l1_rel_groups(g, qo, spec)
    say("L1 relative errors", err, "on the unit-group scale", errg)
    # the FP32 bars, or 3x what FP32 rounding alone does to this case where
    # the high-order weights amplify it more (order 17: about 3e-4)
    sens, sensg = fp32_rounding_l1(spec, q, dts)
    say("FP32-rounding L1 of the oracle", sens, sensg)
    for k in range(4):
        assert errg[k] <= max(1e-4, 3.0 * sensg[k])
    for k in (0, 1, 3):
        assert err[k] <= max(1e-5, 3.0 * sens[k])


# --------------------------------------------------------------------------
# Classic Euler: Roe solver + transverse split (+ tracer, + axisymmetric
# source as a fractional step)
# --------------------------------------------------------------------------
def test_listing1_riemann_problem_classic_euler():
    say("case: Listing 1 2D Euler Riemann problem 100x100, classic Roe, to t=0.3 on the device")
    spec, q = W.listing1_riemann(100)
    qo, dts, info = oracle_run(spec, q, 0.3)
    s = solver(spec, q)
    st = s.advance(0.3, steps_per_graph=8)
    assert st["accepted"] == info["accepted"] and st["rejected"] == info["rejected"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


@pytest.mark.parametrize("tracer,efix", [(0, 0), (1, 1)])
def test_euler_roe_ragged_periodic_replay(tracer, efix):
    say("case: smooth periodic Euler Roe 77x61, tracer", tracer, "efix", efix, "15 steps")
    spec, q = W.random_smooth_euler(77, seed=7)
    q = q[:, :61, :].copy()
    if tracer:
        q = np.concatenate([q, np.random.default_rng(3).uniform(0, 1, (1, 61, 77))])
    spec = dict(spec, scheme="classic", riemann="euler_roe", num_cells=(77, 61),
                upper=(1.0, 61 / 77), limiter="mc", transverse=2, tracer=tracer, entropy_fix=efix,
                cfl_desired=0.8, cfl_max=0.9)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=15)
    g = replay(spec, q, info["dts"][info["acc"] == 1], seg_rows=9)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("trans,lim", [(0, "none"), (1, "minmod"), (2, "mc")])
def test_axisym_shock_bubble_replay(trans, lim):
    say("case: axisymmetric shock-bubble 160x40 (tracer, source), transverse", trans, lim)
    spec, q = W.shock_bubble_axisym(160, 40)
    spec = dict(spec, transverse=trans, limiter=lim)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=25)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


def test_euler_roe_1d_sod_device_controller():
    say("case: 1D Euler Roe Sod 500 cells (one-workgroup run kernel), entropy fix")
    n = 500
    spec = dict(ndim=1, num_cells=(n,), lower=(-0.5,), upper=(0.5,), scheme="classic",
                riemann="euler_roe", problem_data=[1.4], entropy_fix=1, limiter="mc",
                bc_lower=("extrap",), bc_upper=("extrap",), cfl_desired=0.8, cfl_max=0.9)
    x = -0.5 + (np.arange(n) + 0.5) / n
    q = np.zeros((3, 1, n))
    q[0, 0] = np.where(x < 0, 1.0, 0.125)
    q[1, 0] = np.where(x < 0, 0.75, 0.0)
    q[2, 0] = np.where(x < 0, 1.0 / 0.4 + 0.5 * 0.75 ** 2, 0.1 / 0.4)
    qo, dts, info = oracle_run(spec, q, 0.2)
    s = solver(spec, q)
    st = s.advance(0.2)
    assert st["accepted"] == info["accepted"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12
    # and the strip kernel (replayed dt)
    g = replay(spec, q, dts)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_euler_roe_tiling_does_not_change_results(prec):
    say("case: axisymmetric shock-bubble seg_rows 4/16/100 bitwise equal", prec)
    spec, q = W.shock_bubble_axisym(150, 100)
    spec = dict(spec, precision=prec)
    outs = [replay(spec, q, [4e-4] * 6, seg_rows=sr) for sr in (4, 16, 100)]
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_full_size_axisym_shock_bubble_one_step():
    say("case: axisymmetric shock-bubble 1280x320, 10 replayed steps from the seeded state")
    spec, q = W.shock_bubble_axisym(1280, 320)
    g, o, _ = full_size_replay(spec, q, 10, reps=1)
    e = fp64_err(g, o, spec)
    say("max rel err", e)
    assert e <= 1e-12


def test_fp32_kahan_axisym_shock_bubble_l1():
    say("case: FP32+Kahan axisymmetric shock-bubble 320x80, 80 steps (replayed dt)")
    spec, q = W.shock_bubble_axisym(320, 80)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=80)
    g = replay(dict(spec, precision="fp32_kahan"), q, info["dts"][info["acc"] == 1])
    err = l1_rel(g, qo)
    errg = l1_rel_groups(g, qo, spec)
    say("L1 relative errors", err, "on the unit-group scale", errg)
    assert max(errg) <= 1e-5 and max(err[0], err[1], err[3], err[4]) <= 1e-5


# --------------------------------------------------------------------------
# FP32 with Kahan-compensated update
# --------------------------------------------------------------------------
def test_fp32_kahan_radial_dam_break_l1():
    say("case: FP32+Kahan radial dam break 256^2 to t=0.25 (replayed dt)")
    spec, q = W.radial_dam_break(256)
    qo, dts, _ = oracle_run(spec, q, 0.25)
    g = replay(dict(spec, precision="fp32_kahan"), q, dts)
    err = l1_rel(g, qo)
    say("L1 relative errors", err)
    assert max(err) <= 1e-5


def test_fp32_kahan_shock_bubble_l1():
    say("case: FP32+Kahan shock-bubble 256x128, 60 steps (replayed dt)")
    spec, q = W.shock_bubble(256, 128)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=60)
    g = replay(dict(spec, precision="fp32_kahan"), q, info["dts"][info["acc"] == 1])
    err = l1_rel(g, qo)
    say("L1 relative errors", err)
    assert max(err) <= 1e-4


def test_fp32_kahan_elastic_l1():
    say("case: FP32+Kahan layered elasticity 128^2, 60 steps (replayed dt)")
    spec, q, aux = W.layered_elastic(128)
    qo, info = oracle.advance(spec, q, 1.0, aux=aux, max_steps=60)
    g = replay(dict(spec, precision="fp32_kahan"), q, info["dts"][info["acc"] == 1], aux=aux)
    err = l1_rel(g, qo)
    say("L1 relative errors", err)
    assert max(err) <= 1e-4


def test_fp32_kahan_long_run_l1():
    """FP32+Kahan over a whole run (t=0.3, ~100 steps at 128^2) stays within
    the shallow-water L1 bar."""
    say("case: FP32+Kahan radial 128^2 to t=0.3 (replayed dt)")
    spec, q = W.radial_dam_break(128)
    qo, dts, _ = oracle_run(spec, q, 0.3)
    g = replay(dict(spec, precision="fp32_kahan"), q, dts)
    err = l1_rel(g, qo)
    say("L1 relative errors", err)
    assert max(err) <= 1e-5


# --------------------------------------------------------------------------
# Controller, graphs, tiling, batching, checkpoint, failures
# --------------------------------------------------------------------------
@pytest.mark.parametrize("graph", [False, True])
def test_controller_rejection_sequence_1d(graph):
    say("case: forced rejection with dt_initial=1.0 on 16 cells")
    spec, q = W.dam_break_1d(16)
    spec = dict(spec, dt_initial=1.0)
    qo, info = oracle.advance(spec, q, 0.5)
    s = solver(spec, q)
    st = s.advance(0.5, graph=graph)
    assert (st["accepted"], st["rejected"]) == (info["accepted"], info["rejected"])
    assert st["rejected"] >= 1 and st["t"] == 0.5
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


@pytest.mark.parametrize("graph", [False, True])
def test_controller_rejection_sequence_2d(graph):
    say("case: forced rejection 2D 20x18")
    spec, q = W.radial_dam_break(20, ny=18)
    spec = dict(spec, dt_initial=5.0)
    qo, info = oracle.advance(spec, q, 0.4)
    s = solver(spec, q)
    st = s.advance(0.4, graph=graph)
    assert (st["accepted"], st["rejected"]) == (info["accepted"], info["rejected"])
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


def test_sharpclaw_controller_device_vs_host():
    say("case: shock-bubble 96x48 advance on host vs device controller")
    spec, q = W.shock_bubble(96, 48)
    qo, dts, info = oracle_run(spec, q, 0.05)
    a = solver(spec, q)
    sa = a.advance(0.05, graph=False)
    b = solver(spec, q)
    sb = b.advance(0.05, graph=True, steps_per_graph=4)
    assert sa["accepted"] == sb["accepted"] == info["accepted"]
    np.testing.assert_array_equal(a.get_state(), b.get_state())
    assert fp64_err(b.get_state(), qo, spec) <= 1e-12


def test_graph_advance_bitwise_equals_host_advance():
    say("case: radial 128^2 graph vs host controller, bitwise")
    spec, q = W.radial_dam_break(128)
    a = solver(spec, q)
    a.advance(0.2, graph=False)
    b = solver(spec, q)
    b.advance(0.2, graph=True, steps_per_graph=8)
    assert a.clock()["accepted"] == b.clock()["accepted"]
    np.testing.assert_array_equal(a.get_state(), b.get_state())


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_tiling_does_not_change_results(prec):
    say("case: seg_rows 4/16/100 bitwise equal", prec)
    spec, q = W.radial_dam_break(150, ny=100)
    spec = dict(spec, precision=prec)
    outs = []
    for sr in (4, 16, 100):
        outs.append(replay(spec, q, [2e-3] * 12, seg_rows=sr))
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
    # segment counts whose segments start on odd and even rows alike, in
    # every tile order
    for segs, order in ((7, 0), (13, 1), (37, 2), (13, 3), (7, 3)):
        s = solver(spec, q)
        s.set_tuning(segs=segs, order=order)
        for _ in range(12):
            s.step(2e-3)
        np.testing.assert_array_equal(s.get_state(), outs[0])
        s.close()


@pytest.mark.parametrize("order", [0, 1, 2, 3])
def test_tile_order_does_not_change_results(order):
    """Every tile order gives the same bits on every path: classic 2D, split
    sweeps, SharpClaw (FP32 ring and FP64 register windows)."""
    say("case: tile order", order, "bitwise, classic / split / SharpClaw")
    sw, qs = W.radial_dam_break(130, ny=77)
    eu, qe = W.shock_bubble(150, 70)
    for spec, q, dt in ((sw, qs, 2e-3), (dict(sw, dimensional_split="strang"), qs, 2e-3),
                        (eu, qe, 1e-3), (dict(eu, precision="fp32_kahan"), qe, 1e-3)):
        ref = replay(spec, q, [dt] * 5, seg_rows=9)
        s = solver(spec, q)
        s.set_tuning(segs=11, order=order)
        for _ in range(5):
            s.step(dt)
        np.testing.assert_array_equal(s.get_state(), ref)
        s.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_elastic_tiling_does_not_change_results(prec):
    say("case: layered elasticity 120x90, seg_rows 8 / segs 7, 13 / one segment, bitwise", prec)
    spec, q, aux = W.layered_elastic(120, ny=90)
    spec = dict(spec, precision=prec)
    ref = replay(spec, q, [1e-3] * 8, aux=aux, seg_rows=8)
    for segs in (7, 13, 1):
        s = solver(spec, q, aux)
        s.set_tuning(segs=segs)
        for _ in range(8):
            s.step(1e-3)
        np.testing.assert_array_equal(s.get_state(), ref)
        s.close()


def test_batch_results_equal_alone_and_in_mix():
    say("case: batch of 4 uneven grids vs each alone (FP32+Kahan, bitwise)")
    from paper_1111_6583_amd import Batch
    trace = W.serving_trace(n_requests=4, seed=5, nmin=48, nmax=200, t_end=0.15)
    alone = []
    for r in trace:
        spec, q = W.request_problem(r)
        s = solver(spec, q)
        s.advance(r["t_end"])
        alone.append((s.get_state(), s.clock()))
    b = Batch(8)
    members = []
    for r in trace:
        spec, q = W.request_problem(r)
        s = solver(spec, q)
        b.add(s, r["t_end"])
        members.append(s)
    while b.advance(16) > 0:
        pass
    for (qa, ca), s in zip(alone, members):
        ck = b.member_clock(s)
        assert ck["t"] == ca["t"] and ck["accepted"] == ca["accepted"]
        b.remove(s)
        np.testing.assert_array_equal(s.get_state(), qa)


def test_totals_match_oracle():
    say("case: totals after 20 steps, FP64 and FP32+Kahan")
    spec, q = W.random_smooth_sw(96, seed=4)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=20)
    for prec, tol in (("fp64", 1e-13), ("fp32_kahan", 1e-6)):
        s = solver(dict(spec, precision=prec), q)
        for dt in info["dts"][info["acc"] == 1]:
            s.step(dt)
        np.testing.assert_allclose(s.totals(), oracle.totals(spec, qo), rtol=tol, atol=tol)


def test_checkpoint_resume_bitwise():
    """Run to t=0.1 and on to t=0.25 in one handle; separately checkpoint at
    t=0.1 (state + clock), restore into a new handle and continue: the two
    are bitwise equal (the restored clock carries the controller's dt)."""
    say("case: checkpoint at t=0.1, resume in a new handle, compare at t=0.25")
    spec, q = W.radial_dam_break(96)
    a = solver(spec, q)
    a.advance(0.1)
    snap, ck = a.get_state(), a.clock()
    a.advance(0.25)
    c = solver(spec, snap)
    c.set_clock(ck)
    c.advance(0.25)
    assert c.clock()["accepted"] == a.clock()["accepted"]
    assert c.clock()["t"] == a.clock()["t"] == 0.25
    np.testing.assert_array_equal(c.get_state(), a.get_state())


def test_nonphysical_state_reported():
    say("case: NaN in the initial state -> CLAW_E_NONPHYSICAL")
    from paper_1111_6583_amd._claw import ClawError
    spec, q = W.radial_dam_break(64)
    q = q.copy()
    q[0, 10, 10] = np.nan
    s = solver(dict(spec, dt_initial=1e-3), q)
    with pytest.raises(ClawError) as e:
        s.advance(0.1, graph=False)
    assert e.value.rc == -5
    s2 = solver(dict(spec, dt_initial=1e-3), q)
    with pytest.raises(ClawError) as e:
        s2.advance(0.1, graph=True)
    assert e.value.rc == -5


def test_autotune_keeps_results():
    say("case: autotune picks a tiling; results unchanged")
    spec, q = W.radial_dam_break(256)
    base = replay(spec, q, [1e-3] * 5, seg_rows=16)
    s = solver(spec, q)
    sr = s.autotune(reps=2)
    assert sr >= 1
    for _ in range(5):
        s.step(1e-3)
    np.testing.assert_array_equal(s.get_state(), base)


# --------------------------------------------------------------------------
# Dimensionally split classic steps (Godunov x-then-y, Strang x/2 y x/2)
# --------------------------------------------------------------------------
SPLITS = ["godunov", "strang"]


@pytest.mark.parametrize("split", SPLITS)
def test_split_radial_dam_break_ragged_replay(split):
    say("case: split", split, "radial dam break 150x100 (ragged strips and segments), 30 steps")
    spec, q = W.radial_dam_break(150, ny=100)
    spec = dict(spec, dimensional_split=split)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=30)
    dts = info["dts"][info["acc"] == 1]
    assert len(dts) == 30
    g = replay(spec, q, dts, seg_rows=9)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("bcl,bcu", BC_CASES[1:])
def test_split_sw_boundary_conditions(split, bcl, bcu):
    say("case: split", split, "SW hump 70x66 bcs", bcl, bcu)
    spec, q = W.sw_hump(70, amplitude=0.6, width=0.15, x0=(0.3, 0.65))
    q = q[:, :66, :].copy()
    spec = dict(spec, num_cells=(70, 66), upper=(1.0, 66 / 70), bc_lower=bcl, bc_upper=bcu,
                dimensional_split=split)
    q[1] = 0.2 * q[0]
    q[2] = -0.1 * q[0]
    qo, info = oracle.advance(spec, q, 1.0, max_steps=25)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("split", SPLITS)
def test_split_sw_dirichlet_sides(split):
    say("case: split", split, "SW with Dirichlet sides")
    spec, q = W.sw_hump(64, amplitude=0.5, width=0.2)
    spec = dict(spec, bc_lower=("dirichlet", "wall"), bc_upper=("extrap", "dirichlet"),
                bc_state={"x_lower": [1.5, 0.3, 0.0], "y_upper": [1.2, 0.0, -0.2]},
                dimensional_split=split)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=25)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("lim", ["none", "minmod"])
def test_split_limiters_and_advection_exact_shift(lim):
    say("case: split advection 64x48, Courant 1 per sweep, limiter", lim)
    nx, ny = 64, 48
    dt = 1.0 / nx
    spec = dict(ndim=2, num_cells=(nx, ny), lower=(0, 0), upper=(1, 1), riemann="advection",
                limiter=lim, bc_lower=("periodic", "periodic"), bc_upper=("periodic", "periodic"),
                problem_data=[2.0, (1.0 / ny) / dt], dimensional_split="strang")
    q0 = np.random.default_rng(21).standard_normal((1, ny, nx))
    g = replay(spec, q0, [dt] * 5)
    np.testing.assert_allclose(g, np.roll(q0, (5, 10), axis=(1, 2)), rtol=0, atol=1e-12)
    spec = dict(spec, problem_data=[0.7, -0.45], dimensional_split="godunov")
    qo = q0
    for _ in range(12):
        qo, _ = oracle.step(spec, qo, 0.8 / nx)
    g = replay(spec, q0, [0.8 / nx] * 12)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("split", SPLITS)
def test_split_layered_elastic_replay(split):
    say("case: split", split, "layered elasticity 96x80, 20 steps")
    spec, q, aux = W.layered_elastic(96, ny=80)
    spec = dict(spec, dimensional_split=split)
    qo, info = oracle.advance(spec, q, 1.0, aux=aux, max_steps=20)
    g = replay(spec, q, info["dts"][info["acc"] == 1], aux=aux)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("split", SPLITS)
def test_split_axisym_shock_bubble_replay(split):
    say("case: split", split, "axisymmetric shock-bubble 160x40 (tracer, source), 25 steps")
    spec, q = W.shock_bubble_axisym(160, 40)
    spec = dict(spec, dimensional_split=split)
    qo, info = oracle.advance(spec, q, 1.0, max_steps=25)
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("split", SPLITS)
@pytest.mark.parametrize("graph", [False, True])
def test_split_controller_with_rejection(split, graph):
    say("case: split", split, "forced rejection 2D 40x36, graph", graph)
    spec, q = W.radial_dam_break(40, ny=36)
    spec = dict(spec, dt_initial=5.0, dimensional_split=split)
    qo, info = oracle.advance(spec, q, 0.4)
    s = solver(spec, q)
    st = s.advance(0.4, graph=graph, steps_per_graph=4)
    assert (st["accepted"], st["rejected"]) == (info["accepted"], info["rejected"])
    assert st["rejected"] >= 1 and st["t"] == 0.4
    assert st["max_courant"] == pytest.approx(info["max_courant"], rel=1e-12)
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_split_tiling_does_not_change_results(prec):
    say("case: split strang seg_rows 4/16/100 bitwise equal", prec)
    spec, q = W.radial_dam_break(150, ny=100)
    spec = dict(spec, precision=prec, dimensional_split="strang")
    outs = [replay(spec, q, [2e-3] * 10, seg_rows=sr) for sr in (4, 16, 100)]
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])
    for sr, sx in ((5, 1), (100, 7), (16, 100)):   # x sweeps tiled on their own
        s = solver(spec, q)
        s.set_tuning(sr, sx)
        for _ in range(10):
            s.step(2e-3)
        np.testing.assert_array_equal(s.get_state(), outs[0])
        s.close()


@pytest.mark.parametrize("split", SPLITS)
def test_fp32_kahan_split_radial_dam_break_l1(split):
    say("case: FP32+Kahan split", split, "radial dam break 256^2 to t=0.25 (replayed dt)")
    spec, q = W.radial_dam_break(256)
    spec = dict(spec, dimensional_split=split)
    qo, dts, _ = oracle_run(spec, q, 0.25)
    g = replay(dict(spec, precision="fp32_kahan"), q, dts)
    err = l1_rel_groups(g, qo, spec)
    say("L1 relative errors (unit-group scale)", err)
    assert max(err) <= 1e-5


@pytest.mark.parametrize("split", SPLITS)
def test_full_size_split_radial_dam_break_one_step(split):
    say("case: split", split, "radial dam break 1024^2, 10 replayed steps from the seeded state")
    spec, q = W.radial_dam_break(1024)
    spec = dict(spec, dimensional_split=split)
    g, o, _ = full_size_replay(spec, q, 10)
    e = fp64_err(g, o, spec)
    say("max rel err", e)
    assert e <= 1e-12


# --------------------------------------------------------------------------
# Nonlinear p-system in a checkerboard medium (SharpClaw, f-wave flux)
# --------------------------------------------------------------------------
PSYS_VARIANTS = [("ssp104", 5), ("ssp33", 5), ("ssp104", 7), ("ssp104", 11)]


@pytest.mark.parametrize("integ,order", PSYS_VARIANTS)
def test_psystem_checkerboard_ragged_replay(integ, order):
    say("case: p-system checkerboard 70x50 (10 cells/period),", integ, "WENO", order, "12 steps")
    spec, q, aux = W.psystem_checkerboard(10, 7, ny_periods=5, time_integrator=integ,
                                          weno_order=order,
                                          cfl_desired=2.45 if integ == "ssp104" else 0.5,
                                          cfl_max=2.5 if integ == "ssp104" else 0.6)
    qo, info = oracle.advance(spec, q, 100.0, aux=aux, max_steps=12)
    dts = info["dts"][info["acc"] == 1]
    g = replay(spec, q, dts, aux=aux, seg_rows=7)
    assert fp64_err(g, qo, spec) <= (1e-12 if order <= 7 else rounding_tol(spec, q, dts, aux))


def test_psystem_periodic_and_mixed_boundaries():
    say("case: p-system checkerboard 64x48, periodic x / wall-extrap y, 10 steps")
    spec, q, aux = W.psystem_checkerboard(8, 8, ny_periods=6, bc_lower=("periodic", "wall"),
                                          bc_upper=("periodic", "extrap"))
    q[1] = 0.2 * np.cos(2 * np.pi * np.arange(64) / 64.0)[None, :]
    qo, info = oracle.advance(spec, q, 100.0, aux=aux, max_steps=10)
    g = replay(spec, q, info["dts"][info["acc"] == 1], aux=aux)
    assert fp64_err(g, qo, spec) <= 1e-12


def test_psystem_1d_interface_device_controller():
    say("case: 1D p-system impedance interface, 300 cells, device controller to t=0.5")
    n = 300
    spec, aux = W.psystem_layered_1d(n, interfaces=(0.5,), materials=((1.0, 1.0), (5.0, 5.0)))
    x = (np.arange(n) + 0.5) / n
    q = np.zeros((2, 1, n))
    q[0, 0] = 0.05 * np.exp(-((x - 0.25) / 0.05) ** 2)
    q[1, 0] = -q[0, 0]
    qo, dts, info = oracle_run(spec, q, 0.5, aux=aux)
    s = solver(spec, q, aux)
    st = s.advance(0.5, steps_per_graph=8)
    assert st["accepted"] == info["accepted"] and st["rejected"] == info["rejected"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12
    g = replay(spec, q, dts, aux=aux)
    assert fp64_err(g, qo, spec) <= 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_psystem_tiling_does_not_change_results(prec):
    say("case: p-system checkerboard 96x80 seg_rows 4/16/80 bitwise equal", prec)
    spec, q, aux = W.psystem_checkerboard(8, 12, ny_periods=10, precision=prec)
    outs = [replay(spec, q, [0.02] * 3, aux=aux, seg_rows=sr) for sr in (4, 16, 80)]
    np.testing.assert_array_equal(outs[0], outs[1])
    np.testing.assert_array_equal(outs[0], outs[2])


def test_fp32_kahan_psystem_l1():
    say("case: FP32+Kahan p-system checkerboard 120x120 (12 cells/period), 30 steps")
    spec, q, aux = W.psystem_checkerboard(12, 10)
    qo, info = oracle.advance(spec, q, 100.0, aux=aux, max_steps=30)
    g = replay(dict(spec, precision="fp32_kahan"), q, info["dts"][info["acc"] == 1], aux=aux)
    err = l1_rel_groups(g, qo, spec)
    say("L1 relative errors (unit-group scale)", err)
    assert max(err) <= 1e-5


def test_full_size_psystem_window_one_step():
    """The benchmark's grid (20 x 20 periods at 240 cells per period, 4800^2)
    in its tiling: three GPU steps from the seeded state, and 64^2 windows of
    them against the oracle run on the window plus a 3 x 32-cell margin (one
    SSPRK(10,4) step reaches 10 x 3 cells each way).  Errors are measured on
    the scales of the whole grid."""
    say("case: p-system checkerboard 4800^2, windowed parity of 3 steps from the seeded state")
    spec, q, aux = W.psystem_checkerboard(240, 20)
    dt = apriori_dt(spec, q, aux)
    dts = [dt] * 3
    s = solver(spec, q, aux)
    s.autotune(reps=1)
    for d in dts:
        s.step(d)
    g = s.get_state()
    s.close()
    wins = [(700, 1900), (0, 0), (4736, 2500), (10, 300)]
    outs = [windowed_oracle(spec, q, dts, j0, i0, 3 * 32, aux=aux) for (j0, i0) in wins]
    scales = np.max([fp64_scales(q, spec)] + [fp64_scales(o[0], spec) for o in outs], axis=0)
    for (j0, i0), (ow, *_rest) in zip(wins, outs):
        gw = g[:, j0:j0 + 64, i0:i0 + 64]
        e = fp64_err(gw, ow, spec, scales)
        say("window", (j0, i0), "max rel err", e)
        assert e <= 1e-12, (j0, i0)


def test_batch_rejects_split_and_sharpclaw_members():
    say("case: claw_batch_add refuses split-step and SharpClaw handles (CLAW_E_INVAL)")
    from paper_1111_6583_amd import Batch
    from paper_1111_6583_amd._claw import ClawError
    b = Batch(2)
    spec, q = W.radial_dam_break(64)
    for bad in (dict(spec, dimensional_split="godunov"),):
        s = solver(bad, q)
        with pytest.raises(ClawError):
            b.add(s, 0.1)
        s.close()
    ps, pq, pa = W.psystem_checkerboard(8, 4)
    s = solver(ps, pq, pa)
    with pytest.raises(ClawError):
        b.add(s, 0.1)
    s.close()
    ok = solver(spec, q)
    b.add(ok, 0.05)
    while b.advance(8) > 0:
        pass
    b.remove(ok)
    ok.close()


# --------------------------------------------------------------------------
# Degenerate and edge cases: minimum grids, uniform states
# --------------------------------------------------------------------------
def _min_cases():
    sw, swq = W.radial_dam_break(4)
    swq = swq + 0.1 * np.random.default_rng(41).random(swq.shape)
    eu, euq = W.random_smooth_euler(4, seed=3)
    eu9, eu9q = W.random_smooth_euler(9, seed=3)
    ps, psq, psa = W.psystem_checkerboard(2, 2)
    el, elq, ela = W.layered_elastic(4)
    d1, d1q = W.dam_break_1d(4)
    return [("classic sw 4x4", sw, swq, None),
            ("classic sw 4x4 walls", dict(sw, bc_lower=("wall", "wall"), bc_upper=("wall", "wall")), swq, None),
            ("split strang sw 4x4", dict(sw, dimensional_split="strang"), swq, None),
            ("sharpclaw euler weno5 4x4", eu, euq, None),
            ("sharpclaw euler weno7 ssp104 4x4", dict(eu, weno_order=7, time_integrator="ssp104",
                                                      cfl_desired=2.45, cfl_max=2.5), euq, None),
            ("sharpclaw euler weno17 ssp104 9x9", dict(eu9, weno_order=17, time_integrator="ssp104",
                                                       cfl_desired=2.45, cfl_max=2.5), eu9q, None),
            ("sharpclaw euler weno17 9x9 walls", dict(eu9, weno_order=17, bc_lower=("wall", "wall"),
                                                      bc_upper=("wall", "wall")), eu9q, None),
            ("p-system 4x4", ps, psq, psa),
            ("elastic 4x4", el, elq, ela),
            ("classic sw 1d 4 cells", d1, d1q, None)]


@pytest.mark.parametrize("case", range(10))
def test_minimum_grid_every_path(case):
    name, spec, q, aux = _min_cases()[case]
    say("case: minimum grid,", name)
    qo, info = oracle.advance(spec, q, 1e9, aux=aux, max_steps=6)
    dts = info["dts"][info["acc"] == 1]
    g = replay(spec, q, dts, aux=aux)
    high = spec.get("scheme") == "sharpclaw" and spec.get("weno_order", 5) > 7
    assert fp64_err(g, qo, spec) <= (rounding_tol(spec, q, dts, aux) if high else 1e-12)


@pytest.mark.parametrize("prec", ["fp64", "fp32_kahan"])
def test_uniform_state_is_preserved_exactly(prec):
    """A uniform state on a periodic grid has no jumps: every solver must
    leave it unchanged, bit for bit (SharpClaw in FP32: to a few ulps, its
    stage combinations round).  Regression: a face flux fused, unrounded,
    into its own lane's flux difference while the neighbour used the
    rounded value made the p-system at rest drift by ~1e-20."""
    say("case: uniform periodic states stay put,", prec)
    per = dict(bc_lower=("periodic", "periodic"), bc_upper=("periodic", "periodic"), precision=prec)
    sw, _ = W.radial_dam_break(70, ny=66)
    eu, _ = W.random_smooth_euler(70, seed=1)
    ps, _, psa = W.psystem_checkerboard(6, 7, ny_periods=6)
    ax, _ = W.shock_bubble_axisym(70, 30)
    cases = [(dict(sw, **per), [1.3, 0.2, -0.1], None),
             (dict(sw, **per, dimensional_split="godunov"), [1.3, 0.2, -0.1], None),
             (dict(eu, **per), [1.1, 0.3, -0.2, 2.7], None),
             (dict(eu, **per, weno_order=7, time_integrator="ssp104", cfl_desired=2.45, cfl_max=2.5),
              [1.1, 0.3, -0.2, 2.7], None),
             (dict(eu, **per, weno_order=17, time_integrator="ssp104", cfl_desired=2.45, cfl_max=2.5),
              [1.1, 0.3, -0.2, 2.7], None),
             (dict(ax, **per, source="none"), [1.1, 0.3, -0.2, 2.7, 0.4], None),
             (dict(ps, **per), [0.05, 0.0, 0.0], np.ones_like(psa))]
    for spec, vals, aux in cases:
        nx, ny = spec["num_cells"]
        q = np.array(vals)[:, None, None] * np.ones((len(vals), ny, nx))
        g = replay(spec, q, [1e-3] * 4, aux=aux)
        q = replay(spec, q, [], aux=aux)   # the state as stored (FP32: rounded)
        if spec["scheme"] == "classic" or prec == "fp64":
            np.testing.assert_array_equal(g, q)
        else:
            np.testing.assert_allclose(g, q, rtol=0, atol=1e-6 * np.max(np.abs(q)))
