"""GPU parity for cases the other GPU tests do not reach, each against the
FP64 oracle (through the C ABI):

* the shallow-water Harten-Hyman entropy fix (paper Section 5: Roe's solver
  with an entropy fix) on transonic rarefactions, left- and right-going, in
  1D (strip kernel, host controller, one-workgroup run kernel) and in 2D
  (y-uniform, x-uniform and a radial collapse with the radial dam break's
  settings), with the oracle's state showing that the fix fires;
* the Courant number on cells with dx != dy (Section 4: one reduction of
  the maximum wave speed), for every 2D path;
* a batch of uneven grids (one launch per attempt, each grid on its own
  controller) in FP64 against the oracle's controller, and in FP32 with a
  Kahan-compensated update at the shallow-water L1 bar;
* requests served by the continuous-batching loop against the oracle.
"""

import math
import sys

import numpy as np
import pytest

import oracle
from paper_1111_6583_amd import workloads as W

from test_gpu_parity import fp64_err, l1_rel, replay, say, solver

pytestmark = pytest.mark.gpu


# --------------------------------------------------------------------------
# Entropy fix
# --------------------------------------------------------------------------
def sw_efix_faces(q, axis, g=1.0):
    """Faces (between neighbours along `axis` of a (m, ny, nx) shallow-water
    state) where the Harten-Hyman fix fires, per acoustic family: the
    characteristic speed is negative on the wave's left and positive on its
    right (test side, from the Roe waves written out)."""
    n = 1 + axis
    sl = [slice(None)] * 3
    sr = [slice(None)] * 3
    sl[2 - axis] = slice(None, -1)
    sr[2 - axis] = slice(1, None)
    ql, qr = q[tuple(sl)], q[tuple(sr)]
    hl, hr = ql[0], qr[0]
    ul, ur = ql[n] / hl, qr[n] / hr
    wl, wr = np.sqrt(hl), np.sqrt(hr)
    ub = (wl * ul + wr * ur) / (wl + wr)
    cb = np.sqrt(g * 0.5 * (hl + hr))
    dh, dm = hr - hl, qr[n] - ql[n]
    a1 = ((ub + cb) * dh - dm) / (2 * cb)
    a3 = (-(ub - cb) * dh + dm) / (2 * cb)
    h1, m1 = hl + a1, ql[n] + a1 * (ub - cb)
    first = (ul - np.sqrt(g * hl) < 0) & (m1 / h1 - np.sqrt(g * h1) > 0)
    h3, m3 = hr - a3, qr[n] - a3 * (ub + cb)
    last = (m3 / h3 + np.sqrt(g * h3) < 0) & (ur + np.sqrt(g * hr) > 0)
    return int(first.sum()), int(last.sum())


def _transonic_1d(mirror, n=1000):
    hl, hr = (0.05, 4.0) if mirror else (4.0, 0.05)
    return W.dam_break_1d(n, hl=hl, hr=hr)


@pytest.mark.parametrize("mirror", [False, True])
@pytest.mark.parametrize("mode", ["replay", "host", "device"])
def test_sw_entropy_fix_transonic_1d(mirror, mode):
    """cfg1 settings (Roe + fix, MC, CFL 0.9, extrapolation) on a transonic
    dam break (h 4 -> 0.05) and its mirror image, to t = 1."""
    say("case: 1D transonic dam break", "mirror" if mirror else "", mode)
    spec, q = _transonic_1d(mirror)
    qo, info = oracle.advance(spec, q, 1.0)
    assert info["rc"] == 0
    f1, f3 = sw_efix_faces(qo, 0)
    say("faces where the fix fires (first, last family):", f1, f3)
    assert (f3 if mirror else f1) > 0
    if mode == "replay":
        g = replay(spec, q, info["dts"][info["acc"] == 1])
    else:
        s = solver(spec, q)
        st = s.advance(1.0, graph=(mode == "device"))
        assert st["t"] == 1.0
        assert st["accepted"] == info["accepted"] and st["rejected"] == info["rejected"]
        g = s.get_state()
        s.close()
    e = fp64_err(g, qo, spec)
    say("max rel err", e)
    assert e <= 1e-12


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("mirror", [False, True])
def test_sw_entropy_fix_transonic_2d_uniform(axis, mirror):
    """The 1D transonic problem on a 2D grid, uniform across `axis`'s other
    direction (transverse terms cancel), full transverse mode and MC; 100
    replayed steps and the device controller's counts."""
    say("case: 2D transonic dam break along", "xy"[axis], "mirror" if mirror else "")
    n_along, n_across = 250, 24
    hl, hr = (0.05, 4.0) if mirror else (4.0, 0.05)
    nc = (n_along, n_across) if axis == 0 else (n_across, n_along)
    spec = dict(W.radial_dam_break(8)[0], num_cells=nc)
    x, y = W.centers(spec)
    X, Y = np.meshgrid(x, y)
    q = np.zeros((3, nc[1], nc[0]))
    q[0] = np.where((X if axis == 0 else Y) < 0.0, hl, hr)
    qo, info = oracle.advance(spec, q, 0.5)
    assert info["rc"] == 0
    f1, f3 = sw_efix_faces(qo, axis)
    say("faces where the fix fires (first, last family):", f1, f3)
    assert (f3 if mirror else f1) > 0
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    e = fp64_err(g, qo, spec)
    say("replay max rel err", e)
    assert e <= 1e-12
    s = solver(spec, q)
    st = s.advance(0.5)
    assert st["accepted"] == info["accepted"] and st["rejected"] == info["rejected"]
    e = fp64_err(s.get_state(), qo, spec)
    s.close()
    say("device controller max rel err", e)
    assert e <= 1e-12


def test_sw_entropy_fix_transonic_radial():
    """A deep column (h = 4) collapsing into a thin layer (h = 0.05) with the
    radial dam break's settings (Roe + fix, MC, full transverse, CFL 0.9,
    extrapolation) on a ragged 130 x 77 grid: the outgoing flow is
    transonic; the fix fires in both directions."""
    say("case: transonic radial collapse 130x77")
    spec, q = W.radial_dam_break(130, ny=77, h_in=4.0, h_out=0.05)
    qo, info = oracle.advance(spec, q, 0.3)
    assert info["rc"] == 0
    fx, fy = sw_efix_faces(qo, 0), sw_efix_faces(qo, 1)
    say("faces where the fix fires: x", fx, "y", fy)
    assert min(fx) > 0 and min(fy) > 0
    g = replay(spec, q, info["dts"][info["acc"] == 1])
    e = fp64_err(g, qo, spec)
    say("max rel err", e)
    assert e <= 1e-12
    s = solver(spec, q)
    st = s.advance(0.3)
    assert st["accepted"] == info["accepted"] and st["rejected"] == info["rejected"]
    assert fp64_err(s.get_state(), qo, spec) <= 1e-12
    s.close()


def test_fp32_kahan_entropy_fix_transonic_radial_l1():
    say("case: FP32+Kahan transonic radial collapse 130x77 (replayed dt)")
    spec, q = W.radial_dam_break(130, ny=77, h_in=4.0, h_out=0.05)
    qo, info = oracle.advance(spec, q, 0.3)
    g = replay(dict(spec, precision="fp32_kahan"), q, info["dts"][info["acc"] == 1])
    err = l1_rel(g, qo)
    say("L1 relative errors", err)
    assert max(err) <= 1e-5


# --------------------------------------------------------------------------
# Courant number with dx != dy
# --------------------------------------------------------------------------
def _courant_cases():
    sw, qsw = W.random_smooth_sw(8, seed=3, periodic=False)
    yield "sw_classic", sw, None
    yield "sw_split", dict(sw, dimensional_split="strang"), None
    eu, _ = W.shock_bubble(8, 8)
    yield "euler_sharpclaw", eu, None
    yield "euler_roe", dict(eu, scheme="classic", riemann="euler_roe", entropy_fix=1,
                            limiter="mc", transverse=2, cfl_desired=0.8, cfl_max=0.9), None
    el, _, _ = W.layered_elastic(8)
    yield "elastic", el, "elastic"
    ps, _, _ = W.psystem_checkerboard(8, 2, ny_periods=2)
    yield "psystem", ps, "psystem"


def _courant_state(name, spec, nx, ny):
    """A seeded, smooth but non-uniform state of each kind on an nx x ny grid."""
    spec = dict(spec, num_cells=(nx, ny))
    rng = np.random.default_rng(11)
    x, y = W.centers(spec)
    X, Y = np.meshgrid((x - spec["lower"][0]) / (spec["upper"][0] - spec["lower"][0]),
                       (y - spec["lower"][1]) / (spec["upper"][1] - spec["lower"][1]))
    bump = lambda: np.sin(2 * np.pi * (rng.uniform() + X)) * np.cos(2 * np.pi * (rng.uniform() + Y))
    aux = None
    if spec["riemann"] == "sw_roe":
        q = np.array([1.0 + 0.2 * bump(), 0.3 + 0.1 * bump(), -0.6 + 0.1 * bump()])
    elif spec["riemann"] in ("euler_hlle", "euler_roe"):
        rho, u, v, p = 1.0 + 0.2 * bump(), 0.4 + 0.1 * bump(), -0.7 + 0.1 * bump(), 1.0 + 0.2 * bump()
        q = np.array(W.euler_conserved(rho, u, v, p))
    elif spec["riemann"] == "elastic_vc":
        q = 0.1 * np.array([bump() for _ in range(5)])
        aux = np.array([2.0 + bump(), 5.0 + 2 * bump(), 4.0 + 2 * bump()])
    else:
        q = np.array([0.05 * bump(), 0.1 * bump(), 0.1 * bump()])
        aux = np.array([1.5 + 0.5 * bump(), 2.0 + 0.5 * bump()])
    return spec, q, aux


@pytest.mark.parametrize("case", [c[0] for c in _courant_cases()])
@pytest.mark.parametrize("shape", [((200, 70), (2.0, 0.5)), ((70, 130), (0.6, 2.0))])
def test_courant_number_with_unequal_spacing(case, shape):
    """claw_step's Courant number (dt times the largest speed over spacing)
    on cells with dx != dy equals the oracle's, and so does the step."""
    name, base, _ = next(c for c in _courant_cases() if c[0] == case)
    (nx, ny), (Lx, Ly) = shape
    base = dict(base, lower=(0.0, 0.0), upper=(Lx, Ly),
                bc_lower=("extrap", "extrap"), bc_upper=("extrap", "extrap"))
    spec, q, aux = _courant_state(name, base, nx, ny)
    say("case: Courant number", name, nx, "x", ny, "dx", Lx / nx, "dy", Ly / ny)
    dt = 0.2 * min(Lx / nx, Ly / ny)
    qo, speed = oracle.step(spec, q, dt, aux=aux)
    s = solver(spec, q, aux)
    cg = s.step(dt)
    g = s.get_state()
    s.close()
    say("courant gpu", cg, "oracle", dt * speed)
    assert cg == pytest.approx(dt * speed, rel=1e-13)
    assert fp64_err(g, qo, spec) <= 1e-12


# --------------------------------------------------------------------------
# Batches against the oracle
# --------------------------------------------------------------------------
def _batch_trace():
    # uneven grids, several strips and segments each, ragged tails
    return W.serving_trace(n_requests=5, seed=21, nmin=40, nmax=190, t_end=0.12)


def _run_batch(trace, precision):
    from paper_1111_6583_amd import Batch
    b = Batch(8)
    members = []
    for r in trace:
        spec, q = W.request_problem(r, precision=precision)
        s = solver(spec, q)
        b.add(s, r["t_end"])
        members.append(s)
    guard = 0
    while b.advance(16) > 0:
        guard += 1
        assert guard < 1000
    out = []
    for s in members:
        ck = b.member_clock(s)
        b.remove(s)
        out.append((s.get_state(), ck))
        s.close()
    b.close()
    return out


def test_batch_fp64_matches_oracle():
    """Every member of an FP64 batch of uneven grids takes the oracle's
    accepted and rejected steps and matches its state to 1e-12."""
    say("case: FP64 batch of 5 uneven grids vs the oracle's controller")
    trace = _batch_trace()
    res = _run_batch(trace, "fp64")
    for r, (g, ck) in zip(trace, res):
        spec, q = W.request_problem(r, precision="fp64")
        qo, info = oracle.advance(spec, q, r["t_end"])
        assert info["rc"] == 0
        e = fp64_err(g, qo, spec)
        say("member", r["n"], "accepted", ck["accepted"], "oracle", info["accepted"], "err", e)
        assert ck["t"] == r["t_end"]
        assert ck["accepted"] == info["accepted"] and ck["rejected"] == info["rejected"]
        assert e <= 1e-12


def test_batch_fp32_kahan_matches_oracle():
    """Members of an FP32+Kahan batch against the FP64 oracle run to the same
    end time: relative L1 error per component <= 1e-5 (the shallow-water bar)."""
    say("case: FP32+Kahan batch of 5 uneven grids vs the oracle")
    trace = _batch_trace()
    res = _run_batch(trace, "fp32_kahan")
    for r, (g, ck) in zip(trace, res):
        spec, q = W.request_problem(r, precision="fp64")
        qo, info = oracle.advance(spec, q, r["t_end"])
        err = l1_rel(g, qo)
        say("member", r["n"], "L1", err)
        assert ck["t"] == r["t_end"]
        assert max(err) <= 1e-5


def test_served_requests_match_oracle():
    """Requests served by the continuous-batching loop (FP32+Kahan, Poisson
    arrivals, overlapping on the device) against the FP64 oracle."""
    from paper_1111_6583_amd import serve
    say("case: 6 served requests vs the oracle")
    trace = W.serving_trace(n_requests=6, rate=200.0, seed=8, nmin=40, nmax=150, t_end=0.15)
    r = serve.run_trace(trace, keep_results=True, max_grids=4)
    for req in trace:
        out, ck = r["results"][req["id"]]
        spec, q = W.request_problem(req, precision="fp64")
        qo, info = oracle.advance(spec, q, req["t_end"])
        err = l1_rel(out, qo)
        say("request", req["id"], req["n"], "L1", err)
        assert ck["t"] == req["t_end"]
        assert max(err) <= 1e-5


# --------------------------------------------------------------------------
# Compensated against plain FP32 updates
# --------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["sw", "euler"])
def test_kahan_compensation_gain(case):
    """The same replayed run in FP32 with and without the compensated
    update, against the FP64 oracle: the compensation removes the drift of
    plain FP32 sums of small increments (shallow water L1 bar 1e-5 with it;
    Euler 1e-4)."""
    if case == "sw":
        spec, q = W.radial_dam_break(256)
        qo, info = oracle.advance(spec, q, 0.25)
        bar = 1e-5
    else:
        spec, q = W.shock_bubble(256, 128)
        qo, info = oracle.advance(spec, q, 1.0, max_steps=60)
        bar = 1e-4
    dts = info["dts"][info["acc"] == 1]
    gk = replay(dict(spec, precision="fp32_kahan"), q, dts)
    gp = replay(dict(spec, precision="fp32"), q, dts)
    ek, ep = l1_rel(gk, qo), l1_rel(gp, qo)
    say(case, "L1 FP32+Kahan", ek, "plain FP32", ep, "gain", [p_ / max(k, 1e-300) for k, p_ in zip(ek, ep)])
    assert max(ek) <= bar
    assert sum(ek) < sum(ep)
