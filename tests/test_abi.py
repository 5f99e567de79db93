"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/claw.h declares, and its host-only entry points validate configs."""

import ctypes as C
import os

import pytest

from paper_1111_6583_amd import _claw
from paper_1111_6583_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_declares_the_api():
    names = _claw.header_functions()
    for n in ("claw_create", "claw_step", "claw_advance", "claw_advance_graph", "claw_set_state",
              "claw_get_state", "claw_totals", "claw_destroy", "claw_workspace_bytes",
              "claw_batch_create", "claw_batch_advance", "claw_autotune"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = _claw.load_library()
    missing = [n for n in _claw.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_strerror_names_every_status():
    lib = _claw.load_library()
    for rc in [0] + list(_claw.ERRORS):
        assert lib.claw_strerror(rc).decode() != "unknown status"


def _bytes(spec):
    lib = _claw.load_library()
    c = _claw.make_config(spec)
    return lib.claw_workspace_bytes(C.byref(c)), lib.claw_num_eqn(C.byref(c))


def test_workspace_sizes():
    spec, q = W.radial_dam_break(1024)
    n, m = _bytes(spec)
    assert m == 3
    # two FP64 state buffers plus small control blocks
    assert 2 * 3 * 1024 * 1024 * 8 <= n < 2 * 3 * 1024 * 1024 * 8 + 64 * 1024
    spec32 = dict(spec, precision="fp32_kahan")
    n32, _ = _bytes(spec32)
    # q and compensation, ping-pong, float32: same bytes as FP64
    assert abs(n32 - n) < 64 * 1024
    s3, _ = W.shock_bubble(256, 128)
    n3, m3 = _bytes(s3)
    assert m3 == 4 and n3 >= 3 * 4 * 256 * 128 * 8
    s4, _, _ = W.layered_elastic(64)
    n4, m4 = _bytes(s4)
    assert m4 == 5 and n4 >= (2 * 5 + 3) * 64 * 64 * 8


@pytest.mark.parametrize("bad", [
    dict(ndim=3),
    dict(num_cells=(3, 64)),
    dict(riemann="euler_hlle"),                     # HLLE only in SharpClaw
    dict(bc_lower=("periodic", "extrap")),          # periodic must pair
    dict(limiter="superbee"),
    dict(transverse=3),
    dict(cfl_max=0.0),
    dict(upper=(-2.5, 2.5)),
])
def test_invalid_configs_rejected(bad):
    spec, _ = W.radial_dam_break(64)
    spec = dict(spec)
    try:
        spec.update(bad)
        n, _ = _bytes(spec)
    except (KeyError, ValueError):
        return   # rejected already by the spec converter
    assert n == 0


def test_elastic_only_classic_2d():
    spec, _, _ = W.layered_elastic(64)
    assert _bytes(dict(spec, scheme="sharpclaw"))[0] == 0


def test_sharpclaw_integrator_and_weno_order_options():
    spec, _ = W.shock_bubble(256, 128)
    n33, m = _bytes(spec)
    n104, _ = _bytes(dict(spec, time_integrator="ssp104"))
    arr = m * 256 * 128 * 8
    # SSPRK(10,4) keeps one more state-sized register than SSPRK(3,3)
    assert arr <= n104 - n33 < arr + 4096
    for order in (7, 9, 11, 13, 15, 17):
        assert _bytes(dict(spec, weno_order=order))[0] == n33
    for bad in (-5, 1, 3, 4, 6, 8, 16, 19, 21):
        assert _bytes(dict(spec, weno_order=bad))[0] == 0
    # the (order + 1) / 2 ghost layers must map to interior cells
    small, _ = W.random_smooth_euler(9, seed=1)
    assert _bytes(dict(small, weno_order=17))[0] > 0
    assert _bytes(dict(small, weno_order=17, num_cells=(8, 9)))[0] == 0
    assert _bytes(dict(small, weno_order=17, num_cells=(9, 8)))[0] == 0
    assert _bytes(dict(small, weno_order=15, num_cells=(8, 8)))[0] > 0
    # classic ignores both
    sw, _ = W.radial_dam_break(64)
    assert _bytes(dict(sw, time_integrator="ssp104", weno_order=7))[0] == _bytes(sw)[0]


def test_euler_roe_tracer_and_source_options():
    spec, q = W.shock_bubble_axisym(160, 40)
    n, m = _bytes(spec)
    assert m == 5 and n >= 2 * 5 * 160 * 40 * 8
    assert _bytes(dict(spec, tracer=0))[1] == 4
    # a tracer only exists for the Euler Roe solver; the source only in 2D classic Euler Roe
    sw, _ = W.radial_dam_break(64)
    assert _bytes(dict(sw, tracer=1))[0] == 0
    assert _bytes(dict(sw, source="axisymmetric"))[0] == 0
    assert _bytes(dict(spec, scheme="sharpclaw"))[0] == 0
    assert _bytes(dict(spec, lower=(0.0, -0.5)))[0] == 0   # the radius must be >= 0


def test_dimensional_split_options():
    sw, _ = W.radial_dam_break(256, ny=128)
    n0, m = _bytes(sw)
    arr = m * 256 * 128 * 8
    ng, _ = _bytes(dict(sw, dimensional_split="godunov"))
    ns, _ = _bytes(dict(sw, dimensional_split="strang"))
    # Godunov keeps one intermediate state, Strang two
    assert arr <= ng - n0 < arr + 4096
    assert 2 * arr <= ns - n0 < 2 * arr + 8192
    # FP32: each intermediate carries its compensation (same bytes as FP64)
    n32 = _bytes(dict(sw, precision="fp32_kahan"))[0]
    ns32 = _bytes(dict(sw, precision="fp32_kahan", dimensional_split="strang"))[0]
    assert abs((ns32 - n32) - (ns - n0)) < 8192
    # 2D classic only
    d1, _ = W.dam_break_1d(100)
    assert _bytes(dict(d1, dimensional_split="godunov"))[0] == 0
    eu, _ = W.shock_bubble(64, 32)
    assert _bytes(dict(eu, dimensional_split="strang"))[0] == 0
    lib = _claw.load_library()
    c = _claw.make_config(sw)
    c.dimensional_split = 3
    assert lib.claw_workspace_bytes(C.byref(c)) == 0
    # every classic 2D solver splits, with or without the axisymmetric source
    for spec in (W.layered_elastic(64)[0], W.shock_bubble_axisym(64, 16)[0]):
        assert _bytes(dict(spec, dimensional_split="strang"))[0] > _bytes(spec)[0]


def test_psystem_options():
    spec, q, aux = W.psystem_checkerboard(8, 4)
    n, m = _bytes(spec)
    assert m == 3 and q.shape == (3, 32, 32) and aux.shape == (2, 32, 32)
    lib = _claw.load_library()
    c = _claw.make_config(spec)
    assert lib.claw_num_aux(C.byref(c)) == 2
    # Q, S1, S2, S3 (SSPRK(10,4)) and 2 aux fields
    assert n >= (4 * 3 + 2) * 32 * 32 * 8
    s1, _ = W.psystem_layered_1d(64)
    assert _bytes(s1)[1] == 2
    # SharpClaw only
    assert _bytes(dict(spec, scheme="classic"))[0] == 0


def test_size_limit():
    """Grids above 2e9 cells are refused; the largest accepted ones report
    their exact workspace size."""
    spec, _ = W.radial_dam_break(64)
    assert _bytes(dict(spec, num_cells=(50000, 50000)))[0] == 0
    n, m = _bytes(dict(spec, num_cells=(44000, 44000)))
    assert n >= 2 * 3 * 44000 * 44000 * 8


def test_static_step_size_limit_is_checked_on_the_host():
    """claw_step_static rejects a grid whose intermediates exceed its fixed
    array (CLAW_E_TOOBIG) before touching a device, and reports the bytes it
    would use: nothing beyond control blocks for an FP64 classic step (state
    in the caller's buffers), stage buffers for SharpClaw."""
    lib = _claw.load_library()
    spec, _ = W.radial_dam_break(1024)
    c = _claw.make_config(spec)
    assert lib.claw_static_bytes(C.byref(c)) < 64 * 1024
    c32 = _claw.make_config(dict(spec, precision="fp32_kahan"))
    n32 = lib.claw_static_bytes(C.byref(c32))
    assert 4 * 3 * 1024 * 1024 * 4 <= n32 < 4 * 3 * 1024 * 1024 * 4 + 64 * 1024
    big, _ = W.shock_bubble(2048, 1024)
    cb = _claw.make_config(dict(big, precision="fp32_kahan"))
    assert lib.claw_static_bytes(C.byref(cb)) > _claw.STATIC_SCRATCH_BYTES
    # disjoint (never dereferenced) addresses: every check below fails before a launch
    a, b, z = C.c_void_p(1 << 40), C.c_void_p(1 << 41), C.c_void_p(1 << 42)
    rc = lib.claw_step_static(C.byref(cb), a, None, b, 1e-3, z, None)
    assert rc == -9
    assert "CLAW_STATIC_SCRATCH_BYTES" in lib.claw_strerror(rc).decode()
    # argument checks, also host-side
    assert lib.claw_step_static(C.byref(c), None, None, b, 1e-3, z, None) == -1   # no input
    assert lib.claw_step_static(C.byref(c), a, None, a, 1e-3, z, None) == -1      # in = out
    assert lib.claw_step_static(C.byref(c), a, None, b, 0.0, z, None) == -1       # dt <= 0
    el, _, _ = W.layered_elastic(64)
    assert lib.claw_step_static(C.byref(_claw.make_config(el)), a, None, b, 1e-3, z, None) == -1


def test_plain_fp32_precision_only_where_built():
    """CLAW_FP32 (no compensation) exists for classic 2D shallow water and
    SharpClaw 2D Euler with WENO5; other configurations are refused, and its
    workspace holds no compensation arrays."""
    lib = _claw.load_library()
    sw, _ = W.radial_dam_break(256)
    nk = lib.claw_workspace_bytes(C.byref(_claw.make_config(dict(sw, precision="fp32_kahan"))))
    npl = lib.claw_workspace_bytes(C.byref(_claw.make_config(dict(sw, precision="fp32"))))
    assert npl > 0 and npl < nk - 2 * 3 * 256 * 256 * 4 + 64 * 1024
    eu, _ = W.shock_bubble(128, 64)
    assert lib.claw_workspace_bytes(C.byref(_claw.make_config(dict(eu, precision="fp32")))) > 0
    for bad in (dict(eu, precision="fp32", weno_order=7), dict(sw, precision="fp32", dimensional_split="godunov")):
        assert lib.claw_workspace_bytes(C.byref(_claw.make_config(bad))) == 0
    el, _, _ = W.layered_elastic(64)
    assert lib.claw_workspace_bytes(C.byref(_claw.make_config(dict(el, precision="fp32")))) == 0
