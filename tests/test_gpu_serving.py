"""Serving: continuous batching with HBM-budget admission (GPU)."""

import sys

import numpy as np
import pytest

from paper_1111_6583_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_served_results_equal_solo_results():
    """Each request's result is the same alone and in the mix (bitwise for
    FP32+Kahan: per-grid arithmetic does not depend on batch membership)."""
    from paper_1111_6583_amd import serve
    say("case: 10 requests N in [48,160], Poisson 200/s, t_end=0.2")
    trace = W.serving_trace(n_requests=10, rate=200.0, seed=3, nmin=48, nmax=160, t_end=0.2)
    r = serve.run_trace(trace, keep_results=True, max_grids=6)
    assert len(r["latencies"]) == 10 and np.all(r["latencies"] > 0)
    for req in trace:
        out, ck = r["results"][req["id"]]
        solo, cks = serve.solve_alone(req)
        assert ck["accepted"] == cks["accepted"] and ck["t"] == cks["t"] == req["t_end"]
        np.testing.assert_array_equal(out, solo)


def test_budget_admission_serialises_when_tight():
    """A budget that fits one grid at a time still serves every request."""
    from paper_1111_6583_amd import serve
    say("case: tight HBM budget")
    trace = W.serving_trace(n_requests=5, rate=1000.0, seed=4, nmin=64, nmax=64, t_end=0.05)
    spec, _ = W.sw_hump(64, precision="fp32_kahan")
    import ctypes as C
    from paper_1111_6583_amd._claw import load_library, make_config
    nb = load_library().claw_workspace_bytes(C.byref(make_config(spec)))
    r = serve.run_trace(trace, budget_bytes=int(nb * 1.5), keep_results=True)
    assert sorted(r["results"]) == [q["id"] for q in trace]
    assert r["max_resident"] == 1
