"""Continuous-batching server for shallow-water solves (the serving workload).

Requests arrive on a seeded Poisson trace; each is an N x N shallow-water
hump (classic wave propagation, FP32+Kahan) run to its own t_end.  The loop:

  * admits arrived requests in FIFO order while a batch slot is free and the
    sum of the resident workspaces stays within the HBM budget (the exact
    bytes claw_workspace_bytes reports; the state stays resident on the
    device from admission to completion);
  * advances every resident grid by `attempts` device-controlled attempts
    with one batched launch per attempt (replayed from a HIP graph), each grid
    on its own clock and dt controller;
  * retires grids whose controller stopped, copies their result to the host
    and records latency = completion time - arrival time.

New requests join between launch groups while others are mid-solve, so
their work overlaps on the device.  Tiling per grid size comes from the
autotuner over a few size buckets; results do not depend on it.
"""

from __future__ import annotations

import collections
import math
import time

import numpy as np
import torch

import ctypes as C

from ._claw import load_library, make_config
from .solver import Batch, Solver
from . import workloads as W


def workspace_bytes(spec) -> int:
    """Device bytes a request occupies while resident (its libclaw workspace)."""
    return int(load_library().claw_workspace_bytes(C.byref(make_config(spec))))


def hump_state_device(req, device="cuda:0"):
    """Initial state of a request, formed on the device in float64
    (h = 1 + A exp(-|x-x0|^2/w^2), hu = hv = 0 on [0,1]^2)."""
    n = req["n"]
    x = (torch.arange(n, device=device, dtype=torch.float64) + 0.5) / n
    dx2 = (x - req["x0"][0]) ** 2
    dy2 = (x - req["x0"][1]) ** 2
    q = torch.zeros((3, n, n), device=device, dtype=torch.float64)
    q[0] = 1.0 + req["amplitude"] * torch.exp(-(dy2[:, None] + dx2[None, :]) / req["width"] ** 2)
    return q


class Tuner:
    """seg_rows per grid-size bucket, measured once by the library's autotuner."""

    def __init__(self, buckets=(64, 128, 256, 512, 1024), precision="fp32_kahan"):
        self.table = {}
        for n in buckets:
            s = Solver(W.sw_hump_spec(n, precision=precision))
            s.set_state(hump_state_device(dict(n=n, amplitude=0.5, width=0.1, x0=(0.5, 0.5))))
            self.table[n] = s.autotune(reps=3)
            s.close()
        self.buckets = sorted(self.table)

    def seg_rows(self, n):
        b = min(self.buckets, key=lambda k: abs(math.log(k / n)))
        return self.table[b]


def run_trace(trace, budget_bytes=8 << 30, max_grids=64, attempts=16, precision="fp32_kahan",
              tuner=None, keep_results=False, device="cuda:0"):
    """Serve `trace` (list of request dicts, sorted by arrival) in real time.

    Returns dict(latencies, p50, p99, throughput, cell_updates, wall, results).
    """
    pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
    waiting = collections.deque()
    batch = Batch(max_grids, device=device)
    resident = {}          # solver -> (request, bytes)
    used = 0
    lat = {}
    results = {}
    cell_updates = 0
    max_resident = 0
    t0 = time.perf_counter()
    while pending or waiting or resident:
        now = time.perf_counter() - t0
        while pending and pending[0]["arrival"] <= now:
            waiting.append(pending.popleft())
        # admission: FIFO while a slot and budget allow
        while waiting and len(resident) < max_grids:
            req = waiting[0]
            spec = W.sw_hump_spec(req["n"], precision=precision)
            nb = workspace_bytes(spec)
            if used + nb > budget_bytes:
                if not resident:
                    raise RuntimeError(f"request {req['id']} needs {nb} bytes > budget {budget_bytes}")
                break
            waiting.popleft()
            s = Solver(spec, device=device)
            s.set_state(hump_state_device(req, device))
            if tuner is not None:
                s.set_tuning(tuner.seg_rows(req["n"]))
            batch.add(s, req["t_end"])
            resident[s] = (req, nb)
            used += nb
            max_resident = max(max_resident, len(resident))
        if not resident:
            if pending:
                time.sleep(max(0.0, pending[0]["arrival"] - (time.perf_counter() - t0)))
            continue
        batch.advance(attempts)
        for s in batch.finished():
            req, nb = resident.pop(s)
            batch.remove(s)
            ck = s.clock()
            out = s.get_state()
            done = time.perf_counter() - t0
            lat[req["id"]] = done - req["arrival"]
            cell_updates += req["n"] * req["n"] * ck["accepted"]
            if keep_results:
                results[req["id"]] = (out, ck)
            s.close()
            used -= nb
    wall = time.perf_counter() - t0
    batch.close()
    lv = np.array([lat[r["id"]] for r in trace])
    return dict(latencies=lv, p50=float(np.percentile(lv, 50)), p99=float(np.percentile(lv, 99)),
                throughput_req_s=len(trace) / wall, cell_updates=cell_updates,
                cell_updates_per_s=cell_updates / wall, wall=wall, results=results,
                max_resident=max_resident)


def solve_alone(req, precision="fp32_kahan", seg_rows=None, device="cuda:0"):
    """The same request on its own handle (no batch), for comparison."""
    spec = W.sw_hump_spec(req["n"], precision=precision)
    s = Solver(spec, device=device)
    s.set_state(hump_state_device(req, device))
    if seg_rows:
        s.set_tuning(seg_rows)
    s.advance(req["t_end"])
    out, ck = s.get_state(), s.clock()
    s.close()
    return out, ck
