"""Continuous-batching server for shallow-water solves (the serving workload).

Requests arrive on a seeded Poisson trace; each is an N x N shallow-water
hump (classic wave propagation, FP32+Kahan) run to its own t_end.  The loop:

  * admits arrived requests in FIFO order while a batch slot is free and the
    sum of the resident workspaces stays within the HBM budget (the exact
    bytes claw_workspace_bytes reports; the state stays resident on the
    device from admission to completion);
  * keeps groups of `attempts` device-controlled attempts in flight (one
    batched launch per attempt over every resident grid, each grid on its
    own clock and dt controller): the next group is enqueued before the
    host waits for the previous one, so the GPU keeps working while the host
    admits and retires;
  * after each group, retires the grids whose controller stopped, copies
    their result to the host and records latency = completion - arrival.

New requests join the next group while others are mid-solve, so their work
overlaps on the device.  Every handle and the batch enqueue on non-blocking
streams (no implicit ordering with the legacy default stream).  A request's
first step size is the controller's a-priori one, cfl_desired * dx / max
cell speed, from the hump's largest cell depth (the cell centre nearest its
peak in each direction), so admission reads nothing back from the device.
Tiling per grid size comes from a batch-throughput tuner over a few size
buckets (Tuner); results do not depend on it.
"""

from __future__ import annotations

import collections
import ctypes as C
import math
import time

import numpy as np
import torch

from ._claw import load_library, make_config
from .solver import Batch, Solver
from . import workloads as W

G = 1.0   # gravity of the serving workload


def workspace_bytes(spec) -> int:
    """Device bytes a request occupies while resident (its libclaw workspace)."""
    return int(load_library().claw_workspace_bytes(C.byref(make_config(spec))))


def first_dt(req, cfl_desired=0.9) -> float:
    """The controller's a-priori first step: cfl_desired * dx over the largest
    cell speed sqrt(g h) of the hump at rest (its deepest cell is the centre
    nearest the peak in x and in y, the Gaussian being a product of the two)."""
    n = req["n"]
    dx = 1.0 / n
    d2 = 0.0
    for c in req["x0"]:
        k = min(max(int(math.floor(c * n - 0.5 + 0.5)), 0), n - 1)   # nearest centre (k + 0.5) dx
        best = min(abs((j + 0.5) * dx - c) for j in (max(k - 1, 0), k, min(k + 1, n - 1)))
        d2 += best * best
    hmax = 1.0 + req["amplitude"] * math.exp(-d2 / req["width"] ** 2)
    return cfl_desired * dx / math.sqrt(G * hmax)


def request_spec(req, precision="fp32_kahan"):
    return W.sw_hump_spec(req["n"], precision=precision, dt_initial=first_dt(req))


def hump_state_device(req, device="cuda:0"):
    """Initial state of a request, formed on the device in float64 on the
    current torch stream (h = 1 + A exp(-|x-x0|^2/w^2), hu = hv = 0 on [0,1]^2)."""
    n = req["n"]
    x = (torch.arange(n, device=device, dtype=torch.float64) + 0.5) / n
    dx2 = (x - req["x0"][0]) ** 2
    dy2 = (x - req["x0"][1]) ** 2
    q = torch.zeros((3, n, n), device=device, dtype=torch.float64)
    q[0] = 1.0 + req["amplitude"] * torch.exp(-(dy2[:, None] + dx2[None, :]) / req["width"] ** 2)
    return q


class Tuner:
    """Tiling per grid-size bucket for grids that run in a full batch.

    A lone small grid runs fastest in short row segments (more waves for a
    GPU it cannot fill), but in a batch the GPU is full and each segment's
    pipeline prologue (four rows of the classic kernel) is pure extra work.
    So each bucket is timed as a batch: copies of an n x n hump enough to
    fill the GPU, every member at the same candidate rows per segment, a
    group of attempts per candidate; the fastest per cell-update wins.
    Results do not depend on the tiling (bit for bit)."""

    CANDIDATES = (4, 8, 12, 16, 24, 32, 48, 64)

    def __init__(self, buckets=(64, 128, 256, 512, 1024), precision="fp32_kahan",
                 cells_per_batch=12 << 20, max_grids=64, device="cuda:0"):
        self.table, self.rate = {}, {}
        for n in buckets:
            k = max(2, min(max_grids, cells_per_batch // (n * n)))
            req = dict(n=n, amplitude=0.5, width=0.1, x0=(0.5, 0.5), t_end=1e9)
            members = []
            b = Batch(k, device=device)
            for _ in range(k):
                s = Solver(W.sw_hump_spec(n, precision=precision), device=device)
                s.set_state(hump_state_device(req, device))
                members.append(s)
                b.add(s, req["t_end"])
            best, best_rate = None, 0.0
            for c in self.CANDIDATES:
                if c > n:
                    continue
                for s in members:
                    s.set_tuning(c)
                # re-adding picks up the new tiling
                for s in members:
                    b.remove(s)
                    b.add(s, req["t_end"])
                b.advance(16)
                t0 = time.perf_counter()
                b.advance(32)
                dt = time.perf_counter() - t0
                rate = k * n * n * 32 / dt
                if rate > best_rate:
                    best, best_rate = c, rate
            for s in members:
                b.remove(s)
                s.close()
            b.close()
            self.table[n], self.rate[n] = best, best_rate
        self.buckets = sorted(self.table)

    def seg_rows(self, n):
        b = min(self.buckets, key=lambda k: abs(math.log(k / n)))
        return self.table[b]

    def describe(self):
        return {str(n): dict(seg_rows=self.table[n], batch_cell_updates_per_s=round(self.rate[n]))
                for n in self.buckets}


class _PinnedPool:
    """Reusable pinned host buffers for results leaving the device (sizes
    rounded up to a power of two, at least 1 MiB): a fresh pinned allocation
    of every request's size would cost the host more than the copy.  One
    pool per device lives as long as the process, so a warm-up trace leaves
    it filled for the next."""

    def __init__(self):
        self.free = collections.defaultdict(list)

    def take(self, shape, dtype=torch.float64):
        n = int(np.prod(shape)) * torch.tensor([], dtype=dtype).element_size()
        key = max(1 << 20, 1 << (n - 1).bit_length())
        buf = self.free[key].pop() if self.free[key] else torch.empty(key, dtype=torch.uint8,
                                                                        pin_memory=True)
        return buf, buf[:n].view(dtype).view(shape)

    def give(self, buf):
        self.free[buf.numel()].append(buf)


_pools = {}


def _pinned_pool(device):
    key = str(device)
    if key not in _pools:
        _pools[key] = _PinnedPool()
    return _pools[key]


class _Streams:
    """A small pool of non-blocking torch streams for request handles."""

    def __init__(self, n=4, device="cuda:0"):
        self.s = [torch.cuda.Stream(device=device) for _ in range(n)]
        self.k = 0

    def next(self):
        self.k = (self.k + 1) % len(self.s)
        return self.s[self.k]


def _admit(req, precision, tuner, device, stream):
    spec = request_spec(req, precision)
    with torch.cuda.stream(stream):
        s = Solver(spec, device=device, stream=stream)
        q = hump_state_device(req, device)
        s.set_state(q)
    if tuner is not None:
        s.set_tuning(tuner.seg_rows(req["n"]))
    return s


def collect(copying, lat, results, keep, t0, block, pool):
    """Complete the retirements whose result has reached host memory (all of
    them if block): latency ends when that is seen (checked once per group,
    so a result may be counted up to one group late).  Removes them from
    `copying`, returns their pinned buffers to the pool and their
    cell-updates."""
    cu = 0
    still = []
    for item in copying:
        req, ck, dev, buf, host, ev = item
        if block:
            ev.synchronize()
        elif not ev.query():
            still.append(item)
            continue
        lat[req["id"]] = time.perf_counter() - t0 - req["arrival"]
        cu += req["n"] * req["n"] * ck["accepted"]
        if keep:
            results[req["id"]] = (host.numpy().copy(), ck)
        pool.give(buf)
    copying[:] = still
    return cu


def run_trace(trace, budget_bytes=8 << 30, max_grids=64, attempts=16, precision="fp32_kahan",
              tuner=None, keep_results=False, device="cuda:0"):
    """Serve `trace` (list of request dicts, sorted by arrival) in real time.

    Returns dict(latencies, p50, p99, throughput_req_s, cell_updates,
    cell_updates_per_s, wall, results, max_resident, stats)."""
    pending = collections.deque(sorted(trace, key=lambda r: r["arrival"]))
    waiting = collections.deque()
    streams = _Streams(device=device)
    batch = Batch(max_grids, device=device, stream=torch.cuda.Stream(device=device))
    resident = {}          # solver -> (request, bytes)
    used = 0
    lat = {}
    results = {}
    cell_updates = 0
    max_resident = 0
    in_flight = 0
    graveyard = []         # handles retired at the last wait: kept until one more group completes
    copying = []           # (request, clock, device result, pinned buffer, host view, copy-done event)
    pool = _pinned_pool(device)
    groups = 0
    # host time by activity, and the GPU's busy time (events around each group)
    t_admit = t_retire = t_wait = 0.0
    evs = collections.deque()
    gpu_busy = 0.0
    t0 = time.perf_counter()
    while pending or waiting or resident or in_flight or copying:
        now = time.perf_counter() - t0
        while pending and pending[0]["arrival"] <= now:
            waiting.append(pending.popleft())
        # admission: FIFO while a slot and budget allow (joins the next group)
        while waiting and len(resident) < max_grids:
            req = waiting[0]
            nb = workspace_bytes(W.sw_hump_spec(req["n"], precision=precision))
            if used + nb > budget_bytes:
                if not resident:
                    raise RuntimeError(f"request {req['id']} needs {nb} bytes > budget {budget_bytes}")
                break
            waiting.popleft()
            ta = time.perf_counter()
            s = _admit(req, precision, tuner, device, streams.next())
            batch.add(s, req["t_end"])
            t_admit += time.perf_counter() - ta
            resident[s] = (req, nb)
            used += nb
            max_resident = max(max_resident, len(resident))
        if resident and in_flight < 2:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(batch.stream)
            batch.launch(attempts)
            e1.record(batch.stream)
            evs.append((e0, e1))
            in_flight += 1
            groups += 1
            if in_flight < 2:
                continue          # queue a second group before waiting
        if not in_flight:
            cell_updates += collect(copying, lat, results, keep_results, t0,
                                    block=not (pending or waiting), pool=pool)
            if pending:
                time.sleep(max(0.0, pending[0]["arrival"] - (time.perf_counter() - t0)))
            continue
        tw = time.perf_counter()
        batch.wait()
        t_wait += time.perf_counter() - tw
        in_flight -= 1
        e0, e1 = evs.popleft()
        e1.synchronize()      # recorded right after the group's own completion event
        gpu_busy += e0.elapsed_time(e1) * 1e-3
        tr = time.perf_counter()
        # handles retired at the previous wait: no group in flight refers to them now
        for s in graveyard:
            s.close()
        graveyard = []
        for s in batch.finished():
            req, nb = resident.pop(s)
            batch.remove(s)
            ck = s.clock()
            # the result leaves the device asynchronously: float64 on the
            # device, then into pinned host memory on the request's stream
            dev = s.get_state(device=True)
            buf, host = pool.take(dev.shape)
            with torch.cuda.stream(s.stream):
                host.copy_(dev, non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(s.stream)
            copying.append((req, ck, dev, buf, host, ev))
            graveyard.append(s)
            used -= nb
        cell_updates += collect(copying, lat, results, keep_results, t0, block=False, pool=pool)
        t_retire += time.perf_counter() - tr
    wall = time.perf_counter() - t0
    for s in graveyard:
        s.close()
    batch.close()
    lv = np.array([lat[r["id"]] for r in trace])
    return dict(latencies=lv, p50=float(np.percentile(lv, 50)), p99=float(np.percentile(lv, 99)),
                throughput_req_s=len(trace) / wall, cell_updates=cell_updates,
                cell_updates_per_s=cell_updates / wall, wall=wall, results=results,
                max_resident=max_resident,
                stats=dict(groups=groups, attempts_per_group=attempts, gpu_busy_s=round(gpu_busy, 3),
                           host_admit_s=round(t_admit, 3), host_retire_s=round(t_retire, 3),
                           host_wait_s=round(t_wait, 3)))


def solve_alone(req, precision="fp32_kahan", seg_rows=None, device="cuda:0"):
    """The same request on its own handle (no batch), for comparison."""
    spec = request_spec(req, precision)
    s = Solver(spec, device=device)
    s.set_state(hump_state_device(req, device))
    if seg_rows:
        s.set_tuning(seg_rows)
    s.advance(req["t_end"])
    out, ck = s.get_state(), s.clock()
    s.close()
    return out, ck
