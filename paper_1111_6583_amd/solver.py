"""Python front end of libclaw: torch provides device memory and nothing else.

    from paper_1111_6583_amd import Solver
    s = Solver(spec)                 # spec: dict, see workloads.py
    s.set_state(q)                   # numpy/torch float64 (m, ny, nx)
    stats = s.advance(t_end)         # device-resident controller (HIP graphs)
    q = s.get_state()

Every step of the method runs in the HIP kernels of libclaw.so; this module
only allocates the workspace (a torch uint8 tensor), converts arguments and
checks status codes.
"""

from __future__ import annotations

import contextlib
import ctypes as C

import numpy as np
import torch

from ._claw import (ClawStats, ClawTuning, check, load_library, make_config)

_ALIGN = 256


def _aligned_workspace(nbytes: int, device):
    t = torch.empty(nbytes + _ALIGN, dtype=torch.uint8, device=device)
    base = t.data_ptr()
    off = (-base) % _ALIGN
    return t, base + off


class Solver:
    """One grid: a libclaw handle over a torch-allocated workspace."""

    def __init__(self, spec: dict, device="cuda:0", stream=None):
        """stream: a torch.cuda.Stream the handle enqueues on (None: the
        library creates a private stream)."""
        self.lib = load_library()
        self.spec = dict(spec)
        self.cfg = make_config(spec)
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Solver needs a GPU device (cuda:N on ROCm)")
        torch.cuda.set_device(self.device)
        self.nbytes = int(self.lib.claw_workspace_bytes(C.byref(self.cfg)))
        if self.nbytes == 0:
            raise ValueError("invalid or unsupported configuration")
        self.m = int(self.lib.claw_num_eqn(C.byref(self.cfg)))
        self.na = int(self.lib.claw_num_aux(C.byref(self.cfg)))
        nd = self.cfg.ndim
        self.shape = (self.m, self.cfg.num_cells[1] if nd == 2 else 1, self.cfg.num_cells[0])
        self._ws, ptr = _aligned_workspace(self.nbytes, self.device)
        self.stream = stream
        h = C.c_void_p()
        check(self.lib.claw_create(C.byref(self.cfg), C.c_void_p(ptr), self.nbytes,
                                   None if stream is None else C.c_void_p(stream.cuda_stream),
                                   C.byref(h)), "claw_create")
        self.h = h

    # -- state -------------------------------------------------------------
    def _put(self, fn, arr, shape, where):
        if isinstance(arr, torch.Tensor) and arr.is_cuda:
            t = arr.to(torch.float64).contiguous().reshape(shape)
            check(fn(self.h, C.c_void_p(t.data_ptr()), 1), where)
        else:
            a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64).reshape(shape))
            check(fn(self.h, a.ctypes.data_as(C.c_void_p), 0), where)

    def set_state(self, q):
        self._put(self.lib.claw_set_state, q, self.shape, "claw_set_state")

    def set_aux(self, aux):
        self._put(self.lib.claw_set_aux, aux, (self.na,) + self.shape[1:], "claw_set_aux")

    def get_state(self, device=False):
        if device:
            # allocated on the handle's stream, which writes it
            with torch.cuda.stream(self.stream) if self.stream is not None else contextlib.nullcontext():
                out = torch.empty(self.shape, dtype=torch.float64, device=self.device)
            check(self.lib.claw_get_state(self.h, C.c_void_p(out.data_ptr()), 1), "claw_get_state")
            return out
        out = np.empty(self.shape, dtype=np.float64)
        check(self.lib.claw_get_state(self.h, out.ctypes.data_as(C.c_void_p), 0), "claw_get_state")
        return out

    # -- stepping ----------------------------------------------------------
    def step(self, dt: float) -> float:
        cour = C.c_double(0.0)
        check(self.lib.claw_step(self.h, float(dt), C.byref(cour)), "claw_step")
        return cour.value

    def advance(self, t_end: float, max_steps: int = 0, graph: bool = True,
                steps_per_graph: int = 16) -> dict:
        st = ClawStats()
        if graph:
            rc = self.lib.claw_advance_graph(self.h, float(t_end), int(steps_per_graph),
                                             int(max_steps), C.byref(st))
        else:
            rc = self.lib.claw_advance(self.h, float(t_end), int(max_steps), C.byref(st))
        out = st.as_dict()
        out["reached"] = rc != -8
        if rc == -8 and max_steps > 0:
            return out          # stopped after max_steps attempts, as asked
        check(rc, "claw_advance")
        return out

    def totals(self):
        out = np.zeros(self.m)
        check(self.lib.claw_totals(self.h, out.ctypes.data_as(C.POINTER(C.c_double))), "claw_totals")
        return out

    def clock(self) -> dict:
        st = ClawStats()
        check(self.lib.claw_get_clock(self.h, C.byref(st)), "claw_get_clock")
        return st.as_dict()

    def set_clock(self, d: dict):
        st = ClawStats(int(d["accepted"]), int(d["rejected"]), float(d["t"]), float(d["dt_next"]),
                       float(d["max_courant"]), float(d.get("gpu_ms", 0.0)))
        check(self.lib.claw_set_clock(self.h, C.byref(st)), "claw_set_clock")

    def time_kernel(self, dt: float, reps: int = 20) -> float:
        """Average duration (ms) of one launch of the step kernel (SharpClaw:
        of one stage), timed with HIP events on the library's stream."""
        ms = C.c_double(0.0)
        check(self.lib.claw_time_kernel(self.h, float(dt), int(reps), C.byref(ms)),
              "claw_time_kernel")
        return ms.value

    # -- tiling ------------------------------------------------------------
    def set_tuning(self, seg_rows: int = 0, seg_rows_x: int = 0, segs: int = 0, order: int = 0):
        """Rows per workgroup of the 2D kernels (the y sweeps of a split
        step) and of the x sweeps of a split step (0: seg_rows); segs > 0
        sets the number of row segments instead of seg_rows; order: tile
        order over the workgroups (0-3, see claw_tuning)."""
        tn = ClawTuning()
        tn.seg_rows = int(seg_rows)
        tn.seg_rows_x = int(seg_rows_x)
        tn.segs = int(segs)
        tn.order = int(order)
        check(self.lib.claw_set_tuning(self.h, C.byref(tn)), "claw_set_tuning")

    def get_segs(self) -> int:
        tn = ClawTuning()
        check(self.lib.claw_get_tuning(self.h, C.byref(tn)), "claw_get_tuning")
        return tn.segs

    def get_tuning(self) -> int:
        tn = ClawTuning()
        check(self.lib.claw_get_tuning(self.h, C.byref(tn)), "claw_get_tuning")
        return tn.seg_rows

    def get_order(self) -> int:
        tn = ClawTuning()
        check(self.lib.claw_get_tuning(self.h, C.byref(tn)), "claw_get_tuning")
        return tn.order

    def get_tuning_x(self) -> int:
        tn = ClawTuning()
        check(self.lib.claw_get_tuning(self.h, C.byref(tn)), "claw_get_tuning")
        return tn.seg_rows_x

    def autotune(self, reps: int = 3) -> int:
        tn = ClawTuning()
        check(self.lib.claw_autotune(self.h, int(reps), C.byref(tn)), "claw_autotune")
        return tn.seg_rows

    def close(self):
        if getattr(self, "h", None):
            self.lib.claw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several classic 2D grids advanced by one launch per attempt."""

    def __init__(self, max_grids: int, device="cuda:0", stream=None):
        self.lib = load_library()
        self.device = torch.device(device)
        torch.cuda.set_device(self.device)
        nb = int(self.lib.claw_batch_workspace_bytes(int(max_grids)))
        self._ws, ptr = _aligned_workspace(nb, self.device)
        self.stream = stream
        h = C.c_void_p()
        check(self.lib.claw_batch_create(int(max_grids), C.c_void_p(ptr), nb,
                                         None if stream is None else C.c_void_p(stream.cuda_stream),
                                         C.byref(h)), "claw_batch_create")
        self.h = h
        self.members = []

    def add(self, solver: Solver, t_end: float):
        check(self.lib.claw_batch_add(self.h, solver.h, float(t_end)), "claw_batch_add")
        self.members.append(solver)

    def remove(self, solver: Solver):
        check(self.lib.claw_batch_remove(self.h, solver.h), "claw_batch_remove")
        self.members.remove(solver)

    def advance(self, attempts: int) -> int:
        n = C.c_int(0)
        check(self.lib.claw_batch_advance(self.h, int(attempts), C.byref(n)), "claw_batch_advance")
        return n.value

    def launch(self, attempts: int):
        """Enqueue a group of attempts without waiting (at most two in flight)."""
        check(self.lib.claw_batch_launch(self.h, int(attempts)), "claw_batch_launch")

    def wait(self) -> int:
        """Wait for the oldest group in flight; returns its active members."""
        n = C.c_int(0)
        check(self.lib.claw_batch_wait(self.h, C.byref(n)), "claw_batch_wait")
        return n.value

    def finished(self):
        """Members whose controller stopped as of the last advance()."""
        cap = max(1, len(self.members))
        arr = (C.c_void_p * cap)()
        n = C.c_int(0)
        check(self.lib.claw_batch_finished(self.h, arr, cap, C.byref(n)), "claw_batch_finished")
        done = {arr[k] for k in range(n.value)}
        return [s for s in self.members if s.h.value in done]

    def member_clock(self, solver: Solver) -> dict:
        st = ClawStats()
        check(self.lib.claw_batch_member_clock(self.h, solver.h, C.byref(st)),
              "claw_batch_member_clock")
        return st.as_dict()

    def close(self):
        if getattr(self, "h", None):
            self.lib.claw_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
