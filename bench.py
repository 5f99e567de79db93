"""Benchmark: cell-updates/s of the finite-volume step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]

Headline (one JSON line on stdout): the 2D shallow-water radial dam break,
1024x1024 cells, classic wave propagation with Roe + entropy fix, MC
limiter, full transverse corrections, CFL 0.9, FP64, device-resident step
controller replayed from HIP graphs.  W warm-up steps, then exactly K timed
steps; value = cells x accepted steps / wall time of the timed region
(inputs already resident in HBM).

Extra objects on the same line: FP32+Kahan of the same workload (with its L1
error against the FP64 oracle on a 256^2 sample), the 2D Euler shock-bubble
with SharpClaw WENO5 + HLLE + SSPRK(3,3) (FP64 and FP32+Kahan), the layered
elasticity problem, the 1D dam break, the roofline of the dominant kernel and
the oracle's CPU baseline.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1111_6583_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel: str, field: str):
    """A per-launch figure of a kernel from the committed rocprofv3 PMC
    summary (profiles/traffic.json), or None if the kernels changed since the
    counters were taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    v = d.get("kernels", {}).get(kernel)
    return None if v is None else v.get(field)


def measured_traffic(kernel: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, calibrated), or None."""
    return measured_counters(kernel, "bytes_per_launch")


def timed_run(spec, q, aux, steps, warmup, t_end, tune=True, graph_k=16):
    import torch
    from paper_1111_6583_amd import Solver
    s = Solver(spec)
    s.set_state(q)
    if aux is not None:
        s.set_aux(aux)
    seg = s.autotune(reps=3) if tune else s.get_tuning()
    if warmup:
        s.advance(t_end, max_steps=warmup, steps_per_graph=graph_k)
    c0 = s.clock()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.advance(t_end, max_steps=steps, steps_per_graph=graph_k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc = st["accepted"] - c0["accepted"]
    ncell = int(q.shape[1] * q.shape[2])
    kernel_ms = s.time_kernel(st["dt_next"] * 0.5, reps=20)
    out = dict(cells=ncell, steps=acc, rejected=st["rejected"] - c0["rejected"], wall_s=wall,
               gpu_ms=st["gpu_ms"], seg_rows=seg, segs=s.get_segs(), kernel_ms=kernel_ms, t=st["t"],
               value=ncell * acc / wall, ms_per_step=1e3 * wall / max(acc, 1))
    if spec.get("dimensional_split", "none") != "none":
        out["seg_rows_x"] = s.get_tuning_x()
    s.close()
    return out


# Published MI355X peaks (dense, no sparsity): HBM3E bandwidth and vector
# FP64 / FP32 rates (the FP32 figure counts packed dual FP32 issue).
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}

# Algorithmic work per unit, counted from the method's formulas (each add,
# subtract, multiply, divide, square root, min, max or compare is one flop):
#   sw       2D shallow water, classic, Roe + entropy-fix test, MC, full transverse:
#            per cell-step 554 = 2 faces x (Roe solve 73 + limiter 46 +
#            correction 32 + transverse split and accumulation 106) + cell
#            primitives 4 + update 30 + Courant maxima 6
#   euler    2D Euler SharpClaw, per cell and Runge-Kutta stage 1040 = 4
#            components x 2 directions x WENO5 edge pair 100 + 2 faces x HLLE
#            flux 102 + flux difference 20 + stage combination 12 + maxima 2
# and the compulsory HBM bytes per unit (read stage inputs, write the output,
# plus compensation and aux):
#   sw 48 per cell-step (FP64 q; FP32 q + c); euler per stage 256/3 (FP64),
#   160/3 (FP32+Kahan); elastic 104 (FP64), 92 (FP32+Kahan) per cell-step.
#   euler_stage_weno7  the same with WENO7: edge pair per component and
#            direction 200 (candidates 56, smoothness indicators 96, weights
#            and normalisation 48) -> 8 x 200 + 204 + 20 + 12 + 2 = 1838
#   euler_stage WENO of order 2r-1, r >= 4: edge pair = candidates 2r(2r-1)
#            + smoothness indicators r(r^2 + 3r - 4) (r - 1 zero-sum rows of
#            r, r-1, ..., 2 nonzeros, squared, weighted, summed) + weights and
#            normalisation (48 at r = 4; 11r + 2 with one reciprocal per
#            candidate above) -> 8 x edge pair + 238 (r = 5: 2854, r = 9: 10982)
#   SSPRK(10,4) stage bytes, FP64, averaged over the ten stages: eight plain
#   stages 64 B (S in, y out), stage 5 128 B (S, Q in; two registers out),
#   stage 10 96 B (S, S3 in; Q out) -> 73.6 B per cell-stage.
#   euler_roe  2D Euler, classic, Roe + entropy-fix test, MC, full transverse,
#            tracer, axisymmetric source: per cell-step 1160 = 2 faces x (Roe
#            solve 156 + limiter for 5 waves 90 + correction 60 + transverse
#            split and accumulation 214) + cell primitives 16 + update 50 +
#            source (Heun) 48 + Courant maxima 10; HBM 80 B (5 FP64 in + out)
#   sw_sweep   one 1D sweep of a dimensionally split shallow-water step, per
#            cell: 1 face x (Roe solve 73 + limiter 46 + correction 32) + cell
#            primitives 4 + update 15 + Courant maximum 3 = 173; HBM 48 B (FP64
#            q in + out); Godunov splitting is 2 sweeps a step, Strang 3
#   psystem_stage  2D p-system, SharpClaw WENO5, per cell and stage: 3
#            components x 2 directions x WENO5 edge pair 100 + 2 faces x
#            f-wave flux 35 (two exponentials, two impedances, interface
#            velocity and stress, speed) + flux difference 15 + stage
#            combination 9 + maxima 2 = 696; HBM per cell-stage, FP64,
#            SSPRK(10,4) averaged over the stages: plain stages 64 B (S in, y
#            out, 2 aux), stage 5 112 B, stage 10 88 B -> 71.2 B; FP32+Kahan
#            plain 32 B, stage 5 56 B, stage 10 80 B (Q and its compensation
#            in and out) -> 39.2 B
FLOPS_PER_CELL = {"sw": 554.0, "euler_stage": 1040.0, "euler_stage_weno7": 1838.0,
                  "euler_roe": 1160.0, "sw_sweep": 173.0, "psystem_stage": 696.0}


def euler_stage_flops(order: int) -> float:
    """Algorithmic flops per cell and stage of the 2D Euler SharpClaw step
    with WENO of the given order (the counts above)."""
    if order == 5:
        return FLOPS_PER_CELL["euler_stage"]
    r = (order + 1) // 2
    pair = 2 * r * (2 * r - 1) + r * (r * r + 3 * r - 4) + (48 if r == 4 else 11 * r + 2)
    return 8.0 * pair + 238.0


def roofline(bound, cells, gpu_ms, launches, kernel_name, bytes_per_launch, flops_per_launch=None,
             dtype="f64"):
    """Roofline of the dominant kernel from the HIP-event time of the timed
    region (gpu_ms over `launches` kernel launches).  bound "alu": achieved =
    algorithmic flops per launch / launch time against the vector peak of the
    dtype; bound "hbm": algorithmic bytes per launch / launch time against
    8 TB/s.  The other figure is reported beside it."""
    avg_s = gpu_ms * 1e-3 / launches
    gbs = bytes_per_launch / avg_s / 1e9
    tr = measured_traffic(kernel_name)
    out = dict(kernel=kernel_name, avg_launch_us=round(avg_s * 1e6, 2),
               algorithmic_bytes_per_launch=bytes_per_launch, traffic=tr,
               valu_issue_share=measured_counters(kernel_name, "valu_issue_share"))
    if bound == "alu":
        tf = flops_per_launch / avg_s / 1e12
        peak = PEAK_TFLOPS[dtype]
        out.update(bound="alu", achieved=round(tf, 3), peak=peak, unit="TFLOP/s",
                   frac=round(tf / peak, 4), algorithmic_flops_per_launch=flops_per_launch,
                   hbm=dict(achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                            frac=round(gbs / HBM_PEAK_GBS, 4)))
    else:
        out.update(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                   frac=round(gbs / HBM_PEAK_GBS, 4))
        if flops_per_launch:
            tf = flops_per_launch / avg_s / 1e12
            out["alu"] = dict(achieved=round(tf, 3), peak=PEAK_TFLOPS[dtype], unit="TFLOP/s",
                              frac=round(tf / PEAK_TFLOPS[dtype], 4))
    return out


def l1_error_fp32(spec_fn, n, t_end):
    """L1 relative error per component of FP32+Kahan against the FP64 oracle
    (same dt sequence), on an n x n sample of the workload."""
    import numpy as np
    import oracle
    from paper_1111_6583_amd import Solver
    spec, q = spec_fn(n)
    qo, info = oracle.advance(spec, q, t_end)
    s = Solver(dict(spec, precision="fp32_kahan"))
    s.set_state(q)
    for dt in info["dts"][info["acc"] == 1]:
        s.step(dt)
    g = s.get_state()
    s.close()
    return [float(np.sum(np.abs(g[k] - qo[k])) / np.sum(np.abs(qo[k]))) for k in range(q.shape[0])]


def cpu_baseline(spec, q, steps, steps_1t):
    """The FP64 oracle on the host cores, a bounded sample of the workload:
    `steps` steps with every core of the process, then `steps_1t` with one."""
    import oracle
    dt = 0.9 / oracle.max_cell_speed(spec, q)
    oracle.step(spec, q, dt)   # warm (page in, thread pool)

    def run(n):
        t0 = time.perf_counter()
        qq = q
        for _ in range(n):
            qq, sp = oracle.step(spec, qq, dt)
        return time.perf_counter() - t0

    cores = oracle.num_threads()
    wall = run(steps)
    cells = q.shape[1] * q.shape[2]
    out = dict(value=cells * steps / wall, unit="cell-updates/s", cores=cores, kind="oracle",
               sample=f"{steps} steps of the {q.shape[2]}x{q.shape[1]} grid, FP64, {oracle.cpu_model()}",
               wall_s=round(wall, 2))
    if steps_1t > 0:
        oracle.set_threads(1)
        w1 = run(steps_1t)
        oracle.set_threads(cores)
        out["single_thread"] = dict(value=cells * steps_1t / w1, steps=steps_1t, wall_s=round(w1, 2))
    return out


def mall_sweep(sizes, steps):
    """Shallow-water FP64 step at grids larger than the 256 MB Infinity Cache
    (state ping-pong 48 B/cell), for a true HBM fraction."""
    from paper_1111_6583_amd import workloads as W
    out = {}
    for n in sizes:
        spec, q = W.radial_dam_break(n)
        r = timed_run(spec, q, None, steps, 3, 1.0)
        r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], r["steps"] + r["rejected"],
                                 "k_classic2d<double,ShallowWater>", 48 * r["cells"],
                                 FLOPS_PER_CELL["sw"] * r["cells"], "f64")
        r["state_mb"] = round(2 * 24 * r["cells"] / 1e6, 1)
        out[f"sw_radial_{n}_fp64"] = r
    spec, q = W.shock_bubble(4096, 2048)
    r = timed_run(spec, q, None, 5, 2, 1.0)
    r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], 3 * (r["steps"] + r["rejected"]),
                             "k_sharp2d<double,EulerHLLE>", 256 * r["cells"] / 3.0,
                             FLOPS_PER_CELL["euler_stage"] * r["cells"], "f64")
    r["state_mb"] = round(3 * 32 * r["cells"] / 1e6, 1)
    out["euler_shock_bubble_4096x2048_fp64"] = r
    return out


def host_controller(spec, q, steps):
    """The headline workload stepped by the host controller (claw_advance:
    one launch per attempt, the Courant number read back every step)."""
    import torch
    from paper_1111_6583_amd import Solver
    s = Solver(spec)
    s.set_state(q)
    seg = s.autotune(reps=3)
    s.advance(1.0, max_steps=5, graph=False)
    c0 = s.clock()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.advance(1.0, max_steps=steps, graph=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc = st["accepted"] - c0["accepted"]
    s.close()
    return dict(steps=acc, seg_rows=seg, wall_s=wall, ms_per_step=1e3 * wall / max(acc, 1),
                value=q.shape[1] * q.shape[2] * acc / wall)


def _sb104(W, order):
    spec, q = W.shock_bubble(2048, 1024)
    return (dict(spec, time_integrator="ssp104", weno_order=order, cfl_desired=2.45, cfl_max=2.5),
            q, None)


WORKLOADS = {
    "sw": ("2D shallow water radial dam break 1024^2", lambda W: W.radial_dam_break(1024) + (None,)),
    "euler": ("2D Euler shock-bubble 2048x1024 SharpClaw", lambda W: W.shock_bubble(2048, 1024) + (None,)),
    "elastic": ("2D layered elasticity 2048^2", lambda W: W.layered_elastic(2048)),
    "euler_axisym": ("classic axisymmetric Euler shock-bubble 1280x320 (Roe, tracer, source)",
                     lambda W: W.shock_bubble_axisym(1280, 320) + (None,)),
    "psystem": ("2D p-system checkerboard 4800^2 (20 x 20 periods, 240 cells each) SharpClaw",
                lambda W: W.psystem_checkerboard(240, 20)),
    "sw_godunov": ("2D shallow water radial dam break 1024^2, Godunov split",
                   lambda W: (dict(W.radial_dam_break(1024)[0], dimensional_split="godunov"),
                              W.radial_dam_break(1024)[1], None)),
    "euler_weno9": ("2D Euler shock-bubble 2048x1024 SharpClaw SSPRK(10,4) WENO9",
                    lambda W: _sb104(W, 9)),
    "euler_weno17": ("2D Euler shock-bubble 2048x1024 SharpClaw SSPRK(10,4) WENO17",
                     lambda W: _sb104(W, 17)),
    "sw_strang": ("2D shallow water radial dam break 1024^2, Strang split",
                  lambda W: (dict(W.radial_dam_break(1024)[0], dimensional_split="strang"),
                             W.radial_dam_break(1024)[1], None)),
}


def kernel_only(workload, precision, launches, seg_rows=0, seg_rows_x=0, segs=0):
    """Launch only the step kernel (classic) or stages 1-2 (SharpClaw) of a
    workload `launches` times, for hardware-counter runs.  seg_rows > 0 fixes
    the tiling (no autotuning launches in the profile)."""
    from paper_1111_6583_amd import Solver
    from paper_1111_6583_amd import workloads as W
    name, make = WORKLOADS[workload]
    spec, q, aux = make(W)
    s = Solver(dict(spec, precision=precision))
    s.set_state(q)
    if aux is not None:
        s.set_aux(aux)
    if seg_rows > 0 or segs > 0:
        s.set_tuning(seg_rows, seg_rows_x, segs)
    else:
        s.autotune(reps=2)
    s.advance(1e9, max_steps=10)
    ms = s.time_kernel(s.clock()["dt_next"] * 0.5, reps=launches)
    print(json.dumps(dict(mode="kernel", workload=name, precision=precision, launches=launches,
                          avg_kernel_us=ms * 1e3, seg_rows=s.get_tuning(),
                          segs=s.get_segs())), flush=True)


def copy_only(mib, launches):
    """A plain device copy of known size (calibrates the HBM byte counters)."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(launches):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps(dict(mode="copy", bytes_read_per_launch=4 * n, bytes_written_per_launch=4 * n,
                          launches=launches)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=40)
    ap.add_argument("--cpu-steps-1t", type=int, default=2)
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--mode", choices=["bench", "kernel", "copy"], default="bench",
                    help="kernel/copy: launch only one kernel (for rocprofv3 counter runs)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="sw")
    ap.add_argument("--precision", choices=["fp64", "fp32_kahan"], default="fp64")
    ap.add_argument("--launches", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--seg-rows", type=int, default=0, help="kernel mode: fixed rows per segment")
    ap.add_argument("--segs", type=int, default=0,
                    help="kernel mode: fixed number of row segments (overrides --seg-rows)")
    ap.add_argument("--seg-rows-x", type=int, default=0,
                    help="kernel mode, split steps: fixed rows per segment of the x sweeps")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: this build runs the step on a single MI355X "
              "(multi-GPU decomposition is designed but not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.mode == "kernel":
        return kernel_only(a.workload, a.precision, a.launches, a.seg_rows, a.seg_rows_x, a.segs)
    if a.mode == "copy":
        return copy_only(a.copy_mib, a.launches)

    from paper_1111_6583_amd import workloads as W

    # ---- headline: 2D radial dam break, 1024^2, FP64 ------------------------
    spec, q = W.radial_dam_break(1024)
    log("headline: radial dam break 1024^2 FP64")
    h = timed_run(spec, q, None, a.steps, a.warmup, 1.0)
    line = {
        "metric": "cell-updates/s per GPU (FP64 vs FP32 at stated L1 err); p50/p99 solve latency",
        "value": h["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": h["steps"],
        "warmup": a.warmup, "ms_per_step": h["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded initial data generated on the host)",
        "config": {"workload": "2D shallow-water radial dam break, classic wave propagation "
                               "(Roe + entropy fix, MC, full transverse), 1024x1024, CFL 0.9, "
                               "device-controlled steps toward t=1.0",
                   "cells": h["cells"], "seg_rows": h["seg_rows"], "segs": h["segs"],
                   "parallelism": "single GPU"},
    }
    line["roofline"] = roofline("alu", h["cells"], h["gpu_ms"], h["steps"] + h["rejected"],
                                "k_classic2d<double,ShallowWater>", 48 * h["cells"],
                                FLOPS_PER_CELL["sw"] * h["cells"], "f64")
    line["kernel_isolated_us"] = round(h["kernel_ms"] * 1e3, 2)

    if not a.no_extras:
        extras = {}
        log("fp32+kahan radial dam break")
        f = timed_run(dict(spec, precision="fp32_kahan"), q, None, a.steps, a.warmup, 1.0)
        f["l1_err_vs_fp64_oracle"] = l1_error_fp32(lambda n: W.radial_dam_break(n), 256, 0.25)
        f["l1_err_sample"] = "256x256 to t=0.25, oracle dt sequence"
        f["roofline"] = roofline("alu", f["cells"], f["gpu_ms"], f["steps"] + f["rejected"],
                                 "k_classic2d<float,ShallowWater,Kahan>", 48 * f["cells"],
                                 FLOPS_PER_CELL["sw"] * f["cells"], "f32")
        extras["sw_radial_1024_fp32_kahan"] = f

        log("shock-bubble 2048x1024 SharpClaw FP64 / FP32")
        sb_spec, sb_q = W.shock_bubble(2048, 1024)
        for prec, bpc in (("fp64", 256), ("fp32_kahan", 160)):
            r = timed_run(dict(sb_spec, precision=prec), sb_q, None, 40, 5, 1.0)
            r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], 3 * (r["steps"] + r["rejected"]),
                                     f"k_sharp2d<{'double' if prec == 'fp64' else 'float'},EulerHLLE>",
                                     bpc * r["cells"] / 3.0, FLOPS_PER_CELL["euler_stage"] * r["cells"],
                                     "f64" if prec == "fp64" else "f32")
            if prec == "fp32_kahan":
                r["l1_err_vs_fp64_oracle"] = l1_error_fp32(lambda n: W.shock_bubble(2 * n, n), 128, 0.1)
                r["l1_err_sample"] = "256x128 to t=0.1 (shock through the bubble), oracle dt sequence"
            extras[f"euler_shock_bubble_2048x1024_{prec}"] = r

        log("shock-bubble 2048x1024 SharpClaw SSPRK(10,4) (the SharpClaw default), WENO5/7/9/17")
        for order in (5, 7, 9, 17):
            spec104 = dict(sb_spec, time_integrator="ssp104", weno_order=order, cfl_desired=2.45,
                           cfl_max=2.5)
            r = timed_run(spec104, sb_q, None, 10, 2, 1.0)
            r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], 10 * (r["steps"] + r["rejected"]),
                                     f"k_sharp2d<double,EulerHLLE,SSPRK104,WENO{order}>",
                                     73.6 * r["cells"], euler_stage_flops(order) * r["cells"], "f64")
            r["cfl"] = [2.45, 2.5]
            extras[f"euler_shock_bubble_2048x1024_fp64_ssp104_weno{order}"] = r

        log("classic axisymmetric shock-bubble 1280x320 (the paper's run), Roe + tracer, FP64")
        ax_spec, ax_q = W.shock_bubble_axisym(1280, 320)
        r = timed_run(ax_spec, ax_q, None, 100, 10, 1.0)
        r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], r["steps"] + r["rejected"],
                                 "k_classic2d<double,EulerRoe+tracer>", 80 * r["cells"],
                                 FLOPS_PER_CELL["euler_roe"] * r["cells"], "f64")
        extras["euler_shock_bubble_axisym_1280x320_classic_fp64"] = r

        log("dimensionally split radial dam break 1024^2 (Godunov, Strang), FP64")
        for split, nsw in (("godunov", 2), ("strang", 3)):
            r = timed_run(dict(spec, dimensional_split=split), q, None, a.steps, a.warmup, 1.0)
            r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], nsw * (r["steps"] + r["rejected"]),
                                     f"k_sweep_x/y<double,ShallowWater> ({split})", 48 * r["cells"],
                                     FLOPS_PER_CELL["sw_sweep"] * r["cells"], "f64")
            r["sweeps_per_step"] = nsw
            extras[f"sw_radial_1024_fp64_split_{split}"] = r

        log("p-system checkerboard 4800^2 (20 x 20 periods at 240 cells), SharpClaw WENO5 + SSPRK(10,4)")
        ps_spec, ps_q, ps_aux = W.psystem_checkerboard(240, 20)
        for prec in ("fp64", "fp32_kahan"):
            r = timed_run(dict(ps_spec, precision=prec), ps_q, ps_aux, 10, 2, 1e9)
            r["roofline"] = roofline("alu", r["cells"], r["gpu_ms"], 10 * (r["steps"] + r["rejected"]),
                                     f"k_sharp2d<{'double' if prec == 'fp64' else 'float'},PSystem,SSPRK104>",
                                     (71.2 if prec == "fp64" else 39.2) * r["cells"],
                                     FLOPS_PER_CELL["psystem_stage"] * r["cells"],
                                     "f64" if prec == "fp64" else "f32")
            r["cfl"] = [2.45, 2.5]
            extras[f"psystem_checkerboard_4800_{prec}_ssp104_weno5"] = r
        del ps_q, ps_aux

        log("layered elasticity 2048^2")
        el_spec, el_q, el_aux = W.layered_elastic(2048)
        for prec, bpc in (("fp32_kahan", 92), ("fp64", 104)):
            r = timed_run(dict(el_spec, precision=prec), el_q, el_aux, 100, 10, 10.0)
            r["roofline"] = roofline("hbm", r["cells"], r["gpu_ms"], r["steps"] + r["rejected"],
                                     f"k_classic2d<{'float' if prec != 'fp64' else 'double'},Elastic>",
                                     bpc * r["cells"])
            extras[f"elastic_layered_2048_{prec}"] = r

        log("1D dam break 1000 cells to t=2")
        import torch
        from paper_1111_6583_amd import Solver
        s1, q1 = W.dam_break_1d(1000)
        sv = Solver(s1)
        sv.set_state(q1)
        sv.advance(2.0)          # warm
        sv.set_state(q1)
        sv.set_clock(dict(accepted=0, rejected=0, t=0.0, dt_next=0.0, max_courant=0.0))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = sv.advance(2.0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        extras["sw_dam_break_1d_1000"] = dict(steps=st["accepted"], wall_s=wall,
                                              us_per_step=1e6 * wall / st["accepted"],
                                              gpu_ms=st["gpu_ms"],
                                              value=1000 * st["accepted"] / wall,
                                              path="one-workgroup whole-run kernel (LDS resident)")
        sv.close()

        log(f"serving trace: {a.serve_requests} requests at 200 req/s")
        from paper_1111_6583_amd import serve
        tuner = serve.Tuner()
        warm = W.serving_trace(n_requests=8, rate=200.0, seed=99, t_end=0.5)
        serve.run_trace(warm, tuner=tuner)
        trace = W.serving_trace(n_requests=a.serve_requests, rate=200.0, seed=0, t_end=0.5)
        r = serve.run_trace(trace, tuner=tuner)
        extras["serving_sw_poisson200"] = dict(
            requests=len(trace), p50_s=r["p50"], p99_s=r["p99"],
            throughput_req_s=r["throughput_req_s"], cell_updates_per_s=r["cell_updates_per_s"],
            wall_s=r["wall"], max_resident=r["max_resident"], precision="fp32_kahan",
            budget_gib=8, note="latency = completion (result on host) - scheduled arrival")
        log("host-controller mode (headline workload)")
        extras["sw_radial_1024_fp64_host_controller"] = host_controller(spec, q, 100)
        log("size sweep beyond the Infinity Cache")
        extras.update(mall_sweep((2048, 4096, 8192), 20))
        line["extras"] = extras

    log("cpu baseline (oracle)")
    line["cpu_baseline"] = cpu_baseline(spec, q, a.cpu_steps, a.cpu_steps_1t)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
