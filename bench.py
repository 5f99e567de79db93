"""Benchmark: cell-updates/s of the finite-volume step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras]
                    [--headline WORKLOAD] [--precision P] [--segs S]

Headline (one JSON line on stdout): the 2D Euler shock-bubble interaction,
2048x1024 cells, SharpClaw WENO5 (component-wise) + HLLE + SSPRK(3,3), CFL
0.5 / 0.6, FP64, device-resident step controller replayed from HIP graphs.
W warm-up steps, then exactly K timed steps; value = cells x accepted steps
/ wall time of the timed region (inputs already resident in HBM).

`roofline` is that of the stage kernel: algorithmic HBM bytes per launch
over the average launch duration (HIP events on the library's stream around
the timed region, divided by the launches in it) against 8 TB/s, with the
ALU fraction beside it.  `extras` holds the other workloads: the radial dam
break (classic shallow water), FP32 with a Kahan-compensated update and plain
FP32 (each with its L1 error against the FP64 oracle), SSPRK(10,4) with WENO
5/7/9/17, the classic axisymmetric shock-bubble, split steps, the p-system
checkerboard, layered elasticity, the 1D dam break, the serving trace, the
host-controller mode and a size sweep past the Infinity Cache.
`cpu_baseline` is the FP64 oracle on the host's cores.

--headline/--precision/--segs run one workload alone at a fixed tiling (no
autotuner launches), for rocprofv3 runs of exactly the benchmarked launches.
--mode kernel/copy launch only a step kernel / a plain copy (counter runs).
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
# timed steps by default: whole graphs of 16 attempts, so that no early-exit
# launch enters the timed region or a kernel trace of it
DEFAULT_STEPS = 192
# Published MI355X vector peaks (dense): FP64 78.6 TFLOP/s; FP32 157.3 TFLOP/s,
# which counts packed dual FP32 issue (the kernels are built without packed
# FP32, so half of it is their ceiling)
PEAK_TFLOPS = {"f64": 78.6, "f32": 157.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1111_6583_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_counters(key: str):
    """The counter record of a kernel on a grid ("kernel@NXxNY") from the
    committed rocprofv3 summaries (profiles/traffic.json), or None if there
    is none for that grid or the kernels changed since it was taken."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(p) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("source_hash") != kernel_source_hash():
        return None
    return d.get("kernels", {}).get(key)


# ---------------------------------------------------------------------------
# Workloads: the synthetic inputs (seeded, formed on the host) and the
# algorithmic work per unit of each step kernel, counted from the method's
# formulas (each add, subtract, multiply, divide, square root, min, max or
# compare is one flop):
#   sw       2D shallow water, classic, Roe + entropy-fix test, MC, full
#            transverse: per cell-step 554 = 2 faces x (Roe solve 73 + limiter
#            46 + correction 32 + transverse split and accumulation 106) +
#            cell primitives 4 + update 30 + Courant maxima 6
#   euler    2D Euler SharpClaw, per cell and Runge-Kutta stage 1040 = 4
#            components x 2 directions x WENO5 edge pair 100 + 2 faces x HLLE
#            flux 102 + flux difference 20 + stage combination 12 + maxima 2
#   euler at WENO order 2r-1, r >= 4: edge pair = candidates 2r(2r-1)
#            + smoothness indicators r(r^2 + 3r - 4) + weights and
#            normalisation (48 at r = 4; 11r + 2 above) -> 8 x edge pair + 238
#   euler_roe  2D Euler, classic, Roe + entropy-fix test, MC, full transverse,
#            tracer, axisymmetric source: per cell-step 1160
#   sw_sweep one 1D sweep of a split shallow-water step: 173 per cell
#   psystem  2D p-system SharpClaw WENO5, per cell and stage: 696
# and the compulsory HBM bytes per unit (read stage inputs, write the output,
# plus compensation and aux):
#   sw 48 per cell-step (FP64 q in + out; FP32+Kahan q and c; plain FP32 24)
#   euler SSPRK(3,3), per cell-stage (8 state passes of 4 components per
#         step, 3 stages): FP64 256/3, FP32+Kahan 160/3, plain FP32 128/3
#   euler SSPRK(10,4), FP64, averaged over the ten stages: eight plain stages
#         64 B (S in, y out), stage 5 128 B, stage 10 96 B -> 73.6 B
#   elastic 104 (FP64), 92 (FP32+Kahan: q, c in and out + 3 aux) per cell-step
#   euler_roe 80 per cell-step (5 FP64 components in and out)
#   psystem SSPRK(10,4), per cell-stage: FP64 71.2, FP32+Kahan 39.2
#   sw_sweep 48 per cell-sweep (FP64)
# ---------------------------------------------------------------------------
def euler_stage_flops(order: int) -> float:
    if order == 5:
        return 1040.0
    r = (order + 1) // 2
    pair = 2 * r * (2 * r - 1) + r * (r * r + 3 * r - 4) + (48 if r == 4 else 11 * r + 2)
    return 8.0 * pair + 238.0


def _sb104(W, order):
    spec, q = W.shock_bubble(2048, 1024)
    return (dict(spec, time_integrator="ssp104", weno_order=order, cfl_desired=2.45, cfl_max=2.5),
            q, None)


def _split(W, kind):
    spec, q = W.radial_dam_break(1024)
    return dict(spec, dimensional_split=kind), q, None


# template precision in kernel labels ("float+Kahan": FP32 with a compensated update)
KERNEL_PRECISION = {"fp64": "double", "fp32_kahan": "float+Kahan", "fp32": "float"}

# name -> description, maker, launches per step, bytes per cell and launch by
# precision, flops per cell and launch, kernel label, t_end, (steps, warmup)
WORKLOADS = {
    "euler": ("2D Euler shock-bubble (Mach 2 shock, bubble density 0.1), SharpClaw WENO5 "
              "component-wise + HLLE + SSPRK(3,3), 2048x1024, CFL 0.5/0.6",
              lambda W: W.shock_bubble(2048, 1024) + (None,), 3,
              {"fp64": 256 / 3, "fp32_kahan": 160 / 3, "fp32": 128 / 3}, 1040.0,
              "k_sharp2d<{R},EulerHLLE,WENO5>", 1.0, None),
    "sw": ("2D shallow-water radial dam break, classic wave propagation (Roe + entropy fix, MC, "
           "full transverse), 1024x1024, CFL 0.9",
           lambda W: W.radial_dam_break(1024) + (None,), 1,
           {"fp64": 48, "fp32_kahan": 48, "fp32": 24}, 554.0,
           "k_classic2d<{R},ShallowWater>", 1.0, None),
    "elastic": ("2D linear elasticity, 16 seeded layers, classic variable-coefficient Riemann "
                "solver, MC, full transverse, 2048x2048, CFL 0.9",
                lambda W: W.layered_elastic(2048), 1, {"fp64": 104, "fp32_kahan": 92}, None,
                "k_classic2d<{R},Elastic>", 10.0, (96, 16)),
    "euler_axisym": ("classic axisymmetric Euler shock-bubble 1280x320 (Roe, tracer, source)",
                     lambda W: W.shock_bubble_axisym(1280, 320) + (None,), 1, {"fp64": 80}, 1160.0,
                     "k_classic2d<{R},EulerRoe+tracer>", 1.0, (96, 16)),
    "psystem": ("2D p-system checkerboard 4800^2 (20 x 20 periods, 240 cells each), SharpClaw "
                "WENO5 + SSPRK(10,4)", lambda W: W.psystem_checkerboard(240, 20), 10,
                {"fp64": 71.2, "fp32_kahan": 39.2}, 696.0, "k_sharp2d<{R},PSystem,SSPRK104>",
                1e9, (16, 16)),
    "sw_godunov": ("2D shallow-water radial dam break 1024^2, Godunov-split sweeps",
                   lambda W: _split(W, "godunov"), 2, {"fp64": 48}, 173.0,
                   "k_sweep_x/y<{R},ShallowWater> (godunov)", 1.0, None),
    "sw_strang": ("2D shallow-water radial dam break 1024^2, Strang-split sweeps",
                  lambda W: _split(W, "strang"), 3, {"fp64": 48}, 173.0,
                  "k_sweep_x/y<{R},ShallowWater> (strang)", 1.0, None),
}
for _o in (5, 7, 9, 17):
    WORKLOADS[f"euler_ssp104_weno{_o}"] = (
        f"2D Euler shock-bubble 2048x1024, SharpClaw SSPRK(10,4) WENO{_o}, CFL 2.45/2.5",
        (lambda o: (lambda W: _sb104(W, o)))(_o), 10, {"fp64": 73.6}, euler_stage_flops(_o),
        f"k_sharp2d<{{R}},EulerHLLE,SSPRK104,WENO{_o}>", 1.0, (16, 16))


def grid_label(q) -> str:
    return f"{q.shape[2]}x{q.shape[1]}"


def timed_run(spec, q, aux, steps, warmup, t_end, segs=0, order=0, seg_rows_x=0, graph_k=16):
    import torch
    from paper_1111_6583_amd import Solver
    s = Solver(spec)
    s.set_state(q)
    if aux is not None:
        s.set_aux(aux)
    if segs > 0:
        s.set_tuning(segs=segs, order=order, seg_rows_x=seg_rows_x)
    else:
        s.autotune(reps=10)
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
    out = dict(cells=ncell, grid=grid_label(q), steps=acc, warmup=warmup,
               rejected=st["rejected"] - c0["rejected"],
               wall_s=wall, gpu_ms=st["gpu_ms"], segs=s.get_segs(), seg_rows=s.get_tuning(),
               order=s.get_order(), t=st["t"], value=ncell * acc / wall,
               ms_per_step=1e3 * wall / max(acc, 1))
    if spec.get("dimensional_split", "none") != "none":
        out["seg_rows_x"] = s.get_tuning_x()
    s.close()
    return out


def roofline(r, launches_per_step, bytes_per_cell, flops_per_cell, kernel, dtype):
    """Roofline of a step kernel from the HIP-event time of the timed region
    (gpu_ms over its launches): achieved = algorithmic bytes per launch /
    average launch time against 8 TB/s; the ALU fraction (algorithmic flops
    against the vector peak of the dtype) beside it; `traffic` = measured HBM
    bytes per launch of this kernel on this grid (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, calibrated), or null."""
    launches = launches_per_step * (r["steps"] + r["rejected"])
    avg_s = r["gpu_ms"] * 1e-3 / launches
    b = bytes_per_cell * r["cells"]
    gbs = b / avg_s / 1e9
    key = f"{kernel}@{r['grid']}"
    rec = measured_counters(key)
    out = dict(bound="hbm", achieved=round(gbs, 1), peak=HBM_PEAK_GBS, unit="GB/s",
               frac=round(gbs / HBM_PEAK_GBS, 4), traffic=None if rec is None else rec["bytes_per_launch"],
               kernel=key, avg_launch_us=round(avg_s * 1e6, 2), launches=launches,
               algorithmic_bytes_per_launch=round(b))
    if rec is not None:
        out["valu_issue_share"] = rec.get("valu_issue_share")
        out["profile"] = rec.get("profile")
        # what the counters say limits the launch: the share of the SIMDs'
        # time spent issuing VALU instructions against the fraction of the
        # HBM peak its measured traffic takes
        hbm_busy = rec["bytes_per_launch"] / avg_s / (HBM_PEAK_GBS * 1e9)
        out["hbm_busy_measured"] = round(hbm_busy, 3)
        issue = rec.get("valu_issue_share") or 0.0
        out["bound_measured"] = "alu" if issue >= hbm_busy else "hbm"
    if flops_per_cell:
        tf = flops_per_cell * r["cells"] / avg_s / 1e12
        out["alu"] = dict(achieved=round(tf, 3), peak=PEAK_TFLOPS[dtype], unit="TFLOP/s",
                          frac=round(tf / PEAK_TFLOPS[dtype], 4),
                          algorithmic_flops_per_launch=round(flops_per_cell * r["cells"]))
    return out


def run_workload(W, name, precision, steps, warmup, segs=0, order=0, seg_rows_x=0):
    desc, make, lps, bpc, fpc, kernel, t_end, sw = WORKLOADS[name]
    spec, q, aux = make(W)
    if steps is None:
        steps, warmup = sw if sw is not None else (DEFAULT_STEPS, warmup)
    r = timed_run(dict(spec, precision=precision), q, aux, steps, warmup, t_end, segs=segs,
                  order=order, seg_rows_x=seg_rows_x)
    dtype = "f64" if precision == "fp64" else "f32"
    r["roofline"] = roofline(r, lps, bpc[precision], fpc, kernel.format(R=KERNEL_PRECISION[precision]),
                             dtype)
    r["workload"] = desc
    r["precision"] = precision
    return r


def l1_error(spec, q, aux, precision, t_end=1.0, max_steps=None):
    """Relative L1 error per component of an FP32 precision against the FP64
    oracle run with the same dt sequence (oracle on the host)."""
    import numpy as np
    import oracle
    from paper_1111_6583_amd import Solver
    kw = {} if max_steps is None else dict(max_steps=max_steps)
    qo, info = oracle.advance(spec, q, t_end, aux=aux, **kw)
    s = Solver(dict(spec, precision=precision))
    s.set_state(q)
    if aux is not None:
        s.set_aux(aux)
    dts = info["dts"][info["acc"] == 1]
    for dt in dts:
        s.step(dt)
    g = s.get_state()
    s.close()
    return [float(np.sum(np.abs(g[k] - qo[k])) / np.sum(np.abs(qo[k]))) for k in range(q.shape[0])], len(dts)


# L1 samples: each FP32 line's workload at a size the oracle finishes in
# seconds, with the oracle's dt sequence
def l1_sample(W, name, precision):
    if name == "euler":
        spec, q = W.shock_bubble(256, 128)
        err, n = l1_error(spec, q, None, precision, 0.1)
        return err, f"256x128 to t=0.1 ({n} steps, the shock through the bubble)"
    if name == "sw":
        spec, q = W.radial_dam_break(256)
        err, n = l1_error(spec, q, None, precision, 0.25)
        return err, f"256x256 to t=0.25 ({n} steps)"
    if name == "elastic":
        spec, q, aux = W.layered_elastic(256)
        err, n = l1_error(spec, q, aux, precision, 1.0, max_steps=100)
        return err, f"256x256, {n} steps"
    if name == "psystem":
        spec, q, aux = W.psystem_checkerboard(24, 4)
        err, n = l1_error(spec, q, aux, precision, 1e9, max_steps=20)
        return err, f"96x96 (4 x 4 periods at 24 cells), {n} steps"
    return None, None


def cpu_baseline(spec, q, steps, steps_1t):
    """The FP64 oracle on the host cores, a bounded sample of the headline
    workload: `steps` steps with every core of the process, then `steps_1t`
    with one."""
    import oracle
    dt = 0.5 / oracle.max_cell_speed(spec, q)
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
               sample=f"{steps} steps (3 stages each) of the {q.shape[2]}x{q.shape[1]} shock-bubble, "
                      f"FP64, OpenMP over rows, {oracle.cpu_model()}",
               wall_s=round(wall, 2))
    if steps_1t > 0:
        oracle.set_threads(1)
        w1 = run(steps_1t)
        oracle.set_threads(cores)
        v1 = cells * steps_1t / w1
        out["single_thread"] = dict(value=v1, steps=steps_1t, wall_s=round(w1, 2))
        out["parallel_speedup"] = round(out["value"] / v1, 2)
    return out


def host_controller(W, steps):
    """The radial dam break stepped by the host controller (claw_advance: one
    launch per attempt, the Courant number read back every step)."""
    import torch
    from paper_1111_6583_amd import Solver
    spec, q = W.radial_dam_break(1024)
    s = Solver(spec)
    s.set_state(q)
    s.autotune(reps=3)
    s.advance(1.0, max_steps=5, graph=False)
    c0 = s.clock()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = s.advance(1.0, max_steps=steps, graph=False)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    acc = st["accepted"] - c0["accepted"]
    s.close()
    return dict(steps=acc, wall_s=wall, ms_per_step=1e3 * wall / max(acc, 1),
                value=q.shape[1] * q.shape[2] * acc / wall)


def mall_sweep(W):
    """Steps at grids larger than the 256 MB Infinity Cache, for a true HBM
    fraction (shallow water state ping-pong 48 B/cell; Euler Q + 2 stages)."""
    out = {}
    for n in (2048, 4096, 8192):
        spec, q = W.radial_dam_break(n)
        r = timed_run(spec, q, None, 20, 3, 1.0)
        r["roofline"] = roofline(r, 1, 48, 554.0, "k_classic2d<double,ShallowWater>", "f64")
        r["state_mb"] = round(2 * 24 * r["cells"] / 1e6, 1)
        out[f"sw_radial_{n}_fp64"] = r
    spec, q = W.shock_bubble(4096, 2048)
    r = timed_run(spec, q, None, 5, 2, 1.0)
    r["roofline"] = roofline(r, 3, 256 / 3, 1040.0, "k_sharp2d<double,EulerHLLE,WENO5>", "f64")
    r["state_mb"] = round(3 * 32 * r["cells"] / 1e6, 1)
    out["euler_shock_bubble_4096x2048_fp64"] = r
    return out


def serving(W, n_requests, n_warm):
    """S13's trace: Poisson arrivals at 200 req/s of shallow-water humps
    (N ~ U{64..1024}), FP32+Kahan, each to t = 0.5; n_warm requests first
    (not measured), then n_requests measured.  Latency = completion (result
    on the host) - scheduled arrival."""
    import numpy as np
    from paper_1111_6583_amd import serve
    tuner = serve.Tuner()
    warm = W.serving_trace(n_requests=n_warm, rate=200.0, seed=99, t_end=0.5)
    serve.run_trace(warm, tuner=tuner)
    trace = W.serving_trace(n_requests=n_requests, rate=200.0, seed=0, t_end=0.5)
    r = serve.run_trace(trace, tuner=tuner)
    lat = r["latencies"]
    half = lat[: len(lat) // 2]
    # p50 / p99 per 500 consecutive requests (in arrival order): they swing
    # with bursts of large grids, but do not drift if the load is carried
    win = [(round(float(np.percentile(lat[i:i + 500], 50)), 4),
            round(float(np.percentile(lat[i:i + 500], 99)), 4)) for i in range(0, len(lat), 500)]
    st = r.get("stats", {})
    return dict(requests=len(trace), warmup_requests=n_warm, offered_req_s=200.0,
                throughput_req_s=r["throughput_req_s"], p50_s=r["p50"], p99_s=r["p99"],
                first_half_p50_s=float(np.percentile(half, 50)),
                first_half_p99_s=float(np.percentile(half, 99)),
                p50_p99_per_500_requests=win,
                gpu_busy_fraction=round(st["gpu_busy_s"] / r["wall"], 3) if "gpu_busy_s" in st else None,
                cell_updates_per_s=r["cell_updates_per_s"], wall_s=r["wall"],
                max_resident=r["max_resident"], precision="fp32_kahan", budget_gib=8,
                tiling_by_bucket=tuner.describe(), **r.get("stats", {}))


def dam_break_1d(W):
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
    sv.close()
    return dict(steps=st["accepted"], wall_s=wall, us_per_step=1e6 * wall / st["accepted"],
                gpu_ms=st["gpu_ms"], value=1000 * st["accepted"] / wall,
                path="one-workgroup whole-run kernel (LDS resident)")


def kernel_only(workload, precision, launches, segs):
    """Launch only the step kernel (classic) or stages 1-2 (SharpClaw) of a
    workload `launches` times (host dt), for hardware-counter runs."""
    from paper_1111_6583_amd import Solver
    from paper_1111_6583_amd import workloads as W
    desc, make = WORKLOADS[workload][:2]
    spec, q, aux = make(W)
    s = Solver(dict(spec, precision=precision))
    s.set_state(q)
    if aux is not None:
        s.set_aux(aux)
    if segs > 0:
        s.set_tuning(segs=segs)
    else:
        s.autotune(reps=2)
    s.advance(1e9, max_steps=3)
    ms = s.time_kernel(s.clock()["dt_next"] * 0.5, reps=launches)
    print(json.dumps(dict(mode="kernel", workload=desc, precision=precision, launches=launches,
                          avg_kernel_us=ms * 1e3, segs=s.get_segs())), flush=True)


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
    ap.add_argument("--steps", type=int, default=None,
                    help=f"timed steps (default {DEFAULT_STEPS}, or the workload's own count)")
    ap.add_argument("--warmup", type=int, default=16)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--headline", choices=sorted(WORKLOADS), default="euler",
                    help="workload of the headline line (default: the shock-bubble)")
    ap.add_argument("--precision", choices=["fp64", "fp32_kahan", "fp32"], default="fp64")
    ap.add_argument("--segs", type=int, default=0,
                    help="fixed number of row segments of the headline (0: autotune)")
    ap.add_argument("--order", type=int, default=0, help="tile order with --segs (0-3)")
    ap.add_argument("--seg-rows-x", type=int, default=0,
                    help="rows per segment of a split step's x sweeps with --segs")
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--cpu-steps-1t", type=int, default=5)
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-warmup", type=int, default=200)
    ap.add_argument("--mode", choices=["bench", "kernel", "copy"], default="bench")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="euler")
    ap.add_argument("--launches", type=int, default=20)
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py measures one GPU: the step runs on a single MI355X (the multi-GPU "
              "decomposition is designed, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    if a.mode == "kernel":
        return kernel_only(a.workload, a.precision, a.launches, a.segs)
    if a.mode == "copy":
        return copy_only(a.copy_mib, a.launches)

    from paper_1111_6583_amd import workloads as W

    log(f"headline: {a.headline} {a.precision}")
    h = run_workload(W, a.headline, a.precision, a.steps, a.warmup, a.segs, a.order, a.seg_rows_x)
    line = {
        "metric": "cell-updates/s per GPU (FP64 vs FP32 at stated L1 err); p50/p99 solve latency",
        "value": h["value"], "unit": "cell-updates/s", "n_gpus": 1, "steps": h["steps"],
        "warmup": h["warmup"], "ms_per_step": h["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32",
        "data": "synthetic (seeded initial data generated on the host)",
        "config": {"workload": h["workload"] + ", device-controlled steps replayed from HIP graphs",
                   "cells": h["cells"], "grid": h["grid"], "precision": a.precision,
                   "segs": h["segs"], "seg_rows": h["seg_rows"], "tile_order": h["order"],
                   "parallelism": "single GPU"},
        "roofline": h["roofline"],
    }

    if not a.no_extras:
        extras = {}
        for name, prec in (("euler", "fp32_kahan"), ("euler", "fp32"), ("sw", "fp64"),
                           ("sw", "fp32_kahan"), ("sw", "fp32"), ("elastic", "fp32_kahan"),
                           ("elastic", "fp64"), ("psystem", "fp64"), ("psystem", "fp32_kahan"),
                           ("euler_axisym", "fp64"), ("sw_godunov", "fp64"), ("sw_strang", "fp64"),
                           ("euler_ssp104_weno5", "fp64"), ("euler_ssp104_weno7", "fp64"),
                           ("euler_ssp104_weno9", "fp64"), ("euler_ssp104_weno17", "fp64")):
            log(f"{name} {prec}")
            r = run_workload(W, name, prec, a.steps, a.warmup)
            if prec != "fp64":
                err, sample = l1_sample(W, name, prec)
                r["l1_err_vs_fp64_oracle"] = err
                r["l1_err_sample"] = sample
            extras[f"{name}_{r['grid']}_{prec}"] = r
        log("1D dam break 1000 cells to t=2")
        extras["sw_dam_break_1d_1000"] = dam_break_1d(W)
        log(f"serving trace: {a.serve_warmup} + {a.serve_requests} requests at 200 req/s")
        extras["serving_sw_poisson200"] = serving(W, a.serve_requests, a.serve_warmup)
        log("host-controller mode (radial dam break)")
        extras["sw_radial_1024_fp64_host_controller"] = host_controller(W, 100)
        log("size sweep beyond the Infinity Cache")
        extras.update(mall_sweep(W))
        line["extras"] = extras

    if a.cpu_steps > 0 and a.headline == "euler":
        log("cpu baseline (oracle)")
        spec, q = W.shock_bubble(2048, 1024)
        line["cpu_baseline"] = cpu_baseline(spec, q, a.cpu_steps, a.cpu_steps_1t)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
