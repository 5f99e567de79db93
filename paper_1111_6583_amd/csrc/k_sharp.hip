// k_sharp.hip -- the SharpClaw step on gfx950: WENO5 edge values, interface
// flux, flux differencing, SSPRK(3,3) stage combination (Section 2: method of
// lines with WENO reconstruction; Section 2.1: SSP Runge-Kutta in time,
// normal Riemann problems only in multi-D).
//
// One launch per Runge-Kutta stage.  With L(S) = -(F_{i+1/2}-F_{i-1/2})/dx
// - (G_{j+1/2}-G_{j-1/2})/dy evaluated on the stage input S:
//   stage 1: S1 = Q + dt L(Q)                      (speeds for the Courant number)
//   stage 2: S2 = 3/4 Q + 1/4 (S1 + dt L(S1))
//   stage 3: Q  = 1/3 Q + 2/3 (S2 + dt L(S2))      (in place; FP32 mode adds the
//            increment 2/3 ((S2 - Q) + dt L(S2)) to Q with Kahan compensation)
//
// 2D layout: one wavefront per strip of 58 columns (3 halo lanes each side)
// marching up a segment of rows; the y-stencil lives in a five-row register
// window and each y-face flux is computed once and carried to the next row.
#include "dev_common.h"
#include "phys.h"

namespace claw {

// Pointwise inputs of the stage combination for one cell (Q^n, and the
// compensation in FP32 stage 3), read one row ahead of their use.
template <typename R, int M, int STAGE, bool KAHAN>
__device__ __forceinline__ void load_point(gconst<R> Qn, gconst<R> Cn, size_t idx, size_t plane,
                                           R (&qn)[M], R (&cn)[M]) {
#pragma unroll
  for (int k = 0; k < M; ++k) {
    qn[k] = STAGE >= 2 ? Qn[k * plane + idx] : R(0);
    cn[k] = (STAGE == 3 && KAHAN) ? Cn[k * plane + idx] : R(0);
  }
}

// Output of a stage: S1 (stage 1), S2 (stage 2) or Q in place (stage 3, with
// its compensation C in FP32 mode).
template <typename R, int STAGE>
__device__ __forceinline__ gmut<R> stage_out(const GridDesc& G) {
  return as_gmut<R>(STAGE == 1 ? G.s1 : (STAGE == 2 ? G.s2 : G.q[0]));
}

template <typename R, class P, int STAGE, bool KAHAN>
__device__ __forceinline__ void combine_store(gmut<R> O, gmut<R> C, size_t idx, size_t plane,
                                              const R (&S)[P::M], const R (&L)[P::M], R dt,
                                              const R (&qn)[P::M], const R (&cn)[P::M]) {
  constexpr int M = P::M;
  if constexpr (STAGE == 1) {
#pragma unroll
    for (int k = 0; k < M; ++k) O[k * plane + idx] = S[k] + dt * L[k];
  } else if constexpr (STAGE == 2) {
#pragma unroll
    for (int k = 0; k < M; ++k) O[k * plane + idx] = R(0.75) * qn[k] + R(0.25) * (S[k] + dt * L[k]);
  } else {
    if constexpr (KAHAN) {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const R inc = R(2.0 / 3.0) * ((S[k] - qn[k]) + dt * L[k]);
        const R y = inc - cn[k];
        const R t = qn[k] + y;
        C[k * plane + idx] = (t - qn[k]) - y;
        O[k * plane + idx] = t;
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) O[k * plane + idx] = qn[k] / R(3) + R(2.0 / 3.0) * (S[k] + dt * L[k]);
    }
  }
}

// Common prologue: dt of this stage, or an early exit.
template <int STAGE>
__device__ __forceinline__ bool stage_dt(Ctrl* ctrl, int mode, double dt_host, double& dt) {
  if (mode == kDeviceCtrl) {
    if (STAGE == 1) {
      if (!ctrl->active) {
        if (blockIdx.x == 0 && threadIdx.x == 0) ctrl->ok = 0;
        return false;
      }
      dt = ctrl->dt_try;
    } else {
      if (!ctrl->ok) return false;
      dt = ctrl->dt_stage;
    }
  } else {
    dt = dt_host;
  }
  return true;
}

template <int STAGE>
__device__ __forceinline__ void stage_finish(Ctrl* ctrl, int mode, double speed, int nblocks) {
  if constexpr (STAGE == 1) {
    if (mode == kDeviceCtrl) {
      finish_workgroup(ctrl, speed, nblocks, [](Ctrl* c, double sp) {
        const double d = c->dt_try;
        c->ok = ctrl_decide(c, sp) ? 1 : 0;
        c->dt_stage = d;
      });
    } else {
      finish_workgroup(ctrl, speed, nblocks, [](Ctrl* c, double sp) { c->last_speed = sp; });
    }
  }
}

template <typename R, class P, int STAGE, bool KAHAN>
__global__ __launch_bounds__(kLanes) void k_sharp2d(const GridDesc* __restrict__ grids, int mode,
                                                    double dt_host) {
  constexpr int M = P::M;
  constexpr int H = 3, U = kLanes - 2 * H;
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  double dtd;
  if (!stage_dt<STAGE>(ctrl, mode, dt_host, dtd)) return;
  const R dt = (R)dtd;
  const int strip = blockIdx.x % G.strips, seg = blockIdx.x / G.strips;
  const int nx = G.nx, ny = G.ny;
  const size_t plane = (size_t)nx * ny;
  const int lane = threadIdx.x;
  const int i = strip * U - H + lane;
  const bool own = lane >= H && lane < H + U && i < nx;
  const bool own_face = lane >= H && lane <= H + U && i <= nx;
  const int j0 = seg * G.seg_rows;
  const int j1 = min(j0 + G.seg_rows, ny);
  const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], H);
  const int bcy0 = G.bc[2], bcy1 = G.bc[3];
  const EdgeStates<R, M> es = edge_states<R, M>(G, mx);
  const gconst<R> S = as_gconst<R>(STAGE == 1 ? G.q[0] : (STAGE == 2 ? G.s1 : G.s2));
  const R eps = (R)G.weno_eps;
  const R rdx = (R)(1.0 / G.dx), rdy = (R)(1.0 / G.dy);
  const P phys(G);
  R smx = R(0), smy = R(0);

  R w[5][M];          // rows r-4 .. r
  R qyl_prev[M], g_lo[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    qyl_prev[k] = g_lo[k] = R(0);
#pragma unroll
    for (int s = 0; s < 5; ++s) w[s][k] = R(0);
  }
  const gconst<R> Qn = as_gconst<R>(G.q[0]);
  const gconst<R> Cn = as_gconst<R>(G.c[0]);
  const gmut<R> Out = stage_out<R, STAGE>(G);
  const gmut<R> Cout = as_gmut<R>(G.c[0]);
  // Row r+1 is loaded while row r is processed (software pipelining) and
  // enters the window with its boundary conditions applied just before row
  // r's results are stored (the wait for the load then comes a row of work
  // after it was issued, and never behind stores).  The pointwise Q^n (and
  // compensation) of the row finalised next iteration is read ahead too.
  R pre[M], nxt[M], pq[M], pc[M], uq[M], uc[M];
  load_state<R, P>(nxt, S, plane, nx, mx, map_axis(j0 - 3, ny, bcy0, bcy1, H), es);
#pragma unroll
  for (int k = 0; k < M; ++k) pq[k] = pc[k] = uq[k] = uc[k] = R(0);
  const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);   // clamped column for pointwise reads
  for (int r = j0 - 3; r <= j1 + 2; ++r) {
#pragma unroll
    for (int k = 0; k < M; ++k) { uq[k] = pq[k]; uc[k] = pc[k]; }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int k = 0; k < M; ++k) w[s][k] = w[s + 1][k];
#pragma unroll
    for (int k = 0; k < M; ++k) w[4][k] = nxt[k];
    const bool more = r + 1 <= j1 + 2;
    AxisMap mynext{0, 0, 0};
    if (more) {
      mynext = map_axis(r + 1, ny, bcy0, bcy1, H);
      load_raw<R, M>(pre, S, plane, nx, mx, mynext);
    }
    if (STAGE >= 2 && r - 2 >= j0 && r - 2 < j1)
      load_point<R, M, STAGE, KAHAN>(Qn, Cn, (size_t)(r - 2) * nx + ic, plane, pq, pc);
    R Lv[M], Sc[M];
    bool store = false;
    if (r >= j0 + 1) {
      // y edge values of row c = r-2
      R qyl[M], qyr[M];
#pragma unroll
      for (int k = 0; k < M; ++k)
        weno5_edges(w[0][k], w[1][k], w[2][k], w[3][k], w[4][k], eps, qyl[k], qyr[k]);
      if (r >= j0 + 2) {
        // y-face flux at c-1/2
        R g_up[M];
        const R sy = phys.template flux<1>(qyl_prev, qyr, g_up);
        smy = max_nan(smy, sy);
        if (r >= j0 + 3) {
          // row f = r-3 (window row 1) is complete: x edge values, x-face fluxes
          R xl[M], xr[M];
#pragma unroll
          for (int k = 0; k < M; ++k) {
            const R c0 = w[1][k];
            const R m1 = shfl_prev(c0), p1 = shfl_next(c0);
            const R m2 = shfl_prev(m1), p2 = shfl_next(p1);
            weno5_edges(m2, m1, c0, p1, p2, eps, xl[k], xr[k]);
          }
          R ql[M], F[M];
#pragma unroll
          for (int k = 0; k < M; ++k) ql[k] = shfl_prev(xl[k]);
          const R sx = phys.template flux<0>(ql, xr, F);
          if (own_face) smx = max_nan(smx, sx);
#pragma unroll
          for (int k = 0; k < M; ++k) {
            const R Fr = shfl_next(F[k]);
            Lv[k] = -(Fr - F[k]) * rdx - (g_up[k] - g_lo[k]) * rdy;
            Sc[k] = w[1][k];
          }
          store = true;
        }
#pragma unroll
        for (int k = 0; k < M; ++k) g_lo[k] = g_up[k];
      }
#pragma unroll
      for (int k = 0; k < M; ++k) qyl_prev[k] = qyl[k];
    }
    if (more) {
#pragma unroll
      for (int k = 0; k < M; ++k) nxt[k] = pre[k];
      apply_bc<R, P>(nxt, mx, mynext, es);
    }
    if (store && own)
      combine_store<R, P, STAGE, KAHAN>(Out, Cout, (size_t)(r - 3) * nx + i, plane, Sc, Lv, dt, uq, uc);
  }
  const double speed = own ? max_nan((double)smx * (1.0 / G.dx), (double)smy * (1.0 / G.dy))
                           : (own_face ? (double)smx * (1.0 / G.dx) : 0.0);
  stage_finish<STAGE>(ctrl, mode, speed, G.nblocks);
}

template <typename R, class P, int STAGE, bool KAHAN>
__global__ __launch_bounds__(kLanes) void k_sharp1d(const GridDesc* __restrict__ grids, int mode,
                                                    double dt_host) {
  constexpr int M = P::M;
  constexpr int H = 3, U = kLanes - 2 * H;
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  double dtd;
  if (!stage_dt<STAGE>(ctrl, mode, dt_host, dtd)) return;
  const R dt = (R)dtd;
  const int nx = G.nx;
  const int lane = threadIdx.x;
  const int i = blockIdx.x * U - H + lane;
  const bool own = lane >= H && lane < H + U && i < nx;
  const bool own_face = lane >= H && lane <= H + U && i <= nx;
  const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], H);
  const AxisMap my{0, 0, 0};
  const gconst<R> S = as_gconst<R>(STAGE == 1 ? G.q[0] : (STAGE == 2 ? G.s1 : G.s2));
  const R eps = (R)G.weno_eps;
  const R rdx = (R)(1.0 / G.dx);
  const P phys(G);
  R c[M], xl[M], xr[M];
  load_state<R, P>(c, S, (size_t)nx, nx, mx, my, edge_states<R, M>(G, mx));
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const R m1 = shfl_prev(c[k]), p1 = shfl_next(c[k]);
    const R m2 = shfl_prev(m1), p2 = shfl_next(p1);
    weno5_edges(m2, m1, c[k], p1, p2, eps, xl[k], xr[k]);
  }
  R ql[M], F[M], Lv[M];
#pragma unroll
  for (int k = 0; k < M; ++k) ql[k] = shfl_prev(xl[k]);
  const R sx = phys.template flux<0>(ql, xr, F);
#pragma unroll
  for (int k = 0; k < M; ++k) Lv[k] = -(shfl_next(F[k]) - F[k]) * rdx;
  R pq[M], pc[M];
  load_point<R, M, STAGE, KAHAN>(as_gconst<R>(G.q[0]), as_gconst<R>(G.c[0]),
                                 (size_t)(i < 0 ? 0 : (i >= nx ? nx - 1 : i)), (size_t)nx, pq, pc);
  if (own)
    combine_store<R, P, STAGE, KAHAN>(stage_out<R, STAGE>(G), as_gmut<R>(G.c[0]), (size_t)i,
                                      (size_t)nx, c, Lv, dt, pq, pc);
  const double speed = own_face ? (double)sx * (1.0 / G.dx) : 0.0;
  stage_finish<STAGE>(ctrl, mode, speed, G.nblocks);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename R, bool K, int NDIM, int STAGE>
static hipError_t sharp_t(int riemann, dim3 grid, hipStream_t st, const GridDesc* g, int mode,
                          double dt) {
  if (NDIM == 2) {
    switch (riemann) {
      case 1:
        hipLaunchKernelGGL((k_sharp2d<R, AdvectionFlux<R, 2>, STAGE, K>), grid, dim3(kLanes), 0,
                           st, g, mode, dt);
        break;
      case 3:
        hipLaunchKernelGGL((k_sharp2d<R, EulerHLLE<R, 2>, STAGE, K>), grid, dim3(kLanes), 0, st,
                           g, mode, dt);
        break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (riemann) {
      case 1:
        hipLaunchKernelGGL((k_sharp1d<R, AdvectionFlux<R, 1>, STAGE, K>), grid, dim3(kLanes), 0,
                           st, g, mode, dt);
        break;
      case 3:
        hipLaunchKernelGGL((k_sharp1d<R, EulerHLLE<R, 1>, STAGE, K>), grid, dim3(kLanes), 0, st,
                           g, mode, dt);
        break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename R, bool K, int NDIM>
static hipError_t sharp_nd(int riemann, int stage, dim3 grid, hipStream_t st, const GridDesc* g,
                           int mode, double dt) {
  switch (stage) {
    case 1: return sharp_t<R, K, NDIM, 1>(riemann, grid, st, g, mode, dt);
    case 2: return sharp_t<R, K, NDIM, 2>(riemann, grid, st, g, mode, dt);
    case 3: return sharp_t<R, K, NDIM, 3>(riemann, grid, st, g, mode, dt);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sharp_stage(int ndim, int riemann, int fp32, int stage, int nblocks,
                              hipStream_t st, const GridDesc* d_grids, int mode, double dt) {
  const dim3 grid(nblocks);
  if (ndim == 2)
    return fp32 ? sharp_nd<float, true, 2>(riemann, stage, grid, st, d_grids, mode, dt)
                : sharp_nd<double, false, 2>(riemann, stage, grid, st, d_grids, mode, dt);
  return fp32 ? sharp_nd<float, true, 1>(riemann, stage, grid, st, d_grids, mode, dt)
              : sharp_nd<double, false, 1>(riemann, stage, grid, st, d_grids, mode, dt);
}

}  // namespace claw
