// k_sharp.h -- the SharpClaw step on gfx950: WENO edge values (any odd order
// from 5 to 17), interface flux, flux differencing, and the stage
// combinations of SSP Runge-Kutta integrators (Section 2: method of lines
// with WENO reconstruction; Section 2.1: SSP Runge-Kutta in time, normal
// Riemann problems only in multi-D).
//
// One launch per Runge-Kutta stage.  Every stage of both integrators has the
// form
//   y    = S + gamma dt L(S),   L(S) = -(F_{i+1/2}-F_{i-1/2})/dx - (G_{j+1/2}-G_{j-1/2})/dy
//   PLAIN    out1 = y
//   COMBINE  out1 = a1 P1 + b1 y        (and, if out2 is set, out2 = a2 P1 + b2 y)
//   FINAL    Q    = a1 P1 + b1 y        in place; FP32 mode adds the increment
//                                        a1 (P1 - w Q) + b1 ((S - Q) + gamma dt L), w = (1-b1)/a1,
//                                        to Q with Kahan compensation
// with S the stage input and P1 a pointwise input (Q^n or a stored register):
//   SSPRK(3,3): Q -> S1 (PLAIN, gamma 1); S1 -> S2 = 3/4 Q + 1/4 y;
//               S2 -> Q = 1/3 Q + 2/3 y.
//   SSPRK(10,4), two registers: stages 1-4 and 6-9 PLAIN with gamma 1/6
//               (ping-pong S1/S2); stage 5 COMBINE: S3 = Q/25 + 9/25 y and
//               S1 = 3/5 Q + 2/5 y; stage 10 FINAL: Q = S3 + 3/5 y.
//               (The published form updates the register as 15 S3 - 5 y; that
//               is the same value in exact arithmetic, but the cancellation
//               amplifies the FP32 rounding of S3 about twentyfold.)
// The first stage of an attempt measures the Courant number (speeds at Q^n)
// and, in device-controller mode, decides the attempt.
//
// 2D layout: one wavefront per strip of 64 - 2r columns (r halo lanes each
// side for WENO of order 2r - 1) marching up a segment of rows; the y-stencil
// lives in a (2r-1)-row register window and each y-face flux is computed once
// and carried to the next row.
//
// The kernels of each WENO order are instantiated in a translation unit of
// their own (k_sharp.hip: orders 5 and 7; k_sharp_weno<order>.hip: 9 to 17),
// so that the orders compile in parallel.
#pragma once

#include "dev_common.h"
#include "phys.h"
#include "weno_coeffs.h"

namespace claw {

// WENO edge values of the centre cell of the window v[0 .. 2r-2]: qL at its
// right edge (left state of face i+1/2), qR at its left edge (right state of
// face i-1/2).  r = 3 uses the closed form, others the generated tables.
template <int RH, typename R>
__device__ __forceinline__ void weno_edges(const R (&v)[2 * RH - 1], R eps, R& qL, R& qR) {
  if constexpr (RH == 3) {
    weno5_edges(v[0], v[1], v[2], v[3], v[4], eps, qL, qR);
  } else {
    using C = WenoCoeffs<RH>;
    R pR[RH], pL[RH], D[RH];
    // The indicator rows have zero sum, so they act on differences from the
    // centre value: those are small where the data are smooth and, unlike
    // the values themselves, carry no offset whose rounding the rows'
    // large coefficients (up to several hundred at order 17) would amplify
    // into beta.
    R dv[2 * RH - 1];
#pragma unroll
    for (int j = 0; j < 2 * RH - 1; ++j) dv[j] = v[j] - v[RH - 1];
#pragma unroll
    for (int k = 0; k < RH; ++k) {
      R a = R(0), b = R(0), beta = R(0);
#pragma unroll
      for (int j = 0; j < RH; ++j) {
        a += R(C::cR[k][j]) * v[k + j];
        b += R(C::cL[k][j]) * v[k + j];
      }
#pragma unroll
      for (int i = 0; i < RH - 1; ++i) {
        R t = R(0);
#pragma unroll
        for (int j = 0; j < RH; ++j)
          if (C::sv[k][i][j] != 0.0 && k + j != RH - 1) t += R(C::sv[k][i][j]) * dv[k + j];
        beta += R(C::lam[k][i]) * t * t;
      }
      const R e = eps + beta;
      D[k] = e * e;
      pR[k] = a;
      pL[k] = b;
    }
    R sR = R(0), sL = R(0), nR = R(0), nL = R(0);
    if constexpr (sizeof(R) == 8 && RH <= 4) {
      // weights d_k / D_k normalised: multiply through by prod_j D_j, so
      // alpha_k ~ d_k prod_{j != k} D_j and one reciprocal per edge
      R P[RH];
      R pre = R(1);
#pragma unroll
      for (int k = 0; k < RH; ++k) { P[k] = pre; pre *= D[k]; }
      R suf = R(1);
#pragma unroll
      for (int k = RH - 1; k >= 0; --k) { P[k] *= suf; suf *= D[k]; }
#pragma unroll
      for (int k = 0; k < RH; ++k) {
        const R aR = R(C::d[k]) * P[k], aL = R(C::d[RH - 1 - k]) * P[k];
        sR += aR; nR += aR * pR[k];
        sL += aL; nL += aL * pL[k];
      }
    } else {
      // FP32, and orders above 7: a product of many D_k could leave the
      // exponent range; one reciprocal each
#pragma unroll
      for (int k = 0; k < RH; ++k) {
        const R iD = frcp(D[k]);
        const R aR = R(C::d[k]) * iD, aL = R(C::d[RH - 1 - k]) * iD;
        sR += aR; nR += aR * pR[k];
        sL += aL; nL += aL * pL[k];
      }
    }
    qL = nR * frcp(sR);
    qR = nL * frcp(sL);
  }
}

// Interface flux of a face whose two cells have aux fields al / ar (used by
// policies with a spatially varying flux).
template <int D, class P, typename R>
__device__ __forceinline__ R face_flux(const P& phys, const R* ql, const R* qr, const R* al,
                                       const R* ar, R* F) {
  if constexpr (P::NA > 0) return phys.template flux<D>(ql, qr, al, ar, F);
  else return phys.template flux<D>(ql, qr, F);
}

// Stage output for one cell.  S: stage input value, L: operator value,
// pp: pointwise P1, pq: Q^n (FINAL, FP32), pc: compensation (FINAL, FP32).
template <typename R, class P, int KIND, bool KAHAN>
__device__ __forceinline__ void stage_store(const StageArgs& sa, gmut<R> O1, gmut<R> O2, gmut<R> C,
                                            size_t idx, size_t plane, const R (&S)[P::M],
                                            const R (&L)[P::M], R gdt, R a1, R b1, R a2, R b2, R w,
                                            const R (&pp)[P::M], const R (&pq)[P::M],
                                            const R (&pc)[P::M]) {
  constexpr int M = P::M;
  if constexpr (KIND == kStagePlain) {
#pragma unroll
    for (int k = 0; k < M; ++k) O1[k * plane + idx] = S[k] + gdt * L[k];
  } else if constexpr (KIND == kStageCombine) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const R y = S[k] + gdt * L[k];
      const R t = a1 * pp[k] + b1 * y;
      O1[k * plane + idx] = t;
      if (sa.out2) O2[k * plane + idx] = a2 * pp[k] + b2 * y;
    }
  } else {
    if constexpr (KAHAN) {
      const bool p1q = KIND == kStageFinalQ || sa.p1_is_q;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const R q = pq[k];
        const R inc = (p1q ? R(0) : a1 * (pp[k] - w * q)) + b1 * ((S[k] - q) + gdt * L[k]);
        const R y = inc - pc[k];
        const R t = q + y;
        C[k * plane + idx] = (t - q) - y;
        O1[k * plane + idx] = t;
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) O1[k * plane + idx] = a1 * pp[k] + b1 * (S[k] + gdt * L[k]);
    }
  }
}

// Common prologue: dt of this stage, or an early exit.
__device__ __forceinline__ bool stage_dt(Ctrl* ctrl, int mode, double dt_host, int first,
                                         double& dt) {
  if (mode == kDeviceCtrl) {
    if (first) {
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

__device__ __forceinline__ void stage_finish(const GridDesc& G, int mode, int first,
                                             double speed) {
  if (!first) return;
  Ctrl* ctrl = G.ctrl;
  const int b = blockIdx.x, nblocks = G.nblocks;
  if (mode == kDeviceCtrl) {
    finish_workgroup(ctrl, G.slots, b, nblocks, speed, [](Ctrl* c, double sp) {
      const double d = c->dt_try;
      c->ok = ctrl_decide(c, sp) ? 1 : 0;
      c->dt_stage = d;
    });
  } else {
    finish_workgroup(ctrl, G.slots, b, nblocks, speed,
                     [](Ctrl* c, double sp) { c->last_speed = sp; });
  }
}

// FP32 WENO5 keeps the stencil's rows in an LDS ring instead of registers:
// row r enters slot r mod 5 (boundary conditions applied) over the row that
// left the window, the y stencil reads the five rows of its own column and
// the x stencil the four neighbouring columns of the row being finalised.
// The window then costs no row-to-row moves and x-neighbours no lane shifts
// (FP32 stage 59 against 62 us at 2048x1024).  FP64 keeps the register window:
// there the ring saved no time at two waves per SIMD, and the register budget
// of three waves (168) made the compiler spill (stage 160 us).
template <typename R, int RH> struct UseRing {
  static constexpr bool value = RH == 3 && sizeof(R) == 4;
};

// The ring of one wave: rows x components x 64 lanes, padded by two elements
// at each end so that reads at lane +-2 of any row stay inside the array (the
// edge lanes that read a neighbouring row's or the padding's values are halo
// lanes whose results are discarded).
template <typename R, int M, int NW>
struct Ring {
  R v[2 + NW * M * kLanes + 2];
  __device__ __forceinline__ R& at(int slot, int k, int lane) {
    return v[2 + (slot * M + k) * kLanes + lane];
  }
};

// Waves per SIMD the 2D stage kernel is built for: the FP32 WENO5 kernels
// (window in LDS) fit four in 128 registers, and every stage must, or the
// one tiling shared by the stages leaves a partial second round of waves
// in the stage that fits fewer (the compensated final stage needed 136).
template <typename R, int RH>
constexpr int sharp2d_waves_per_simd() {
  return UseRing<R, RH>::value ? 4 : 1;
}

template <typename R, class P, int RH, int KIND, bool KAHAN>
__global__ __launch_bounds__(kLanes) __attribute__((amdgpu_waves_per_eu(
    sharp2d_waves_per_simd<R, RH>()))) void k_sharp2d(const GridDesc* __restrict__ grids, int mode,
                                                      double dt_host, StageArgs sa) {
  constexpr int M = P::M, NW = 2 * RH - 1;
  constexpr int H = RH, U = kLanes - 2 * H;
  constexpr bool kRing = UseRing<R, RH>::value;
  __shared__ Ring<R, M, kRing ? NW : 1> ring;
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  double dtd;
  if (!stage_dt(ctrl, mode, dt_host, sa.first, dtd)) return;
  const R gdt = (R)(sa.gamma * dtd);
  const R a1 = (R)sa.a1, b1 = (R)sa.b1, a2 = (R)sa.a2, b2 = (R)sa.b2, wq = (R)sa.w;
  int strip, seg;
  tile_of(blockIdx.x, G.strips, G.segs, G.order, strip, seg);
  const int nx = G.nx, ny = G.ny;
  const size_t plane = (size_t)nx * ny;
  const int lane = threadIdx.x;
  const int i = strip * U - H + lane;
  const bool own = lane >= H && lane < H + U && i < nx;
  const bool own_face = lane >= H && lane <= H + U && i <= nx;
  const int j0 = seg_begin(seg, ny, G.segs);
  const int j1 = seg_begin(seg + 1, ny, G.segs);
  const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], H);
  const int bcy0 = G.bc[2], bcy1 = G.bc[3];
  const EdgeStates<R, M> es = edge_states<R, M>(G, mx);
  const gconst<R> S = as_gconst<R>(sa.in);
  const R eps = (R)G.weno_eps;
  const R rdx = (R)(1.0 / G.dx), rdy = (R)(1.0 / G.dy);
  const P phys(G);
  R smx = R(0), smy = R(0);
  // aux fields (material) of window rows c-1, c (the centre) and c+1 (read a
  // row ahead)
  constexpr int NA = P::NA > 0 ? P::NA : 1;
  const gconst<R> aux = as_gconst<R>(G.aux);
  R aP[NA], aC[NA], aN[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) aP[k] = aC[k] = aN[k] = R(0);
  if constexpr (P::NA > 0) {
    load_aux<R, P>(aC, aux, plane, nx, mx, map_axis(j0 - 2 * RH, ny, bcy0, bcy1, H));
    load_aux<R, P>(aN, aux, plane, nx, mx, map_axis(j0 - 2 * RH + 1, ny, bcy0, bcy1, H));
  }

  constexpr int NWR = kRing ? 1 : NW;
  R w[NWR][M];         // register window: rows r-NW+1 .. r
  R qyl_prev[M], g_lo[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    qyl_prev[k] = g_lo[k] = R(0);
#pragma unroll
    for (int s = 0; s < NWR; ++s) w[s][k] = R(0);
  }
  int slot = 0;        // ring slot of row r
  const gconst<R> P1 = as_gconst<R>(sa.p1);
  const gconst<R> Qn = as_gconst<R>(G.q[0]);
  const gconst<R> Cn = as_gconst<R>(G.c[0]);
  const gmut<R> O1 = as_gmut<R>(sa.out1);
  const gmut<R> O2 = as_gmut<R>(sa.out2);
  const gmut<R> Cout = as_gmut<R>(G.c[0]);
  constexpr bool kPoint = KIND != kStagePlain;
  constexpr bool kQ = KIND >= kStageFinal && KAHAN;
  // Row r+1 is loaded while row r is processed (software pipelining) and
  // enters the window with its boundary conditions applied at the end of
  // the iteration (the wait for the load then comes a row of work after it
  // was issued).  The finished row is stored where it is computed, so its
  // results are not carried to the end of the iteration.  The pointwise
  // inputs of the row finalised next iteration are read ahead too.
  R pre[M], nxt[M], pp[M], pq[M], pc[M], up[M], uq[M], uc[M];
  load_state<R, P>(nxt, S, plane, nx, mx, map_axis(j0 - RH, ny, bcy0, bcy1, H), es);
#pragma unroll
  for (int k = 0; k < M; ++k) pp[k] = pq[k] = pc[k] = up[k] = uq[k] = uc[k] = R(0);
  const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);   // clamped column for pointwise reads
  for (int r = j0 - RH; r <= j1 + RH - 1; ++r) {
#pragma unroll
    for (int k = 0; k < M; ++k) { up[k] = pp[k]; uq[k] = pq[k]; uc[k] = pc[k]; }
    if constexpr (kRing) {
      // row r replaces row r - NW in the ring; the barriers keep the other
      // lanes' reads of the old row before, and their reads of row r after
      __syncthreads();
#pragma unroll
      for (int k = 0; k < M; ++k) ring.at(slot, k, lane) = nxt[k];
      __syncthreads();
    } else {
#pragma unroll
      for (int s = 0; s < NW - 1; ++s)
#pragma unroll
        for (int k = 0; k < M; ++k) w[s][k] = w[s + 1][k];
#pragma unroll
      for (int k = 0; k < M; ++k) w[NW - 1][k] = nxt[k];
    }
    // ring slot of window row s (0 = oldest, NW - 1 = row r)
    auto wslot = [&](int s_) { const int t = slot + 1 + s_; return t >= NW ? t - NW : t; };
    const bool more = r + 1 <= j1 + RH - 1;
    AxisMap mynext{0, 0, 0};
    if (more) {
      mynext = map_axis(r + 1, ny, bcy0, bcy1, H);
      load_raw<R, M>(pre, S, plane, nx, mx, mynext);
    }
    if constexpr (P::NA > 0) {
#pragma unroll
      for (int k = 0; k < NA; ++k) { aP[k] = aC[k]; aC[k] = aN[k]; }
      load_aux<R, P>(aN, aux, plane, nx, mx, map_axis(r - RH + 2, ny, bcy0, bcy1, H));
    }
    const int fn = r + 1 - RH;   // row finalised next iteration
    if (kPoint && fn >= j0 && fn < j1) {
      const size_t idx = (size_t)fn * nx + ic;
#pragma unroll
      for (int k = 0; k < M; ++k) {
        if constexpr (KIND == kStageFinalQ) {
          pq[k] = Qn[k * plane + idx];
        } else {
          pp[k] = P1[k * plane + idx];
          if constexpr (kQ) pq[k] = sa.p1_is_q ? pp[k] : Qn[k * plane + idx];
        }
        if constexpr (kQ) pc[k] = Cn[k * plane + idx];
      }
    }
    if (r >= j0 + RH - 2) {
      // y edge values of the window's centre row c = r - RH + 1
      R qyl[M], qyr[M];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        R col[NW];
#pragma unroll
        for (int s = 0; s < NW; ++s) {
          if constexpr (kRing) col[s] = ring.at(wslot(s), k, lane);
          else col[s] = w[s][k];
        }
        weno_edges<RH>(col, eps, qyl[k], qyr[k]);
      }
      if (r >= j0 + RH - 1) {
        // y-face flux at c-1/2
        R g_up[M];
        const R sy = face_flux<1>(phys, qyl_prev, qyr, aP, aC, g_up);
        smy = max_nan(smy, sy);
        if (r >= j0 + RH) {
          // row f = c-1 (window row RH-2) is complete: x edge values, x-face fluxes
          R xl[M], xr[M];
          R Sf[M];
#pragma unroll
          for (int k = 0; k < M; ++k) {
            if constexpr (!kRing && RH == 3) {
              // each lane forms one first difference, v(i+1) - v(i); the
              // others are its neighbours' (the same subtraction of the same
              // values), so four lane shifts and one subtraction per component
              const R v0 = w[RH - 2][k];
              const R dc = shfl_next(v0) - v0;
              const R db = shfl_prev(dc);
              weno5_edges_d(v0, shfl_prev(db), db, dc, shfl_next(dc), eps, xl[k], xr[k]);
              Sf[k] = v0;
            } else {
              R row[NW];
              if constexpr (kRing) {
                const int fs = wslot(RH - 2);
#pragma unroll
                for (int s = 0; s < NW; ++s) row[s] = ring.at(fs, k, lane - (RH - 1) + s);
              } else {
                row[RH - 1] = w[RH - 2][k];
#pragma unroll
                for (int s = 1; s < RH; ++s) {
                  row[RH - 1 - s] = shfl_prev(row[RH - s]);
                  row[RH - 1 + s] = shfl_next(row[RH - 2 + s]);
                }
              }
              Sf[k] = row[RH - 1];
              weno_edges<RH>(row, eps, xl[k], xr[k]);
            }
          }
          R ql[M], F[M], al[NA], Lv[M];
#pragma unroll
          for (int k = 0; k < M; ++k) ql[k] = shfl_prev(xl[k]);
#pragma unroll
          for (int k = 0; k < NA; ++k) al[k] = P::NA > 0 ? shfl_prev(aP[k]) : R(0);
          const R sx = face_flux<0>(phys, ql, xr, al, aP, F);
          if (own_face) smx = max_nan(smx, sx);
#pragma unroll
          for (int k = 0; k < M; ++k) {
            const R Fr = shfl_next(F[k]);
            Lv[k] = -(Fr - F[k]) * rdx - (g_up[k] - g_lo[k]) * rdy;
          }
          if (own)
            stage_store<R, P, KIND, KAHAN>(sa, O1, O2, Cout, (size_t)(r - RH) * nx + i, plane, Sf,
                                           Lv, gdt, a1, b1, a2, b2, wq, up, uq, uc);
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
    slot = slot + 1 == NW ? 0 : slot + 1;
  }
  const double speed = own ? max_nan((double)smx * (1.0 / G.dx), (double)smy * (1.0 / G.dy))
                           : (own_face ? (double)smx * (1.0 / G.dx) : 0.0);
  stage_finish(G, mode, sa.first, speed);
}

template <typename R, class P, int RH, int KIND, bool KAHAN>
__global__ __launch_bounds__(kLanes) void k_sharp1d(const GridDesc* __restrict__ grids, int mode,
                                                    double dt_host, StageArgs sa) {
  constexpr int M = P::M, NW = 2 * RH - 1;
  constexpr int H = RH, U = kLanes - 2 * H;
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  double dtd;
  if (!stage_dt(ctrl, mode, dt_host, sa.first, dtd)) return;
  const R gdt = (R)(sa.gamma * dtd);
  const int nx = G.nx;
  const int lane = threadIdx.x;
  const int i = blockIdx.x * U - H + lane;
  const bool own = lane >= H && lane < H + U && i < nx;
  const bool own_face = lane >= H && lane <= H + U && i <= nx;
  const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], H);
  const AxisMap my{0, 0, 0};
  const gconst<R> S = as_gconst<R>(sa.in);
  const R eps = (R)G.weno_eps;
  const R rdx = (R)(1.0 / G.dx);
  const P phys(G);
  R c[M], xl[M], xr[M];
  load_state<R, P>(c, S, (size_t)nx, nx, mx, my, edge_states<R, M>(G, mx));
  constexpr int NA = P::NA > 0 ? P::NA : 1;
  R ac[NA], al[NA];
  load_aux<R, P>(ac, as_gconst<R>(G.aux), (size_t)nx, nx, mx, my);
#pragma unroll
  for (int k = 0; k < NA; ++k) al[k] = P::NA > 0 ? shfl_prev(ac[k]) : R(0);
#pragma unroll
  for (int k = 0; k < M; ++k) {
    R row[NW];
    row[RH - 1] = c[k];
#pragma unroll
    for (int s = 1; s < RH; ++s) {
      row[RH - 1 - s] = shfl_prev(row[RH - s]);
      row[RH - 1 + s] = shfl_next(row[RH - 2 + s]);
    }
    weno_edges<RH>(row, eps, xl[k], xr[k]);
  }
  R ql[M], F[M], Lv[M];
#pragma unroll
  for (int k = 0; k < M; ++k) ql[k] = shfl_prev(xl[k]);
  const R sx = face_flux<0>(phys, ql, xr, al, ac, F);
#pragma unroll
  for (int k = 0; k < M; ++k) Lv[k] = -(shfl_next(F[k]) - F[k]) * rdx;
  R pp[M], pq[M], pc[M];
  const size_t ic = (size_t)(i < 0 ? 0 : (i >= nx ? nx - 1 : i));
#pragma unroll
  for (int k = 0; k < M; ++k) {
    pp[k] = KIND != kStagePlain ? as_gconst<R>(sa.p1)[k * (size_t)nx + ic] : R(0);
    pq[k] = (KIND == kStageFinal && KAHAN && !sa.p1_is_q) ? as_gconst<R>(G.q[0])[k * (size_t)nx + ic]
                                                          : pp[k];
    pc[k] = (KIND == kStageFinal && KAHAN) ? as_gconst<R>(G.c[0])[k * (size_t)nx + ic] : R(0);
  }
  if (own)
    stage_store<R, P, KIND, KAHAN>(sa, as_gmut<R>(sa.out1), as_gmut<R>(sa.out2),
                                   as_gmut<R>(G.c[0]), (size_t)i, (size_t)nx, c, Lv, gdt,
                                   (R)sa.a1, (R)sa.b1, (R)sa.a2, (R)sa.b2, (R)sa.w, pp, pq, pc);
  const double speed = own_face ? (double)sx * (1.0 / G.dx) : 0.0;
  stage_finish(G, mode, sa.first, speed);
}

// ---------------------------------------------------------------------------
// Launchers.
// ---------------------------------------------------------------------------
template <typename R, bool K, int NDIM, int RH, int KIND>
static hipError_t sharp_t(int riemann, dim3 grid, hipStream_t st, const GridDesc* g, int mode,
                          double dt, const StageArgs& sa) {
  if (NDIM == 2) {
    switch (riemann) {
      case 1:
        hipLaunchKernelGGL((k_sharp2d<R, AdvectionFlux<R, 2>, RH, KIND, K>), grid, dim3(kLanes), 0,
                           st, g, mode, dt, sa);
        break;
      case 3:
        hipLaunchKernelGGL((k_sharp2d<R, EulerHLLE<R, 2>, RH, KIND, K>), grid, dim3(kLanes), 0, st,
                           g, mode, dt, sa);
        break;
      case 7:
        hipLaunchKernelGGL((k_sharp2d<R, PSystem<R, 2>, RH, KIND, K>), grid, dim3(kLanes), 0, st,
                           g, mode, dt, sa);
        break;
      default: return hipErrorInvalidValue;
    }
  } else {
    switch (riemann) {
      case 1:
        hipLaunchKernelGGL((k_sharp1d<R, AdvectionFlux<R, 1>, RH, KIND, K>), grid, dim3(kLanes), 0,
                           st, g, mode, dt, sa);
        break;
      case 3:
        hipLaunchKernelGGL((k_sharp1d<R, EulerHLLE<R, 1>, RH, KIND, K>), grid, dim3(kLanes), 0, st,
                           g, mode, dt, sa);
        break;
      case 7:
        hipLaunchKernelGGL((k_sharp1d<R, PSystem<R, 1>, RH, KIND, K>), grid, dim3(kLanes), 0, st,
                           g, mode, dt, sa);
        break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename R, bool K, int NDIM, int RH>
static hipError_t sharp_kind(int riemann, int kind, dim3 grid, hipStream_t st, const GridDesc* g,
                             int mode, double dt, const StageArgs& sa) {
  switch (kind) {
    case kStagePlain: return sharp_t<R, K, NDIM, RH, kStagePlain>(riemann, grid, st, g, mode, dt, sa);
    case kStageCombine:
      return sharp_t<R, K, NDIM, RH, kStageCombine>(riemann, grid, st, g, mode, dt, sa);
    case kStageFinal:
      if constexpr (K && NDIM == 2 && RH == 3) {
        if (sa.p1_is_q)
          return sharp_t<R, K, NDIM, RH, kStageFinalQ>(riemann, grid, st, g, mode, dt, sa);
      }
      return sharp_t<R, K, NDIM, RH, kStageFinal>(riemann, grid, st, g, mode, dt, sa);
  }
  return hipErrorInvalidValue;
}

template <int RH>
hipError_t launch_sharp_order(int ndim, int riemann, int fp32, int kind, dim3 grid, hipStream_t st,
                              const GridDesc* g, int mode, double dt, const StageArgs& sa) {
  if (ndim == 2)
    return fp32 ? sharp_kind<float, true, 2, RH>(riemann, kind, grid, st, g, mode, dt, sa)
                : sharp_kind<double, false, 2, RH>(riemann, kind, grid, st, g, mode, dt, sa);
  return fp32 ? sharp_kind<float, true, 1, RH>(riemann, kind, grid, st, g, mode, dt, sa)
              : sharp_kind<double, false, 1, RH>(riemann, kind, grid, st, g, mode, dt, sa);
}

// Orders 9-17: instantiated in k_sharp_weno<order>.hip.
#define CLAW_SHARP_ORDER_DECL(RH)                                                              \
  extern template hipError_t launch_sharp_order<RH>(int, int, int, int, dim3, hipStream_t,   \
                                                    const GridDesc*, int, double,             \
                                                    const StageArgs&);
CLAW_SHARP_ORDER_DECL(5)
CLAW_SHARP_ORDER_DECL(6)
CLAW_SHARP_ORDER_DECL(7)
CLAW_SHARP_ORDER_DECL(8)
CLAW_SHARP_ORDER_DECL(9)
#undef CLAW_SHARP_ORDER_DECL

}  // namespace claw
