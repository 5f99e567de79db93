// k_split.hip -- dimensionally split classic steps on gfx950.
//
// Method (Section 2.1: the classic algorithms come dimensionally split or
// fully multidimensional): a 2D step is a sequence of 1D wave-propagation
// sweeps (eq. lwflux / eq. fluxdiff along one axis, no transverse terms):
//   Godunov splitting   x over dt, then y over dt;
//   Strang splitting    x over dt/2, y over dt, x over dt/2.
// Each sweep reads one whole state and writes another, so a step costs one
// state read + write per sweep; in exchange a sweep solves Riemann problems
// along one axis only and carries no transverse terms.
//
// x sweep: every row is an independent 1D problem.  One 64-lane wavefront
// owns 60 columns (2 halo lanes a side, x-neighbours by DPP lane shifts) and
// walks a segment of rows; row r+1 is loaded while row r is computed.
//
// y sweep: every column is an independent 1D problem.  One wavefront owns 64
// adjacent columns (one per lane: coalesced rows, no lane traffic and no halo
// lanes) and marches up a segment of rows with the y-faces' waves in
// registers, as in the unsplit kernel:
//   (A) y-face r-1/2 : normal solve between rows r-1 and r
//   (B) y-face r-3/2 : limiter (faces r-5/2 and r-1/2), correction flux
//   (D) row    r-2   : update and store
//
// Courant number of a split step: dt times the running maximum of the sweeps'
// largest |s|/spacing, taken in sweep order and stopped at the first sweep
// whose own value (dt times its speed) exceeds cfl_max or is not finite;
// that sweep rejects the step (or flags it non-physical) and the sweeps
// after it, which act on an unstable intermediate, do not count.  Each
// non-final sweep's last workgroup stores the sweep's maximum in a field of
// its own; the final sweep's last workgroup combines them (host dt: records
// the speed; device controller: decides the step and flips the ping-pong).  The axisymmetric
// source is applied by the final sweep, after the hyperbolic update of the
// cell, over the full dt (a fractional step, as in the unsplit kernel).
#include "dev_common.h"
#include "phys.h"

namespace claw {

// The step's speed from the earlier sweeps' totals (cleared for the next
// step) and the final sweep's own maximum `last`.
__device__ inline double split_speed(Ctrl* c, int nprev, double dt, double cfl_max, double last) {
  CLAW_GLOBAL Ctrl* g = (CLAW_GLOBAL Ctrl*)c;
  double s = 0.0;
  bool open = true;
  for (int k = 0; k < nprev; ++k) {
    const double sk = bitsd(
        __hip_atomic_load(&g->sweep_bits[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    __hip_atomic_store(&g->sweep_bits[k], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (!open) continue;
    s = max_nan(s, sk);
    if (!(dt * sk <= cfl_max)) open = false;
  }
  return open ? max_nan(s, last) : s;
}

// End of a sweep's workgroup: a non-final sweep stores its total in its own
// controller field; the final sweep combines them and closes the step.
__device__ inline void close_sweep(const GridDesc& G, int mode, const SweepArgs& sa, double dt,
                                   double speed) {
  Ctrl* ctrl = G.ctrl;
  const int nprev = sa.index;
  const double cfl_max = G.cfl_max;
  if (!sa.final_sweep) {
    finish_workgroup(ctrl, G.slots, blockIdx.x, sa.nblocks, speed, [=](Ctrl* c, double sp) {
      CLAW_GLOBAL Ctrl* g = (CLAW_GLOBAL Ctrl*)c;
      __hip_atomic_store(&g->sweep_bits[nprev], dbits(sp), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    });
  } else if (mode == kDeviceCtrl) {
    finish_workgroup(ctrl, G.slots, blockIdx.x, sa.nblocks, speed, [=](Ctrl* c, double sp) {
      if (ctrl_decide(c, split_speed(c, nprev, dt, cfl_max, sp))) c->src ^= 1;
    });
  } else {
    finish_workgroup(ctrl, G.slots, blockIdx.x, sa.nblocks, speed, [=](Ctrl* c, double sp) {
      c->last_speed = split_speed(c, nprev, dt, cfl_max, sp);
    });
  }
}

// The cell update (hyperbolic increment `inc`, then the source over the full
// dt on the final sweep), Kahan-compensated in FP32 mode.
template <typename R, class P, bool KAHAN>
__device__ __forceinline__ void sweep_store(const P& phys, const GridDesc& G, bool source,
                                            int row, double dt, const R (&q)[P::M],
                                            R (&inc)[P::M], const R (&cprev)[P::M], gmut<R> qo,
                                            gmut<R> co, size_t plane, size_t off) {
  constexpr int M = P::M;
  if constexpr (P::kSource) {
    if (source) {
      const R ir = (R)(1.0 / (G.ylo + (row + 0.5) * G.dy));
      R qs[4], ds[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) qs[k] = q[k] + inc[k];
      phys.source_increment(qs, ir, (R)dt, ds);
#pragma unroll
      for (int k = 0; k < 4; ++k) inc[k] += ds[k];
    }
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    if constexpr (KAHAN) {
      const R y = inc[k] - cprev[k];
      const R t = q[k] + y;
      co[k * plane + off] = (t - q[k]) - y;
      qo[k * plane + off] = t;
    } else {
      qo[k * plane + off] = q[k] + inc[k];
    }
  }
}

template <typename R, class P, bool KAHAN, int LIM>
__global__ __launch_bounds__(kLanes) void k_sweep_x(const GridDesc* __restrict__ grids, int mode,
                                                    double dt_host, int src_host, SweepArgs sa) {
  constexpr int M = P::M, MW = P::MW, NA = P::NA > 0 ? P::NA : 1;
  constexpr int H = 2, U = kLanes - 2 * H;
  using Face = typename P::Face;
  using Cell = typename P::Cell;
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  double dt;
  int src;
  if (mode == kDeviceCtrl) {
    if (!ctrl->active) return;
    dt = ctrl->dt_try;
    src = ctrl->src;
  } else {
    dt = dt_host;
    src = src_host;
  }
  int strip, seg;
  tile_of(blockIdx.x, sa.strips, sa.segs, G.order, strip, seg);
  const int nx = G.nx, ny = G.ny;
  const size_t plane = (size_t)nx * ny;
  const int lane = threadIdx.x;
  const int i = strip * U - H + lane;
  const bool own = lane >= H && lane < H + U && i < nx;
  const bool own_face = lane >= H && lane <= H + U && i <= nx;
  const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);
  const int j0 = seg_begin(seg, ny, sa.segs);
  const int j1 = seg_begin(seg + 1, ny, sa.segs);
  const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], H);
  const EdgeStates<R, M> es = edge_states<R, M>(G, mx);
  const gconst<R> q = as_gconst<R>(sa.in ? sa.in : G.q[src]);
  const gmut<R> qo = as_gmut<R>(sa.out ? sa.out : G.q[src ^ 1]);
  const gconst<R> aux = as_gconst<R>(G.aux);
  const gconst<R> cin = as_gconst<R>(sa.cin ? sa.cin : G.c[src]);
  const gmut<R> cout = as_gmut<R>(sa.cout ? sa.cout : G.c[src ^ 1]);
  const R dtdx = (R)(sa.frac * dt / G.dx);
  const bool source = sa.final_sweep && G.source;
  const P phys(G);

  R smx = R(0);
  R qc[M], ac[NA], qpre[M], apre[NA];
  {
    const AxisMap my{j0, 0, 0};
    load_state<R, P>(qc, q, plane, nx, mx, my, es);
    load_aux<R, P>(ac, aux, plane, nx, mx, my);
  }
  for (int r = j0; r < j1; ++r) {
    const bool more = r + 1 < j1;
    const AxisMap myn{r + 1, 0, 0};
    if (more) {
      load_raw<R, M>(qpre, q, plane, nx, mx, myn);
      load_aux<R, P>(apre, aux, plane, nx, mx, myn);
    }
    const size_t off = (size_t)r * nx + ic;
    R cprev[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if constexpr (KAHAN) cprev[k] = cin[k * plane + off];
      else cprev[k] = R(0);
    }

    const Cell cc = phys.cell(qc, ac);
    R ql[M];
#pragma unroll
    for (int k = 0; k < M; ++k) ql[k] = shfl_prev(qc[k]);
    R W[MW][M], s[MW], am[M], ap[M];
    Face f{};
    phys.template normal<0>(ql, qc, P::shfl_prev_cell(cc), cc, W, s, am, ap, f);
    R cq[M];
#pragma unroll
    for (int k = 0; k < M; ++k) cq[k] = R(0);
#pragma unroll
    for (int p = 0; p < MW; ++p) {
      R nrm = R(0), dl = R(0);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        if (!P::template nz<0>(p, k)) continue;
        nrm += W[p][k] * W[p][k];
        dl += shfl_prev(W[p][k]) * W[p][k];
      }
      const R dr = shfl_next(dl);   // the right neighbour's dot product with this face
      const R phi = limiter_phi_t<LIM>(s[p] > R(0) ? dl : dr, nrm);
      const R as = rabs(s[p]);
      if (own_face) smx = max_nan(smx, as);
      const R w = as * (R(1) - dtdx * as) * phi;
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (P::template nz<0>(p, k)) cq[k] += w * W[p][k];
    }
    R inc[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
      const R fp = ap[k] - R(0.5) * cq[k];                 // A^+dQ - F~ at i-1/2
      const R fm = shfl_next(am[k] + R(0.5) * cq[k]);      // A^-dQ + F~ at i+1/2
      inc[k] = -(dtdx * (fp + fm));
    }
    if (more) apply_bc<R, P>(qpre, mx, myn, es);
    if (own) sweep_store<R, P, KAHAN>(phys, G, source, r, dt, qc, inc, cprev, qo, cout, plane, off);
    if (more) {
#pragma unroll
      for (int k = 0; k < M; ++k) qc[k] = qpre[k];
#pragma unroll
      for (int k = 0; k < NA; ++k) ac[k] = apre[k];
    }
  }
  close_sweep(G, mode, sa, dt, own_face ? (double)smx / G.dx : 0.0);
}

template <typename R, class P, bool KAHAN, int LIM>
__global__ __launch_bounds__(kLanes) void k_sweep_y(const GridDesc* __restrict__ grids, int mode,
                                                    double dt_host, int src_host, SweepArgs sa) {
  constexpr int M = P::M, MW = P::MW, NA = P::NA > 0 ? P::NA : 1;
  constexpr int H = 2;
  using Face = typename P::Face;
  using Cell = typename P::Cell;
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  double dt;
  int src;
  if (mode == kDeviceCtrl) {
    if (!ctrl->active) return;
    dt = ctrl->dt_try;
    src = ctrl->src;
  } else {
    dt = dt_host;
    src = src_host;
  }
  int strip, seg;
  tile_of(blockIdx.x, sa.strips, sa.segs, G.order, strip, seg);
  const int nx = G.nx, ny = G.ny;
  const size_t plane = (size_t)nx * ny;
  const int i = strip * kLanes + (int)threadIdx.x;
  const bool own = i < nx;
  const int ic = own ? i : nx - 1;                  // lanes past the edge read the last column
  const AxisMap mx{ic, 0, 0};                       // x boundaries play no part in a y sweep
  const int bcy0 = G.bc[2], bcy1 = G.bc[3];
  const int j0 = seg_begin(seg, ny, sa.segs);
  const int j1 = seg_begin(seg + 1, ny, sa.segs);
  const EdgeStates<R, M> es = edge_states<R, M>(G, mx);
  const gconst<R> q = as_gconst<R>(sa.in ? sa.in : G.q[src]);
  const gmut<R> qo = as_gmut<R>(sa.out ? sa.out : G.q[src ^ 1]);
  const gconst<R> aux = as_gconst<R>(G.aux);
  const gconst<R> cin = as_gconst<R>(sa.cin ? sa.cin : G.c[src]);
  const gmut<R> cout = as_gmut<R>(sa.cout ? sa.cout : G.c[src ^ 1]);
  const R dtdy = (R)(sa.frac * dt / G.dy);
  const bool source = sa.final_sweep && G.source;
  const P phys(G);

  R smy = R(0);
  R q0[M], q1[M];                                   // rows r-2, r-1
  Cell c1{};
  R ydl1[MW];                                       // W_p(r-5/2) . W_p(r-3/2)
  R yW1[MW][M], ys1[MW], yam1[M], yap1[M];          // y-face r-3/2
  R glo[M];                                         // B^+dQ - G~ at r-5/2 (for row r-2)
#pragma unroll
  for (int k = 0; k < M; ++k) q0[k] = q1[k] = yam1[k] = yap1[k] = glo[k] = R(0);
#pragma unroll
  for (int p = 0; p < MW; ++p) {
    ydl1[p] = ys1[p] = R(0);
#pragma unroll
    for (int k = 0; k < M; ++k) yW1[p][k] = R(0);
  }
  R qpre[M], apre[NA], qnext[M];
  {
    const AxisMap my = map_axis(j0 - 2, ny, bcy0, bcy1, H);
    load_state<R, P>(qnext, q, plane, nx, mx, my, es);
    load_aux<R, P>(apre, aux, plane, nx, mx, my);
  }
  // rows j0-2 .. j0+1 fill the pipeline; j0+2 .. j1 are steady; j1+1 drains
  for (int r = j0 - 2; r <= j1 + 1; ++r) {
    const bool st_a = r >= j0 - 1, sb = r >= j0 + 1, sd = r >= j0 + 2, sload = r + 1 <= j1 + 1;
    R qn[M], an[NA];
#pragma unroll
    for (int k = 0; k < M; ++k) qn[k] = qnext[k];
#pragma unroll
    for (int k = 0; k < NA; ++k) an[k] = apre[k];
    AxisMap mynext{0, 0, 0};
    if (sload) {
      mynext = map_axis(r + 1, ny, bcy0, bcy1, H);
      load_raw<R, M>(qpre, q, plane, nx, mx, mynext);
      load_aux<R, P>(apre, aux, plane, nx, mx, mynext);
    }
    R cprev[M];
    const size_t off = (size_t)(r - 2) * nx + ic;   // row r-2 (used only when sd)
#pragma unroll
    for (int k = 0; k < M; ++k) {
      if constexpr (KAHAN) cprev[k] = sd ? cin[k * plane + off] : R(0);
      else cprev[k] = R(0);
    }
    const Cell cn = phys.cell(qn, an);

    // (A) y-face r-1/2
    R yW2[MW][M], ys2[MW], yam2[M], yap2[M];
    if (st_a) {
      Face yf2{};
      phys.template normal<1>(q1, qn, c1, cn, yW2, ys2, yam2, yap2, yf2);
    } else {
#pragma unroll
      for (int p = 0; p < MW; ++p) {
        ys2[p] = R(0);
#pragma unroll
        for (int k = 0; k < M; ++k) yW2[p][k] = R(0);
      }
#pragma unroll
      for (int k = 0; k < M; ++k) yam2[k] = yap2[k] = R(0);
    }
    R ydl2[MW];
#pragma unroll
    for (int p = 0; p < MW; ++p) {
      R d = R(0);
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (P::template nz<1>(p, k)) d += yW1[p][k] * yW2[p][k];
      ydl2[p] = d;
    }

    // (B) y-face r-3/2: limiter and correction flux
    R ghi[M], glo_n[M];
#pragma unroll
    for (int k = 0; k < M; ++k) ghi[k] = glo_n[k] = R(0);
    if (sb) {
      R cq[M];
#pragma unroll
      for (int k = 0; k < M; ++k) cq[k] = R(0);
#pragma unroll
      for (int p = 0; p < MW; ++p) {
        R nrm = R(0);
#pragma unroll
        for (int k = 0; k < M; ++k)
          if (P::template nz<1>(p, k)) nrm += yW1[p][k] * yW1[p][k];
        const R phi = limiter_phi_t<LIM>(ys1[p] > R(0) ? ydl1[p] : ydl2[p], nrm);
        const R as = rabs(ys1[p]);
        if (own) smy = max_nan(smy, as);
        const R w = as * (R(1) - dtdy * as) * phi;
#pragma unroll
        for (int k = 0; k < M; ++k)
          if (P::template nz<1>(p, k)) cq[k] += w * yW1[p][k];
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        ghi[k] = yam1[k] + R(0.5) * cq[k];     // B^-dQ + G~ at r-3/2 (for row r-2)
        glo_n[k] = yap1[k] - R(0.5) * cq[k];   // B^+dQ - G~ at r-3/2 (for row r-1)
      }
    }

    if (sload) {
#pragma unroll
      for (int k = 0; k < M; ++k) qnext[k] = qpre[k];
      apply_bc<R, P>(qnext, mx, mynext, es);
    }

    // (D) row r-2 is complete
    if (sd && own) {
      R inc[M];
#pragma unroll
      for (int k = 0; k < M; ++k) inc[k] = -(dtdy * (glo[k] + ghi[k]));
      sweep_store<R, P, KAHAN>(phys, G, source, r - 2, dt, q0, inc, cprev, qo, cout, plane, off);
    }

    // rotate
#pragma unroll
    for (int k = 0; k < M; ++k) {
      q0[k] = q1[k];
      q1[k] = qn[k];
      yam1[k] = yam2[k];
      yap1[k] = yap2[k];
      glo[k] = glo_n[k];
    }
    c1 = cn;
#pragma unroll
    for (int p = 0; p < MW; ++p) {
      ys1[p] = ys2[p];
      ydl1[p] = ydl2[p];
#pragma unroll
      for (int k = 0; k < M; ++k) yW1[p][k] = yW2[p][k];
    }
  }
  close_sweep(G, mode, sa, dt, own ? (double)smy / G.dy : 0.0);
}

// ---------------------------------------------------------------------------
// Host-side launcher (dispatch on axis, solver, limiter and precision).
// ---------------------------------------------------------------------------
template <typename R, bool K, int LIM, class P>
static void launch_sweep_p(int dir, hipStream_t st, const GridDesc* g, int mode, double dt,
                           int src, const SweepArgs& sa) {
  if (dir == 0)
    hipLaunchKernelGGL((k_sweep_x<R, P, K, LIM>), dim3(sa.nblocks), dim3(kLanes), 0, st, g, mode,
                       dt, src, sa);
  else
    hipLaunchKernelGGL((k_sweep_y<R, P, K, LIM>), dim3(sa.nblocks), dim3(kLanes), 0, st, g, mode,
                       dt, src, sa);
}

template <typename R, bool K, int LIM>
static hipError_t launch_sweep_l(int dir, int riemann, hipStream_t st, const GridDesc* g, int mode,
                                 double dt, int src, const SweepArgs& sa) {
  switch (riemann) {
    case 1: launch_sweep_p<R, K, LIM, Advection<R, 2>>(dir, st, g, mode, dt, src, sa); break;
    case 2: launch_sweep_p<R, K, LIM, ShallowWater<R, 2>>(dir, st, g, mode, dt, src, sa); break;
    case 4: launch_sweep_p<R, K, LIM, Elastic<R>>(dir, st, g, mode, dt, src, sa); break;
    case 5: launch_sweep_p<R, K, LIM, EulerRoe<R, 2, false>>(dir, st, g, mode, dt, src, sa); break;
    case 6: launch_sweep_p<R, K, LIM, EulerRoe<R, 2, true>>(dir, st, g, mode, dt, src, sa); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R, bool K>
static hipError_t launch_sweep_t(int dir, int riemann, int lim, hipStream_t st, const GridDesc* g,
                                 int mode, double dt, int src, const SweepArgs& sa) {
  switch (lim) {
    case 0: return launch_sweep_l<R, K, 0>(dir, riemann, st, g, mode, dt, src, sa);
    case 1: return launch_sweep_l<R, K, 1>(dir, riemann, st, g, mode, dt, src, sa);
    case 2: return launch_sweep_l<R, K, 2>(dir, riemann, st, g, mode, dt, src, sa);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep(int dir, int riemann, int fp32, int lim, hipStream_t st,
                        const GridDesc* d_grid, int mode, double dt, int src,
                        const SweepArgs& sa) {
  if (sa.nblocks < 1 || sa.strips < 1 || sa.segs < 1) return hipErrorInvalidValue;
  return fp32 ? launch_sweep_t<float, true>(dir, riemann, lim, st, d_grid, mode, dt, src, sa)
              : launch_sweep_t<double, false>(dir, riemann, lim, st, d_grid, mode, dt, src, sa);
}

}  // namespace claw
