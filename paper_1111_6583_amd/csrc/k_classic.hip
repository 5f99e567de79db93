// k_classic.hip -- the Clawpack wave-propagation step on gfx950.
//
// Method (Section 2, eq. lwflux / eq. fluxdiff; Section 2.1, transverse
// corrections of the unsplit 2D algorithm; LeVeque 1997):
//   per interface: Riemann solve -> waves W^p, speeds s^p, fluctuations A^-dQ, A^+dQ;
//   limited waves  W~ = phi(theta) W, theta from the upwind neighbour's wave;
//   correction     F~ = 1/2 sum_p |s|(1 - dt/dx |s|) W~^p;
//   2D transverse: split A^-dQ + cq, A^+dQ - cq (mode 2; A^-/+ dQ in mode 1)
//                  with the transverse solver and add -dt/(2dx) B^-/+ (...) to
//                  the correction fluxes of the four neighbouring faces;
//   update         Q -= dt/dx (A^+dQ_{i-1/2} + A^-dQ_{i+1/2} + F~_{i+1/2} - F~_{i-1/2})
//                     + the same in y.
//
// 2D layout of the work ("marching"): one 64-lane wavefront per workgroup
// owns a strip of 60 columns (2 halo lanes each side) and marches up a
// segment of rows.  x-neighbours are adjacent lanes (shuffles); everything
// along y stays in registers from one row to the next, so each interface's
// Riemann problem is solved once per strip, there is no LDS traffic and no
// barrier.  Rows are read once per segment plus 4 halo rows.
//
// Pipeline when row r has just been loaded:
//   (A) y-face r-1/2 : normal solve between rows r-1 and r
//   (B) y-face r-3/2 : limit (needs faces r-5/2 and r-1/2), correction flux,
//                      transverse split of its fluctuations into the x-faces
//                      of cells (i, r-1) and (i, r-2)
//   (C) x-row  r-1   : normal solves, limiting across lanes, correction flux,
//                      transverse split into the y-faces of row r-1
//   (D) row    r-2   : complete -> update and store
#include <type_traits>

#include "dev_common.h"
#include "phys.h"

namespace claw {

// Rows read ahead by the 2D marching kernel: 1, or 2 (two row buffers used
// alternately; the loop body is instantiated for both buffer phases, so no
// buffer is copied while its loads are in flight).  Measured on MI355X:
// two rows ahead take 8-12% off the elasticity step (the kernel that waits on
// memory most), 7% off FP32 shallow water and 7% off the Euler step with a
// tracer (one wave per SIMD: nothing else hides its loads); the FP64
// shallow-water step is as fast or faster with one (more code, same
// occupancy).
template <typename R, class P>
constexpr int classic_prefetch() {
  return (std::is_same<P, Elastic<R>>::value || std::is_same<P, EulerRoe<R, 2, true>>::value ||
          (sizeof(R) == 4 && std::is_same<P, ShallowWater<R, 2>>::value))
             ? 2
             : 1;
}

// Stages A-C of every row in one basic block (prologue rows then compute
// values nobody reads; the Courant maxima and the stores stay conditional),
// so the scheduler can interleave the independent y-face and x-row work.
// Measured: 7% off the elasticity step, but slower shallow-water and Euler
// steps (their register budget is already full).
template <typename R, class P>
constexpr bool classic_eager_stages() {
  return std::is_same<P, Elastic<R>>::value;
}

// Which pipeline stages a row of the marching loop runs.  cfl: the x-row of
// stage C is an output row of the segment (its speeds enter the Courant
// number).
struct Stages {
  bool a, b, c, d, load, cfl;
};

template <typename R, class P, bool KAHAN, int LIM, int TRANS,
          int PF = classic_prefetch<R, P>(), bool EAGER = classic_eager_stages<R, P>()>
__global__ __launch_bounds__(kLanes) void k_classic2d(const GridDesc* __restrict__ grids,
                                                      const int* __restrict__ bstart, int ngrids,
                                                      int mode, double dt_host, int src_host) {
  constexpr int M = P::M, MW = P::MW, NA = P::NA > 0 ? P::NA : 1;
  constexpr int H = 2, U = kLanes - 2 * H;
  using Face = typename P::Face;

  const int b = blockIdx.x;
  const int gi = find_grid(bstart, ngrids, b);
  const GridDesc& G = grids[gi];
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
  const int lb = ngrids > 1 ? b - bstart[gi] : b;
  int strip, seg;
  tile_of(lb, G.strips, G.segs, G.order, strip, seg);
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
  const int ic = i < 0 ? 0 : (i >= nx ? nx - 1 : i);   // clamped column for pointwise reads
  const EdgeStates<R, M> es = edge_states<R, M>(G, mx);
  const gconst<R> q = as_gconst<R>(G.q[src]);
  const gmut<R> qo = as_gmut<R>(G.q[src ^ 1]);
  const gconst<R> aux = as_gconst<R>(G.aux);
  const gconst<R> cin = as_gconst<R>(G.c[src]);
  const gmut<R> cout = as_gmut<R>(G.c[src ^ 1]);
  const R dtdx = (R)(dt / G.dx), dtdy = (R)(dt / G.dy);
  const R nux = R(0.5) * dtdx, nuy = R(0.5) * dtdy;
  constexpr int trans = TRANS;
  const P phys(G);

  using Cell = typename P::Cell;
  R smx = R(0), smy = R(0);
  // rolling state (see the pipeline above)
  R q0[M], q1[M];
  Cell c0{}, c1{};                                        // cell data of rows r-2, r-1
  R ydl1[MW];                                             // W_p(r-5/2) . W_p(r-3/2)
  R yW1[MW][M], ys1[MW], yam1[M], yap1[M];                // y-face r-3/2
  Face yf1{};
  R glo[M], gtr_lo[M], gtop2[M], fxm2[M], fxp2[M], faL2[M], faR2[M];
#pragma unroll
  for (int k = 0; k < M; ++k) {
    q0[k] = q1[k] = yam1[k] = yap1[k] = R(0);
    glo[k] = gtr_lo[k] = gtop2[k] = fxm2[k] = fxp2[k] = faL2[k] = faR2[k] = R(0);
  }
#pragma unroll
  for (int p = 0; p < MW; ++p) {
    ydl1[p] = ys1[p] = R(0);
#pragma unroll
    for (int k = 0; k < M; ++k) yW1[p][k] = R(0);
  }

  // Row r+PF is loaded while row r is processed (software pipelining).  Row
  // r+1's boundary conditions are applied just before row r's results are
  // stored, so the wait for its loads comes PF rows of work after they were
  // issued and never behind this row's stores.
  R qnext[M], anext[NA];
  R qb[2][M], ab[2][NA];
  AxisMap myb[2] = {AxisMap{0, 0, 0}, AxisMap{0, 0, 0}};
  {
    const AxisMap my = map_axis(j0 - 2, ny, bcy0, bcy1, H);
    load_state<R, P>(qnext, q, plane, nx, mx, my, es);
    load_aux<R, P>(anext, aux, plane, nx, mx, my);
    if constexpr (PF == 2) {
      // row j0-1 goes to the buffer the first row reads (see the loop below)
      const AxisMap m1 = map_axis(j0 - 1, ny, bcy0, bcy1, H);
      if ((j0 - 2) & 1) {
        myb[0] = m1;
        load_raw<R, M>(qb[0], q, plane, nx, mx, m1);
        load_aux<R, P>(ab[0], aux, plane, nx, mx, m1);
      } else {
        myb[1] = m1;
        load_raw<R, M>(qb[1], q, plane, nx, mx, m1);
        load_aux<R, P>(ab[1], aux, plane, nx, mx, m1);
      }
    }
  }
  // One row of the pipeline (the stages that row r runs are in st; phase
  // selects the row buffers when PF == 2).
  auto row = [&](const Stages st, const int r, auto phase) {
    constexpr int ph = decltype(phase)::value;
    constexpr int cb = PF == 1 ? 0 : (ph ^ 1);   // buffer holding row r+1
    R qn[M], an[NA];
#pragma unroll
    for (int k = 0; k < M; ++k) qn[k] = qnext[k];
#pragma unroll
    for (int k = 0; k < NA; ++k) an[k] = anext[k];
    if constexpr (PF == 1) {
      if (st.load) {
        myb[0] = map_axis(r + 1, ny, bcy0, bcy1, H);
        load_raw<R, M>(qb[0], q, plane, nx, mx, myb[0]);
        load_aux<R, P>(ab[0], aux, plane, nx, mx, myb[0]);
      }
    } else {
      if (r + 2 <= j1 + 1) {
        myb[ph] = map_axis(r + 2, ny, bcy0, bcy1, H);
        load_raw<R, M>(qb[ph], q, plane, nx, mx, myb[ph]);
        load_aux<R, P>(ab[ph], aux, plane, nx, mx, myb[ph]);
      }
    }
    // the compensation of row r-2 (finalised below), read ahead of its use
    R cprev[M];
    if constexpr (KAHAN) {
      if (st.d) {
        const size_t off = (size_t)(r - 2) * nx + ic;
#pragma unroll
        for (int k = 0; k < M; ++k) cprev[k] = cin[k * plane + off];
      } else {
#pragma unroll
        for (int k = 0; k < M; ++k) cprev[k] = R(0);
      }
    }
    const Cell cn = phys.cell(qn, an);

    // (A) y-face r-1/2
    R yW2[MW][M], ys2[MW], yam2[M], yap2[M];
    Face yf2{};
    if (EAGER || st.a) {
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

    // dot products of the new face's waves with those of the face below: the
    // face below needs them now (its upper neighbour), the new face later
    // (its lower neighbour)
    R ydl2[MW];
#pragma unroll
    for (int p = 0; p < MW; ++p) {
      R d = R(0);
#pragma unroll
      for (int k = 0; k < M; ++k)
        if (P::template nz<1>(p, k)) d += yW1[p][k] * yW2[p][k];
      ydl2[p] = d;
    }

    // (B) y-face r-3/2: limiter, correction, transverse split into F
    R ghi[M], glo_n[M], faL1[M], faR1[M];
#pragma unroll
    for (int k = 0; k < M; ++k) ghi[k] = glo_n[k] = faL1[k] = faR1[k] = R(0);
    if (EAGER || st.b) {
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
        smy = st.b ? max_nan(smy, as) : smy;
        const R w = as * (R(1) - dtdy * as) * phi;
#pragma unroll
        for (int k = 0; k < M; ++k)
          if (P::template nz<1>(p, k)) cq[k] += w * yW1[p][k];
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        ghi[k] = yam1[k] + R(0.5) * cq[k];
        glo_n[k] = yap1[k] - R(0.5) * cq[k];
      }
      if (trans) {
        R bmq[M], bpq[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
          bmq[k] = yam1[k] + (trans == 2 ? cq[k] : R(0));
          bpq[k] = yap1[k] - (trans == 2 ? cq[k] : R(0));
        }
        // B^+ part lives in cell (i, r-1): its x-neighbours' cell data
        R lm[M], lp[M];
        phys.template transverse<1>(yf1, P::shfl_prev_cell(c1), c1, P::shfl_next_cell(c1), bpq,
                                    lm, lp);
#pragma unroll
        for (int k = 0; k < M; ++k) { faL1[k] = -nuy * lm[k]; faR1[k] = -nuy * lp[k]; }
        // B^- part lives in cell (i, r-2)
        phys.template transverse<1>(yf1, P::shfl_prev_cell(c0), c0, P::shfl_next_cell(c0), bmq,
                                    lm, lp);
#pragma unroll
        for (int k = 0; k < M; ++k) { faL2[k] -= nuy * lm[k]; faR2[k] -= nuy * lp[k]; }
      }
    }

    // (C) x-row r-1: normal solves across lanes, limiter, transverse split into G
    R fxm1[M], fxp1[M], gtop1[M], gtr_cur[M];
#pragma unroll
    for (int k = 0; k < M; ++k) fxm1[k] = fxp1[k] = gtop1[k] = gtr_cur[k] = R(0);
    if (EAGER || st.c) {
      R ql[M];
#pragma unroll
      for (int k = 0; k < M; ++k) ql[k] = shfl_prev(q1[k]);
      R xW[MW][M], xs[MW], xam[M], xap[M];
      Face xf{};
      phys.template normal<0>(ql, q1, P::shfl_prev_cell(c1), c1, xW, xs, xam, xap, xf);
      R cq[M];
#pragma unroll
      for (int k = 0; k < M; ++k) cq[k] = R(0);
#pragma unroll
      for (int p = 0; p < MW; ++p) {
        R nrm = R(0), dl = R(0);
#pragma unroll
        for (int k = 0; k < M; ++k) {
          if (!P::template nz<0>(p, k)) continue;
          nrm += xW[p][k] * xW[p][k];
          dl += shfl_prev(xW[p][k]) * xW[p][k];
        }
        const R dr = shfl_next(dl);   // the right neighbour's dot product with this face
        const R phi = limiter_phi_t<LIM>(xs[p] > R(0) ? dl : dr, nrm);
        const R as = rabs(xs[p]);
        if (st.cfl && own_face) smx = max_nan(smx, as);
        const R w = as * (R(1) - dtdx * as) * phi;
#pragma unroll
        for (int k = 0; k < M; ++k)
          if (P::template nz<0>(p, k)) cq[k] += w * xW[p][k];
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        fxm1[k] = xam[k] + R(0.5) * cq[k];
        fxp1[k] = xap[k] - R(0.5) * cq[k];
      }
      R gbot1[M];
#pragma unroll
      for (int k = 0; k < M; ++k) gbot1[k] = R(0);
      if (trans) {
        R amq[M], apq[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
          amq[k] = xam[k] + (trans == 2 ? cq[k] : R(0));
          apq[k] = xap[k] - (trans == 2 ? cq[k] : R(0));
        }
        // A^+ of face i-1/2 lives in cell (i, r-1); A^- of face i+1/2 too (from lane+1)
        R bm[M], bp[M], bm2[M], bp2[M], amn[M];
        phys.template transverse<0>(xf, c0, c1, cn, apq, bm, bp);
#pragma unroll
        for (int k = 0; k < M; ++k) amn[k] = shfl_next(amq[k]);
        const Face xfn = P::shfl_next_face(xf);
        phys.template transverse<0>(xfn, c0, c1, cn, amn, bm2, bp2);
#pragma unroll
        for (int k = 0; k < M; ++k) {
          gbot1[k] = -nux * (bm[k] + bm2[k]);
          gtop1[k] = -nux * (bp[k] + bp2[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < M; ++k) gtr_cur[k] = gtop2[k] + gbot1[k];
    }

    if (st.load) {
#pragma unroll
      for (int k = 0; k < M; ++k) qnext[k] = qb[cb][k];
      apply_bc<R, P>(qnext, mx, myb[cb], es);
#pragma unroll
      for (int k = 0; k < NA; ++k) anext[k] = ab[cb][k];
    }

    // (D) row r-2 is complete
    if (st.d) {
      const int f = r - 2;
      const size_t off = (size_t)f * nx + i;
      R xs[M], ys[M];
#pragma unroll
      for (int k = 0; k < M; ++k) {
        const R ftr = shfl_prev(faR2[k]) + faL2[k];   // transverse part of F~ at x-face i-1/2
        const R fp = fxp2[k] - ftr;                    // A^+dQ - F~ at i-1/2
        const R fm = shfl_next(fxm2[k] + ftr);         // A^-dQ + F~ at i+1/2
        const R gp = glo[k] - gtr_lo[k];               // B^+dQ - G~ at r-5/2
        const R gm = ghi[k] + gtr_cur[k];              // B^-dQ + G~ at r-3/2
        xs[k] = fp + fm;
        ys[k] = gp + gm;
      }
      if constexpr (P::kSource) {
        // geometric source as a fractional step after the hyperbolic update,
        // fused here: pointwise on the updated cell, so the same arithmetic
        // as a separate pass over the new state
        R inc[M];
#pragma unroll
        for (int k = 0; k < M; ++k) inc[k] = -(dtdx * xs[k] + dtdy * ys[k]);
        if (G.source) {
          const R ir = (R)(1.0 / (G.ylo + (f + 0.5) * G.dy));
          R qs[4], ds[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) qs[k] = q0[k] + inc[k];
          phys.source_increment(qs, ir, (R)dt, ds);
#pragma unroll
          for (int k = 0; k < 4; ++k) inc[k] += ds[k];
        }
        if (own) {
#pragma unroll
          for (int k = 0; k < M; ++k) {
            if constexpr (KAHAN) {
              const R y = inc[k] - cprev[k];
              const R t = q0[k] + y;
              cout[k * plane + off] = (t - q0[k]) - y;
              qo[k * plane + off] = t;
            } else {
              qo[k * plane + off] = q0[k] + inc[k];
            }
          }
        }
      } else if (own) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
          if constexpr (KAHAN) {
            const R inc = -(dtdx * xs[k] + dtdy * ys[k]);
            const R y = inc - cprev[k];
            const R t = q0[k] + y;
            cout[k * plane + off] = (t - q0[k]) - y;
            qo[k * plane + off] = t;
          } else {
            qo[k * plane + off] = q0[k] - dtdx * xs[k] - dtdy * ys[k];
          }
        }
      }
    }

    // rotate
#pragma unroll
    for (int k = 0; k < M; ++k) {
      q0[k] = q1[k];
      q1[k] = qn[k];
      yam1[k] = yam2[k];
      yap1[k] = yap2[k];
      glo[k] = glo_n[k];
      gtr_lo[k] = gtr_cur[k];
      gtop2[k] = gtop1[k];
      fxm2[k] = fxm1[k];
      fxp2[k] = fxp1[k];
      faL2[k] = faL1[k];
      faR2[k] = faR1[k];
    }
    c0 = c1;
    c1 = cn;
#pragma unroll
    for (int p = 0; p < MW; ++p) {
      ys1[p] = ys2[p];
      ydl1[p] = ydl2[p];
#pragma unroll
      for (int k = 0; k < M; ++k) yW1[p][k] = yW2[p][k];
    }
    yf1 = yf2;
  };
  // rows j0-2 .. j0+1 fill the pipeline; j0+2 .. j1 are steady; j1+1 drains
  auto stages = [&](const int r) {
    return Stages{r >= j0 - 1, r >= j0 + 1, r >= j0, r >= j0 + 2, r + 1 <= j1 + 1,
                  r - 1 >= j0 && r - 1 < j1};
  };
  if constexpr (PF == 1) {
    for (int r = j0 - 2; r <= j1 + 1; ++r) row(stages(r), r, std::integral_constant<int, 0>{});
  } else {
    // Every row runs in the phase of its parity, whatever the tiling: the two
    // instantiations of the body may round differently (contractions), and
    // results must not depend on where segments start.
    int r = j0 - 2;
    if (r & 1) {
      row(stages(r), r, std::integral_constant<int, 1>{});
      ++r;
    }
    for (; r <= j1 + 1; r += 2) {
      row(stages(r), r, std::integral_constant<int, 0>{});
      if (r + 1 <= j1 + 1) row(stages(r + 1), r + 1, std::integral_constant<int, 1>{});
    }
  }

  const double speed = own ? max_nan((double)smx / G.dx, (double)smy / G.dy)
                           : (own_face ? (double)smx / G.dx : 0.0);
  if (mode == kDeviceCtrl) {
    finish_workgroup(ctrl, G.slots, lb, G.nblocks, speed, [](Ctrl* c, double sp) {
      if (ctrl_decide(c, sp)) c->src ^= 1;
    });
  } else {
    finish_workgroup(ctrl, G.slots, lb, G.nblocks, speed,
                     [](Ctrl* c, double sp) { c->last_speed = sp; });
  }
}

// ---------------------------------------------------------------------------
// 1D classic step: one wavefront per 60-cell strip (2 halo lanes each side).
// ---------------------------------------------------------------------------
template <typename R, class P, bool KAHAN>
__global__ __launch_bounds__(kLanes) void k_classic1d(const GridDesc* __restrict__ grids,
                                                      const int* __restrict__ bstart, int ngrids,
                                                      int mode, double dt_host, int src_host) {
  constexpr int M = P::M, MW = P::MW;
  constexpr int H = 2, U = kLanes - 2 * H;
  using Face = typename P::Face;
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
  const int nx = G.nx;
  const int lane = threadIdx.x;
  const int i = blockIdx.x * U - H + lane;
  const bool own = lane >= H && lane < H + U && i < nx;
  const bool own_face = lane >= H && lane <= H + U && i <= nx;
  const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], H);
  const AxisMap my{0, 0, 0};
  const gconst<R> q = as_gconst<R>(G.q[src]);
  const gmut<R> qo = as_gmut<R>(G.q[src ^ 1]);
  const R dtdx = (R)(dt / G.dx);
  const P phys(G);
  using Cell = typename P::Cell;
  R qc[M], ql[M];
  R dummy[1] = {R(0)};
  load_state<R, P>(qc, q, (size_t)nx, nx, mx, my, edge_states<R, M>(G, mx));
#pragma unroll
  for (int k = 0; k < M; ++k) ql[k] = shfl_prev(qc[k]);
  const Cell cc = phys.cell(qc, dummy);
  R W[MW][M], s[MW], am[M], ap[M];
  Face f{};
  phys.template normal<0>(ql, qc, P::shfl_prev_cell(cc), cc, W, s, am, ap, f);
  R cq[M];
#pragma unroll
  for (int k = 0; k < M; ++k) cq[k] = R(0);
  R smx = R(0);
#pragma unroll
  for (int p = 0; p < MW; ++p) {
    R nrm = R(0), dl = R(0);
#pragma unroll
    for (int k = 0; k < M; ++k) {
      nrm += W[p][k] * W[p][k];
      dl += shfl_prev(W[p][k]) * W[p][k];
    }
    const R dr = shfl_next(dl);
    const R phi = limiter_phi(G.limiter, s[p] > R(0) ? dl : dr, nrm);
    const R as = rabs(s[p]);
    smx = max_nan(smx, as);
    const R w = as * (R(1) - dtdx * as) * phi;
#pragma unroll
    for (int k = 0; k < M; ++k) cq[k] += w * W[p][k];
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const R fp = ap[k] - R(0.5) * cq[k];
    const R fm = shfl_next(am[k] + R(0.5) * cq[k]);
    if (own) {
      if constexpr (KAHAN) {
        const gconst<R> cin = as_gconst<R>(G.c[src]);
        const gmut<R> cout = as_gmut<R>(G.c[src ^ 1]);
        const R inc = -(dtdx * (fp + fm));
        const R y = inc - cin[(size_t)k * nx + i];
        const R t = qc[k] + y;
        cout[(size_t)k * nx + i] = (t - qc[k]) - y;
        qo[(size_t)k * nx + i] = t;
      } else {
        qo[(size_t)k * nx + i] = qc[k] - dtdx * (fp + fm);
      }
    }
  }
  const double speed = own_face ? (double)smx / G.dx : 0.0;
  if (mode == kDeviceCtrl) {
    finish_workgroup(ctrl, G.slots, blockIdx.x, G.nblocks, speed, [](Ctrl* c, double sp) {
      if (ctrl_decide(c, sp)) c->src ^= 1;
    });
  } else {
    finish_workgroup(ctrl, G.slots, blockIdx.x, G.nblocks, speed,
                     [](Ctrl* c, double sp) { c->last_speed = sp; });
  }
}

// ---------------------------------------------------------------------------
// 1D whole-run kernel for small grids: one workgroup keeps the grid in LDS
// and runs the step controller itself, so a complete advance to t_end is one
// launch.  Per attempt: every face solves its Riemann problem and those of
// its two neighbours (for the limiter), writes A^-dQ + F~ and A^+dQ - F~ to
// LDS; the workgroup reduces the speed, decides, and applies the update.
// ---------------------------------------------------------------------------
constexpr int kPersistThreads = 1024;

template <typename R, class P, bool KAHAN>
__global__ __launch_bounds__(kPersistThreads) void k_classic1d_run(const GridDesc* __restrict__ grids) {
  constexpr int M = P::M, MW = P::MW;
  using Face = typename P::Face;
  extern __shared__ unsigned char smem_raw[];
  const GridDesc& G = grids[0];
  Ctrl* ctrl = G.ctrl;
  const int nx = G.nx;
  R* sq = (R*)smem_raw;               // q[M][nx]
  R* sc = sq + (size_t)M * nx;        // compensation [M][nx] (FP32 mode)
  R* sfm = sc + (KAHAN ? (size_t)M * nx : 0);   // [M][nx+1]
  R* sfp = sfm + (size_t)M * (nx + 1);          // [M][nx+1]
  __shared__ double red[kPersistThreads / kLanes];
  __shared__ int s_go, s_ok;
  __shared__ double s_dt;
  const int tid = threadIdx.x;
  const R* __restrict__ q = (const R*)G.q[ctrl->src];
  for (int n = tid; n < M * nx; n += blockDim.x) sq[n] = q[n];
  if constexpr (KAHAN) {
    const R* __restrict__ c = (const R*)G.c[ctrl->src];
    for (int n = tid; n < M * nx; n += blockDim.x) sc[n] = c[n];
  }
  if (tid == 0) {
    s_go = ctrl->active;
    s_dt = ctrl->dt_try;
  }
  __syncthreads();
  const P phys(G);
  const AxisMap my{0, 0, 0};
  R dummy[1] = {R(0)};
  auto cell = [&](int i, R (&v)[M]) {
    const AxisMap mx = map_axis(i, nx, G.bc[0], G.bc[1], 2);
    if (mx.kind == 2) {
#pragma unroll
      for (int k = 0; k < M; ++k) v[k] = (R)G.bcstate[mx.side][k];
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) v[k] = sq[k * nx + mx.idx];
      if (mx.kind == 1) {
#pragma unroll
        for (int k = 0; k < M; ++k)
          if (P::odd(0, k)) v[k] = -v[k];
      }
    }
  };
  while (s_go) {
    const double dt = s_dt;
    const R dtdx = (R)(dt / G.dx);
    R smx = R(0);
    for (int f = tid; f <= nx; f += blockDim.x) {
      // faces f-1, f, f+1 (face f lies between cells f-1 and f)
      R c0[M], c1[M], c2[M], c3[M];
      cell(f - 2, c0); cell(f - 1, c1); cell(f, c2); cell(f + 1, c3);
      const typename P::Cell e0 = phys.cell(c0, dummy), e1 = phys.cell(c1, dummy),
                             e2 = phys.cell(c2, dummy), e3 = phys.cell(c3, dummy);
      R Wl[MW][M], sl[MW], aml[M], apl[M], W[MW][M], s[MW], am[M], ap[M], Wr[MW][M], sr[MW],
          amr[M], apr[M];
      Face fa{};
      phys.template normal<0>(c0, c1, e0, e1, Wl, sl, aml, apl, fa);
      phys.template normal<0>(c1, c2, e1, e2, W, s, am, ap, fa);
      phys.template normal<0>(c2, c3, e2, e3, Wr, sr, amr, apr, fa);
      R cq[M];
#pragma unroll
      for (int k = 0; k < M; ++k) cq[k] = R(0);
#pragma unroll
      for (int p = 0; p < MW; ++p) {
        R nrm = R(0), dl = R(0), dr = R(0);
#pragma unroll
        for (int k = 0; k < M; ++k) {
          nrm += W[p][k] * W[p][k];
          dl += Wl[p][k] * W[p][k];
          dr += Wr[p][k] * W[p][k];
        }
        const R phi = limiter_phi(G.limiter, s[p] > R(0) ? dl : dr, nrm);
        const R as = rabs(s[p]);
        smx = max_nan(smx, as);
        const R w = as * (R(1) - dtdx * as) * phi;
#pragma unroll
        for (int k = 0; k < M; ++k) cq[k] += w * W[p][k];
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        sfm[k * (nx + 1) + f] = am[k] + R(0.5) * cq[k];
        sfp[k * (nx + 1) + f] = ap[k] - R(0.5) * cq[k];
      }
    }
    double sp = wave_max((double)smx / G.dx);
    if ((tid & (kLanes - 1)) == 0) red[tid / kLanes] = sp;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int w = 0; w < (int)(blockDim.x / kLanes); ++w) m = max_nan(m, red[w]);
      s_ok = ctrl_decide(ctrl, m) ? 1 : 0;
      s_go = ctrl->active;
      s_dt = ctrl->dt_try;
    }
    __syncthreads();
    if (s_ok) {
      for (int n = tid; n < M * nx; n += blockDim.x) {
        const int k = n / nx, i = n - k * nx;
        const R inc = -(dtdx * (sfp[k * (nx + 1) + i] + sfm[k * (nx + 1) + i + 1]));
        if constexpr (KAHAN) {
          const R y = inc - sc[n];
          const R t = sq[n] + y;
          sc[n] = (t - sq[n]) - y;
          sq[n] = t;
        } else {
          sq[n] = sq[n] + inc;
        }
      }
    }
    __syncthreads();
  }
  R* __restrict__ qo = (R*)G.q[ctrl->src];
  for (int n = tid; n < M * nx; n += blockDim.x) qo[n] = sq[n];
  if constexpr (KAHAN) {
    R* __restrict__ co = (R*)G.c[ctrl->src];
    for (int n = tid; n < M * nx; n += blockDim.x) co[n] = sc[n];
  }
}

// ---------------------------------------------------------------------------
// Host-side launchers (dispatch on solver and precision).
// ---------------------------------------------------------------------------
template <typename R, bool K, int LIM, int TRANS>
static hipError_t launch2d_lt(int riemann, dim3 grid, hipStream_t st, const GridDesc* g,
                              const int* bs, int ng, int mode, double dt, int src) {
  switch (riemann) {
    case 1:
      hipLaunchKernelGGL((k_classic2d<R, Advection<R, 2>, K, LIM, TRANS>), grid, dim3(kLanes), 0,
                         st, g, bs, ng, mode, dt, src);
      break;
    case 2:
      hipLaunchKernelGGL((k_classic2d<R, ShallowWater<R, 2>, K, LIM, TRANS>), grid, dim3(kLanes),
                         0, st, g, bs, ng, mode, dt, src);
      break;
    case 4:
      hipLaunchKernelGGL((k_classic2d<R, Elastic<R>, K, LIM, TRANS>), grid, dim3(kLanes), 0, st, g,
                         bs, ng, mode, dt, src);
      break;
    case 5:
      hipLaunchKernelGGL((k_classic2d<R, EulerRoe<R, 2, false>, K, LIM, TRANS>), grid, dim3(kLanes),
                         0, st, g, bs, ng, mode, dt, src);
      break;
    case 6:
      hipLaunchKernelGGL((k_classic2d<R, EulerRoe<R, 2, true>, K, LIM, TRANS>), grid, dim3(kLanes),
                         0, st, g, bs, ng, mode, dt, src);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename R, bool K, int LIM>
static hipError_t launch2d_l(int riemann, int trans, dim3 grid, hipStream_t st, const GridDesc* g,
                             const int* bs, int ng, int mode, double dt, int src) {
  switch (trans) {
    case 0: return launch2d_lt<R, K, LIM, 0>(riemann, grid, st, g, bs, ng, mode, dt, src);
    case 1: return launch2d_lt<R, K, LIM, 1>(riemann, grid, st, g, bs, ng, mode, dt, src);
    case 2: return launch2d_lt<R, K, LIM, 2>(riemann, grid, st, g, bs, ng, mode, dt, src);
  }
  return hipErrorInvalidValue;
}

template <typename R, bool K>
static hipError_t launch2d_t(int riemann, int lim, int trans, dim3 grid, hipStream_t st,
                             const GridDesc* g, const int* bs, int ng, int mode, double dt,
                             int src) {
  switch (lim) {
    case 0: return launch2d_l<R, K, 0>(riemann, trans, grid, st, g, bs, ng, mode, dt, src);
    case 1: return launch2d_l<R, K, 1>(riemann, trans, grid, st, g, bs, ng, mode, dt, src);
    case 2: return launch2d_l<R, K, 2>(riemann, trans, grid, st, g, bs, ng, mode, dt, src);
  }
  return hipErrorInvalidValue;
}

// limiter and transverse mode are compile-time in the 2D kernel (no branches
// in the marching loop); every member of a batch shares them
// plain FP32 (no compensation): shallow water only
template <int LIM, int TRANS>
static hipError_t launch2d_plain32_lt(dim3 grid, hipStream_t st, const GridDesc* g, const int* bs,
                                      int ng, int mode, double dt, int src) {
  hipLaunchKernelGGL((k_classic2d<float, ShallowWater<float, 2>, false, LIM, TRANS>), grid,
                     dim3(kLanes), 0, st, g, bs, ng, mode, dt, src);
  return hipGetLastError();
}
template <int LIM>
static hipError_t launch2d_plain32_l(int trans, dim3 grid, hipStream_t st, const GridDesc* g,
                                     const int* bs, int ng, int mode, double dt, int src) {
  switch (trans) {
    case 0: return launch2d_plain32_lt<LIM, 0>(grid, st, g, bs, ng, mode, dt, src);
    case 1: return launch2d_plain32_lt<LIM, 1>(grid, st, g, bs, ng, mode, dt, src);
    case 2: return launch2d_plain32_lt<LIM, 2>(grid, st, g, bs, ng, mode, dt, src);
  }
  return hipErrorInvalidValue;
}

// prec: 0 FP64, 1 FP32 with Kahan-compensated updates, 2 plain FP32
hipError_t launch_classic2d(int riemann, int prec, int lim, int trans, int nblocks, hipStream_t st,
                            const GridDesc* d_grids, const int* d_bstart, int ngrids, int mode,
                            double dt, int src) {
  const dim3 grid(nblocks);
  if (prec == 2) {
    if (riemann != 2) return hipErrorInvalidValue;
    switch (lim) {
      case 0: return launch2d_plain32_l<0>(trans, grid, st, d_grids, d_bstart, ngrids, mode, dt, src);
      case 1: return launch2d_plain32_l<1>(trans, grid, st, d_grids, d_bstart, ngrids, mode, dt, src);
      case 2: return launch2d_plain32_l<2>(trans, grid, st, d_grids, d_bstart, ngrids, mode, dt, src);
    }
    return hipErrorInvalidValue;
  }
  return prec ? launch2d_t<float, true>(riemann, lim, trans, grid, st, d_grids, d_bstart, ngrids,
                                        mode, dt, src)
              : launch2d_t<double, false>(riemann, lim, trans, grid, st, d_grids, d_bstart, ngrids,
                                          mode, dt, src);
}

template <typename R, bool K>
static hipError_t launch1d_t(int riemann, dim3 grid, hipStream_t st, const GridDesc* g, int mode,
                             double dt, int src) {
  switch (riemann) {
    case 1:
      hipLaunchKernelGGL((k_classic1d<R, Advection<R, 1>, K>), grid, dim3(kLanes), 0, st, g,
                         nullptr, 1, mode, dt, src);
      break;
    case 2:
      hipLaunchKernelGGL((k_classic1d<R, ShallowWater<R, 1>, K>), grid, dim3(kLanes), 0, st, g,
                         nullptr, 1, mode, dt, src);
      break;
    case 5:
      hipLaunchKernelGGL((k_classic1d<R, EulerRoe<R, 1, false>, K>), grid, dim3(kLanes), 0, st, g,
                         nullptr, 1, mode, dt, src);
      break;
    case 6:
      hipLaunchKernelGGL((k_classic1d<R, EulerRoe<R, 1, true>, K>), grid, dim3(kLanes), 0, st, g,
                         nullptr, 1, mode, dt, src);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_classic1d(int riemann, int fp32, int nblocks, hipStream_t st,
                            const GridDesc* d_grids, int mode, double dt, int src) {
  const dim3 grid(nblocks);
  return fp32 ? launch1d_t<float, true>(riemann, grid, st, d_grids, mode, dt, src)
              : launch1d_t<double, false>(riemann, grid, st, d_grids, mode, dt, src);
}

size_t classic1d_run_smem(int m, int nx, int fp32) {
  const size_t rb = fp32 ? 4 : 8;
  return rb * ((size_t)m * nx * (fp32 ? 2 : 1) + 2 * (size_t)m * (nx + 1));
}

template <typename R, bool K>
static hipError_t launch1d_run_t(int riemann, size_t smem, hipStream_t st, const GridDesc* g) {
  switch (riemann) {
    case 1:
      hipLaunchKernelGGL((k_classic1d_run<R, Advection<R, 1>, K>), dim3(1), dim3(kPersistThreads),
                         smem, st, g);
      break;
    case 2:
      hipLaunchKernelGGL((k_classic1d_run<R, ShallowWater<R, 1>, K>), dim3(1),
                         dim3(kPersistThreads), smem, st, g);
      break;
    case 5:
      hipLaunchKernelGGL((k_classic1d_run<R, EulerRoe<R, 1, false>, K>), dim3(1),
                         dim3(kPersistThreads), smem, st, g);
      break;
    case 6:
      hipLaunchKernelGGL((k_classic1d_run<R, EulerRoe<R, 1, true>, K>), dim3(1),
                         dim3(kPersistThreads), smem, st, g);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_classic1d_run(int riemann, int fp32, int m, int nx, hipStream_t st,
                                const GridDesc* d_grids) {
  const size_t smem = classic1d_run_smem(m, nx, fp32);
  return fp32 ? launch1d_run_t<float, true>(riemann, smem, st, d_grids)
              : launch1d_run_t<double, false>(riemann, smem, st, d_grids);
}

}  // namespace claw
