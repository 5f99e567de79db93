// phys.h -- Riemann solvers, transverse solvers and numerical fluxes for the
// gfx950 kernels (the problem-specific kernels of the paper's Section 2.1:
// the Riemann solver is the only problem-specific part of the algorithms).
//
// Each classic policy P provides
//   M, MW, NA                      equations, waves, aux fields
//   nz<D>(p, k)                    compile-time zero pattern of wave p at a
//                                  face normal to D (lets the marching kernels
//                                  skip known-zero components)
//   odd(d, k)                      sign flip of component k at a wall normal to d
//   Cell, cell(q, aux)             per-cell quantities computed once per loaded
//                                  cell and shared by its four faces
//                                  (velocities, celerity, material speeds)
//   Face                           data of a normal solve reused by the
//                                  transverse split (e.g. Roe averages)
//   normal<D>(ql, qr, cl, cr, W, s, amdq, apdq, face)
//   transverse<D>(face, c_lo, c_c, c_hi, asdq, bm, bp)
//                                  split a fluctuation produced at a face
//                                  normal to D, living in cell c_c, into the
//                                  parts moving toward lower (bm) and higher
//                                  (bp) index in the other direction; c_lo /
//                                  c_hi are that cell's neighbours there
//   shfl_prev_cell / shfl_next_cell / shfl_next_face   lane shifts of these
//   cell_speed(q, a, rdx, rdy)     largest characteristic speed/spacing of a
//                                  cell (a-priori first step)
//
// SharpClaw policies provide M, NA, odd(d, k) and flux<D>(ql, qr, F) ->
// max |speed| (Section 2.1: normal Riemann problems only); with NA > 0 the
// flux is flux<D>(ql, qr, al, ar, F), al / ar the aux fields (material) of
// the two cells the face separates.
#pragma once

#include "dev_common.h"

namespace claw {

// min / max as single v_min / v_max instructions (operands are finite here)
__device__ __forceinline__ double rmin(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ double rmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float rmin(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ float rmax(float a, float b) { return __builtin_fmaxf(a, b); }
template <typename R> __device__ __forceinline__ R rabs(R a) { return a < R(0) ? -a : a; }

// A product rounded on its own.  Interface fluxes end with one: left free,
// the compiler may fuse a lane's own unrounded flux into the flux difference
// while the neighbour's arrives rounded through the lane shift, so the two
// cells of a face would see fluxes differing in the last bit (a uniform state
// then drifts, and conservation holds one ulp less exactly).
template <typename R>
__device__ __forceinline__ R mul_rounded(R a, R b) {
#pragma clang fp contract(off)
  return a * b;
}

// ---------------------------------------------------------------------------
// Scalar advection q_t + u q_x + v q_y = 0 (test problem: exact translation,
// convergence).  One wave, the jump, at speed u (x) or v (y).
// ---------------------------------------------------------------------------
template <typename R, int NDIM>
struct Advection {
  static constexpr int M = 1, MW = 1, NA = 0;
  static constexpr bool kSource = false;
  struct Cell {};
  struct Face {};
  R u, v;
  __device__ explicit Advection(const GridDesc& G) : u((R)G.pd[0]), v((R)G.pd[1]) {}
  template <int D> static constexpr bool nz(int, int) { return true; }
  static constexpr bool odd(int, int) { return false; }
  __device__ __forceinline__ Cell cell(const R*, const R*) const { return Cell{}; }
  __device__ __forceinline__ static Cell shfl_prev_cell(const Cell& c) { return c; }
  __device__ __forceinline__ static Cell shfl_next_cell(const Cell& c) { return c; }
  __device__ __forceinline__ static Face shfl_next_face(const Face& f) { return f; }

  template <int D>
  __device__ __forceinline__ void normal(const R* ql, const R* qr, const Cell&, const Cell&,
                                         R (&W)[MW][M], R (&s)[MW], R (&am)[M], R (&ap)[M],
                                         Face&) const {
    const R un = D == 0 ? u : v;
    const R dq = qr[0] - ql[0];
    W[0][0] = dq;
    s[0] = un;
    am[0] = rmin(un, R(0)) * dq;
    ap[0] = rmax(un, R(0)) * dq;
  }
  template <int D>
  __device__ __forceinline__ void transverse(const Face&, const Cell&, const Cell&, const Cell&,
                                             const R* asdq, R* bm, R* bp) const {
    const R vt = D == 0 ? v : u;
    bm[0] = rmin(vt, R(0)) * asdq[0];
    bp[0] = rmax(vt, R(0)) * asdq[0];
  }
  __device__ __forceinline__ double cell_speed(const R*, const R*, double rdx, double rdy) const {
    double s = fabs((double)u) * rdx;
    if (NDIM == 2) s = fmax(s, fabs((double)v) * rdy);
    return s;
  }
};

// ---------------------------------------------------------------------------
// Shallow water, Roe linearisation with an optional Harten-Hyman entropy fix
// (the Roe solver with an entropy fix of the paper's Section 5; formulas as
// in LeVeque 2002, ch. 15).  q = (h, hu) in 1D, (h, hu, hv) in 2D.  Families:
// 0 = left acoustic (u-c), [1 = shear (u), 2D only], last = right acoustic
// (u+c).
// ---------------------------------------------------------------------------
template <typename R, int NDIM>
struct ShallowWater {
  static constexpr int M = NDIM == 1 ? 2 : 3;
  static constexpr int MW = M;
  static constexpr int NA = 0;
  static constexpr int LAST = MW - 1;
  static constexpr bool kSource = false;
  struct Cell {
    R u, v, sh, c;   // velocities, sqrt(h), celerity sqrt(g h)
  };
  struct Face {
    R u, v, c, i2c;  // Roe-averaged normal / tangential velocity, celerity, 1/(2c)
  };
  R g, sg;
  int efix;
  __device__ explicit ShallowWater(const GridDesc& G)
      : g((R)G.pd[0]), sg((R)sqrt(G.pd[0])), efix(G.efix) {}

  // zero pattern: acoustic waves (1, u -/+ c, v); shear wave: tangential only
  template <int D>
  static constexpr bool nz(int p, int k) {
    if (NDIM == 1) return true;
    return (p == 1) ? (k == 2 - D) : true;
  }
  static constexpr bool odd(int d, int k) { return k == 1 + d; }

  __device__ __forceinline__ Cell cell(const R* q, const R*) const {
    const R rs = frsq(q[0]);          // 1/sqrt(h)
    const R rh = rs * rs;             // 1/h
    Cell c;
    c.sh = q[0] * rs;
    c.u = q[1] * rh;
    c.v = NDIM == 2 ? q[2] * rh : R(0);
    c.c = sg * c.sh;
    return c;
  }
  __device__ __forceinline__ static Cell shfl_prev_cell(const Cell& c) {
    return Cell{shfl_prev(c.u), NDIM == 2 ? shfl_prev(c.v) : R(0), shfl_prev(c.sh), shfl_prev(c.c)};
  }
  __device__ __forceinline__ static Cell shfl_next_cell(const Cell& c) {
    return Cell{shfl_next(c.u), NDIM == 2 ? shfl_next(c.v) : R(0), shfl_next(c.sh), shfl_next(c.c)};
  }
  __device__ __forceinline__ static Face shfl_next_face(const Face& f) {
    return Face{shfl_next(f.u), shfl_next(f.v), shfl_next(f.c), shfl_next(f.i2c)};
  }

  template <int D>
  __device__ __forceinline__ void normal(const R* ql, const R* qr, const Cell& cl, const Cell& cr,
                                         R (&W)[MW][M], R (&s)[MW], R (&am)[M], R (&ap)[M],
                                         Face& f) const {
    constexpr int n = 1 + D;      // normal momentum
    constexpr int t = 2 - D;      // tangential momentum (2D)
    const R hl = ql[0], hr = qr[0];
    const R unl = D == 0 ? cl.u : cl.v, unr = D == 0 ? cr.u : cr.v;
    const R rden = frcp(cl.sh + cr.sh);
    f.u = (cl.sh * unl + cr.sh * unr) * rden;
    if constexpr (NDIM == 2) {
      const R utl = D == 0 ? cl.v : cl.u, utr = D == 0 ? cr.v : cr.u;
      f.v = (cl.sh * utl + cr.sh * utr) * rden;
    } else {
      f.v = R(0);
    }
    const R c2 = g * (R(0.5) * (hl + hr));
    const R rs = frsq(c2);
    f.c = c2 * rs;
    f.i2c = R(0.5) * rs;
    const R d0 = qr[0] - ql[0], dn = qr[n] - ql[n];
    const R a1 = ((f.u + f.c) * d0 - dn) * f.i2c;
    const R a3 = (-(f.u - f.c) * d0 + dn) * f.i2c;
    const R s1 = f.u - f.c, s3 = f.u + f.c;
    W[0][0] = a1; W[0][n] = a1 * s1;
    W[LAST][0] = a3; W[LAST][n] = a3 * s3;
    s[0] = s1;
    s[LAST] = s3;
    if constexpr (NDIM == 2) {
      W[0][t] = a1 * f.v;
      W[2][t] = a3 * f.v;
      W[1][0] = R(0); W[1][n] = R(0);
      W[1][t] = (qr[t] - ql[t]) - f.v * d0;
      s[1] = f.u;
    }
    R coef[MW];
#pragma unroll
    for (int p = 0; p < MW; ++p) coef[p] = rmin(s[p], R(0));
    if (efix) {
      // Harten-Hyman: an acoustic wave whose left-side characteristic speed is
      // negative and right-side one positive is a transonic rarefaction; its
      // contribution to A^-dQ becomes lam_l (lam_r - s) / (lam_r - lam_l) W.
      // The expensive right/left speed is formed only when a cheap exact test
      // (u_m > c_m  <=>  hu_m > 0 and hu_m^2 > g h_m^3, for h_m > 0) says the
      // wave is transonic; the coefficient is continuous where the test flips.
      {
        const R lam_l = unl - cl.c;
        const R hm = hl + W[0][0], hum = ql[n] + W[0][n];
        if (lam_l < R(0) && hm > R(0) && hum > R(0) && hum * hum > g * hm * hm * hm) {
          const R lam_r = hum * frcp(hm) - fsqrt(g * hm);
          if (R(0) < lam_r) coef[0] = lam_l * (lam_r - s1) * frcp(lam_r - lam_l);
        }
      }
      {
        const R lam_r = unr + cr.c;
        const R hm = hr - W[LAST][0], hum = qr[n] - W[LAST][n];
        if (lam_r > R(0) && hm > R(0) && hum < R(0) && hum * hum > g * hm * hm * hm) {
          const R lam_l = hum * frcp(hm) + fsqrt(g * hm);
          if (lam_l < R(0)) coef[LAST] = lam_l * (lam_r - s3) * frcp(lam_r - lam_l);
        }
      }
#pragma unroll
      for (int k = 0; k < M; ++k) {
        R a = R(0), sw = R(0);
#pragma unroll
        for (int p = 0; p < MW; ++p) {
          if (!nz<D>(p, k)) continue;
          a += coef[p] * W[p][k];
          sw += s[p] * W[p][k];
        }
        am[k] = a;
        ap[k] = sw - a;
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) {
        R a = R(0), b = R(0);
#pragma unroll
        for (int p = 0; p < MW; ++p) {
          if (!nz<D>(p, k)) continue;
          a += coef[p] * W[p][k];
          b += rmax(s[p], R(0)) * W[p][k];
        }
        am[k] = a;
        ap[k] = b;
      }
    }
  }

  // Split in the transverse direction with the face's Roe averages:
  // speeds v-c, v, v+c; eigenvectors (1, u, v-c), e_n, (1, u, v+c) in
  // (depth, normal, tangential) ordering of the face.
  template <int D>
  __device__ __forceinline__ void transverse(const Face& f, const Cell&, const Cell&, const Cell&,
                                             const R* d, R* bm, R* bp) const {
    if constexpr (NDIM == 2) {
      constexpr int n = 1 + D, t = 2 - D;
      const R b1 = ((f.v + f.c) * d[0] - d[t]) * f.i2c;
      const R b3 = (-(f.v - f.c) * d[0] + d[t]) * f.i2c;
      const R b2 = d[n] - f.u * d[0];
      const R l1 = f.v - f.c, l2 = f.v, l3 = f.v + f.c;
      const R m1 = rmin(l1, R(0)) * b1, m2 = rmin(l2, R(0)) * b2, m3 = rmin(l3, R(0)) * b3;
      const R p1 = rmax(l1, R(0)) * b1, p2 = rmax(l2, R(0)) * b2, p3 = rmax(l3, R(0)) * b3;
      bm[0] = m1 + m3;
      bm[n] = (m1 + m3) * f.u + m2;
      bm[t] = m1 * l1 + m3 * l3;
      bp[0] = p1 + p3;
      bp[n] = (p1 + p3) * f.u + p2;
      bp[t] = p1 * l1 + p3 * l3;
    }
  }

  __device__ __forceinline__ double cell_speed(const R* q, const R*, double rdx, double rdy) const {
    const double h = (double)q[0];
    const double c = sqrt((double)g * h);
    double s = (fabs((double)q[1] / h) + c) * rdx;
    if (NDIM == 2) s = fmax(s, (fabs((double)q[2] / h) + c) * rdy);
    return s;
  }
};

// ---------------------------------------------------------------------------
// 2D linear elasticity with variable coefficients (LeVeque 2002, ch. 22,
// decomposed as for variable-coefficient acoustics, ch. 9).
// q = (s11, s22, s12, u, v); aux = (rho, lambda, mu).  Waves: left P
// (speed -cp_l), left S (-cs_l), right S (+cs_r), right P (+cp_r); left-going
// waves carry the left material's eigenvectors, right-going the right's; the
// jump in the other normal stress sits in a stationary wave that moves nothing.
// ---------------------------------------------------------------------------
template <typename R>
struct Elastic {
  static constexpr int M = 5, MW = 4, NA = 3;
  static constexpr bool kSource = false;
  struct Cell {
    R lam, mu, a, cp, cs;   // Lame parameters, lambda + 2 mu, P and S speeds
  };
  struct Face {};
  __device__ explicit Elastic(const GridDesc&) {}
  // index map for direction D: normal stress, other normal stress, shear,
  // normal velocity, tangential velocity
  static constexpr int SN(int D) { return D == 0 ? 0 : 1; }
  static constexpr int SO(int D) { return D == 0 ? 1 : 0; }
  static constexpr int SH = 2;
  static constexpr int VN(int D) { return D == 0 ? 3 : 4; }
  static constexpr int VT(int D) { return D == 0 ? 4 : 3; }
  template <int D>
  static constexpr bool nz(int p, int k) {
    return (p == 0 || p == 3) ? (k == SN(D) || k == SO(D) || k == VN(D)) : (k == SH || k == VT(D));
  }
  static constexpr bool odd(int d, int k) { return k == 2 || k == 3 + d; }

  __device__ __forceinline__ Cell cell(const R*, const R* a) const {
    Cell m;
    m.lam = a[1];
    m.mu = a[2];
    m.a = a[1] + R(2) * a[2];
    const R ir = frcp(a[0]);
    m.cp = fsqrt(m.a * ir);
    m.cs = fsqrt(a[2] * ir);
    return m;
  }
  __device__ __forceinline__ static Cell shfl_prev_cell(const Cell& c) {
    return Cell{shfl_prev(c.lam), shfl_prev(c.mu), shfl_prev(c.a), shfl_prev(c.cp), shfl_prev(c.cs)};
  }
  __device__ __forceinline__ static Cell shfl_next_cell(const Cell& c) {
    return Cell{shfl_next(c.lam), shfl_next(c.mu), shfl_next(c.a), shfl_next(c.cp), shfl_next(c.cs)};
  }
  __device__ __forceinline__ static Face shfl_next_face(const Face& f) { return f; }

  template <int D>
  __device__ __forceinline__ void normal(const R* ql, const R* qr, const Cell& L, const Cell& Rm,
                                         R (&W)[MW][M], R (&s)[MW], R (&am)[M], R (&ap)[M],
                                         Face&) const {
    constexpr int sn = SN(D), so = SO(D), vn = VN(D), vt = VT(D);
    R dq[M];
#pragma unroll
    for (int k = 0; k < M; ++k) dq[k] = qr[k] - ql[k];
    const R iD1 = frcp(L.a * Rm.cp + Rm.a * L.cp);
    const R a1 = (Rm.cp * dq[sn] + Rm.a * dq[vn]) * iD1;
    const R a4 = (L.cp * dq[sn] - L.a * dq[vn]) * iD1;
    const R iDs = frcp(L.mu * Rm.cs + Rm.mu * L.cs);
    const R a2 = (Rm.cs * dq[SH] + Rm.mu * dq[vt]) * iDs;
    const R a3 = (L.cs * dq[SH] - L.mu * dq[vt]) * iDs;
#pragma unroll
    for (int p = 0; p < MW; ++p)
#pragma unroll
      for (int k = 0; k < M; ++k) W[p][k] = R(0);
    W[0][sn] = a1 * L.a; W[0][so] = a1 * L.lam; W[0][vn] = a1 * L.cp;
    W[1][SH] = a2 * L.mu; W[1][vt] = a2 * L.cs;
    W[2][SH] = a3 * Rm.mu; W[2][vt] = -a3 * Rm.cs;
    W[3][sn] = a4 * Rm.a; W[3][so] = a4 * Rm.lam; W[3][vn] = -a4 * Rm.cp;
    s[0] = -L.cp; s[1] = -L.cs; s[2] = Rm.cs; s[3] = Rm.cp;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      am[k] = s[0] * W[0][k] + s[1] * W[1][k];
      ap[k] = s[2] * W[2][k] + s[3] * W[3][k];
    }
  }

  // Transverse split of a fluctuation living in cell C with neighbours Mm
  // (lower) and P (upper) in the transverse direction.
  template <int D>
  __device__ __forceinline__ void transverse(const Face&, const Cell& Mm, const Cell& C,
                                             const Cell& P, const R* d, R* bm, R* bp) const {
    constexpr int T = 1 - D;
    constexpr int sn = SN(T), so = SO(T), vn = VN(T), vt = VT(T);
    const R b1 = (C.cp * d[sn] + C.a * d[vn]) * frcp(Mm.a * C.cp + C.a * Mm.cp);
    const R b2 = (C.cs * d[SH] + C.mu * d[vt]) * frcp(Mm.mu * C.cs + C.mu * Mm.cs);
    const R b3 = (C.cs * d[SH] - C.mu * d[vt]) * frcp(C.mu * P.cs + P.mu * C.cs);
    const R b4 = (C.cp * d[sn] - C.a * d[vn]) * frcp(C.a * P.cp + P.a * C.cp);
    bm[sn] = -Mm.cp * b1 * Mm.a;
    bm[so] = -Mm.cp * b1 * Mm.lam;
    bm[vn] = -Mm.cp * b1 * Mm.cp;
    bm[SH] = -Mm.cs * b2 * Mm.mu;
    bm[vt] = -Mm.cs * b2 * Mm.cs;
    bp[SH] = P.cs * b3 * P.mu;
    bp[vt] = -P.cs * b3 * P.cs;
    bp[sn] = P.cp * b4 * P.a;
    bp[so] = P.cp * b4 * P.lam;
    bp[vn] = -P.cp * b4 * P.cp;
  }

  __device__ __forceinline__ double cell_speed(const R*, const R* a, double rdx, double rdy) const {
    const double cp = sqrt(((double)a[1] + 2.0 * (double)a[2]) / (double)a[0]);
    return fmax(cp * rdx, cp * rdy);
  }
};

// ---------------------------------------------------------------------------
// Wave limiters (LeVeque 2002, ch. 6): phi(theta) for theta = num/den.
// den = W.W.  A wave whose W.W is below kTinyNorm (|W| < 1e-100 in FP64,
// 1e-15 in FP32) is limited to zero: its correction is far below rounding of
// any state value, and the reciprocal estimate of a subnormal norm would not
// be finite.
// ---------------------------------------------------------------------------
template <typename R> struct TinyNorm;
template <> struct TinyNorm<double> { static constexpr double v = 1e-200; };
template <> struct TinyNorm<float> { static constexpr float v = 1e-30f; };

template <typename R>
__device__ __forceinline__ R limiter_phi(int lim, R num, R den) {
  if (lim == 0) return R(1);
  const bool ok = den > TinyNorm<R>::v;
  const R th = num * frcp(ok ? den : R(1));
  const R phi = lim == 1 ? rmax(R(0), rmin(R(1), th))
                         : rmax(R(0), rmin(rmin((R(1) + th) * R(0.5), R(2)), R(2) * th));
  return ok ? phi : R(0);
}

// The same with the limiter fixed at compile time (no branches).
template <int LIM, typename R>
__device__ __forceinline__ R limiter_phi_t(R num, R den) {
  if constexpr (LIM == 0) {
    return R(1);
  } else {
    const bool ok = den > TinyNorm<R>::v;
    const R th = num * frcp(ok ? den : R(1));
    R phi;
    if constexpr (LIM == 1)
      phi = rmax(R(0), rmin(R(1), th));
    else
      phi = rmax(R(0), rmin(rmin((R(1) + th) * R(0.5), R(2)), R(2) * th));
    return ok ? phi : R(0);
  }
}

// ---------------------------------------------------------------------------
// Euler equations, Roe solver (LeVeque 2002, ch. 15; the 2D system adds a
// shear wave), optional passive tracer phi advected at the Roe velocity, and
// an optional Harten-Hyman entropy fix on the acoustic waves.
// q = (rho, rho u, [rho v,] E [, phi]).  For a face normal to D the waves are
//   0 acoustic  a1 (1, u-c, v, H - u c)      speed u - c
//   1 entropy   a2 (1, u,   v, (u^2+v^2)/2)  speed u
//   2 shear     a3 (0, 0,   1, v)    [2D]    speed u
//   . acoustic  a4 (1, u+c, v, H + u c)      speed u + c
//   . tracer    d_phi e_phi          [opt]   speed u
// in (rho, normal, tangential, E) order with Roe averages u (normal), v
// (tangential), H, c; a3 = d_t - v d_rho, a2 = (gamma-1)/c^2 ((H - u^2 - v^2)
// d_rho + u d_n + v d_t - d_E), a4 = (d_n + (c - u) d_rho - c a2) / (2c),
// a1 = d_rho - a2 - a4.  2D axisymmetric flows (z = x, r = y) add the
// geometric source of eq. euler-rz as a fractional step (Heun's method).
// ---------------------------------------------------------------------------
template <typename R, int NDIM, bool TRACER>
struct EulerRoe {
  static constexpr int M = 2 + NDIM + (TRACER ? 1 : 0);
  static constexpr int MW = M;
  static constexpr int NA = 0;
  static constexpr int EI = 1 + NDIM;                  // energy
  static constexpr int PHI = TRACER ? 2 + NDIM : -1;   // tracer
  static constexpr int ACR = NDIM == 2 ? 3 : 2;        // right acoustic wave
  static constexpr bool kSource = NDIM == 2;
  struct Cell {
    R u, v, sr, H, c;   // velocities, sqrt(rho), enthalpy, sound speed
  };
  struct Face {
    R un, ut, H, c, q2, i2c, g1c2;   // Roe averages; 1/(2c); (gamma-1)/c^2
  };
  R gamma, g1;
  int efix;
  __device__ explicit EulerRoe(const GridDesc& G)
      : gamma((R)G.pd[0]), g1((R)G.pd[0] - R(1)), efix(G.efix) {}

  template <int D>
  static constexpr bool nz(int p, int k) {
    if (TRACER && (p == M - 1 || k == M - 1)) return p == M - 1 && k == M - 1;
    if (NDIM == 2 && p == 2) return k == 2 - D || k == EI;   // shear: tangential momentum, E
    return true;
  }
  static constexpr bool odd(int d, int k) { return k == 1 + d; }

  __device__ __forceinline__ Cell cell(const R* q, const R*) const {
    const R is = frsq(q[0]);           // 1/sqrt(rho)
    const R ir = is * is;
    Cell c;
    c.sr = q[0] * is;
    c.u = q[1] * ir;
    c.v = NDIM == 2 ? q[2] * ir : R(0);
    const R p = g1 * (q[EI] - R(0.5) * (q[1] * c.u + (NDIM == 2 ? q[2] * c.v : R(0))));
    c.H = (q[EI] + p) * ir;
    c.c = fsqrt(gamma * p * ir);
    return c;
  }
  __device__ __forceinline__ static Cell shfl_prev_cell(const Cell& c) {
    return Cell{shfl_prev(c.u), NDIM == 2 ? shfl_prev(c.v) : R(0), shfl_prev(c.sr), shfl_prev(c.H),
                shfl_prev(c.c)};
  }
  __device__ __forceinline__ static Cell shfl_next_cell(const Cell& c) {
    return Cell{shfl_next(c.u), NDIM == 2 ? shfl_next(c.v) : R(0), shfl_next(c.sr), shfl_next(c.H),
                shfl_next(c.c)};
  }
  __device__ __forceinline__ static Face shfl_next_face(const Face& f) {
    return Face{shfl_next(f.un), shfl_next(f.ut), shfl_next(f.H), shfl_next(f.c), shfl_next(f.q2),
                shfl_next(f.i2c), shfl_next(f.g1c2)};
  }

  // normal velocity, pressure of a state in the frame of a face normal to D
  template <int D>
  __device__ __forceinline__ void prim(const R* q, R& un, R& p) const {
    constexpr int n = 1 + D, t = 2 - D;
    const R ir = frcp(q[0]);
    un = q[n] * ir;
    const R kin = q[n] * q[n] + (NDIM == 2 ? q[t] * q[t] : R(0));
    p = g1 * (q[EI] - R(0.5) * kin * ir);
  }

  template <int D>
  __device__ __forceinline__ void normal(const R* ql, const R* qr, const Cell& cl, const Cell& cr,
                                         R (&W)[MW][M], R (&s)[MW], R (&am)[M], R (&ap)[M],
                                         Face& f) const {
    constexpr int n = 1 + D, t = 2 - D;
    const R unl = D == 0 ? cl.u : cl.v, unr = D == 0 ? cr.u : cr.v;
    const R rden = frcp(cl.sr + cr.sr);
    f.un = (cl.sr * unl + cr.sr * unr) * rden;
    if constexpr (NDIM == 2) {
      const R utl = D == 0 ? cl.v : cl.u, utr = D == 0 ? cr.v : cr.u;
      f.ut = (cl.sr * utl + cr.sr * utr) * rden;
    } else {
      f.ut = R(0);
    }
    f.H = (cl.sr * cl.H + cr.sr * cr.H) * rden;
    f.q2 = f.un * f.un + f.ut * f.ut;
    const R c2 = g1 * (f.H - R(0.5) * f.q2);
    const R rs = frsq(c2);
    f.c = c2 * rs;
    f.i2c = R(0.5) * rs;
    f.g1c2 = g1 * rs * rs;
    R dq[M];
#pragma unroll
    for (int k = 0; k < M; ++k) dq[k] = qr[k] - ql[k];
    const R dtn = NDIM == 2 ? dq[t] : R(0);
    const R a2 = f.g1c2 * ((f.H - f.q2) * dq[0] + f.un * dq[n] + f.ut * dtn - dq[EI]);
    const R a4 = (dq[n] + (f.c - f.un) * dq[0] - f.c * a2) * f.i2c;
    const R a1 = dq[0] - a2 - a4;
#pragma unroll
    for (int p = 0; p < MW; ++p)
#pragma unroll
      for (int k = 0; k < M; ++k) W[p][k] = R(0);
    W[0][0] = a1; W[0][n] = a1 * (f.un - f.c); W[0][EI] = a1 * (f.H - f.un * f.c);
    W[1][0] = a2; W[1][n] = a2 * f.un; W[1][EI] = a2 * R(0.5) * f.q2;
    W[ACR][0] = a4; W[ACR][n] = a4 * (f.un + f.c); W[ACR][EI] = a4 * (f.H + f.un * f.c);
    s[0] = f.un - f.c;
    s[1] = f.un;
    s[ACR] = f.un + f.c;
    if constexpr (NDIM == 2) {
      const R a3 = dq[t] - f.ut * dq[0];
      W[0][t] = a1 * f.ut;
      W[1][t] = a2 * f.ut;
      W[ACR][t] = a4 * f.ut;
      W[2][t] = a3;
      W[2][EI] = a3 * f.ut;
      s[2] = f.un;
    }
    if constexpr (TRACER) {
      W[M - 1][PHI] = dq[PHI];
      s[M - 1] = f.un;
    }
    R coef[MW];
#pragma unroll
    for (int p = 0; p < MW; ++p) coef[p] = rmin(s[p], R(0));
    if (efix) {
      // Harten-Hyman: a transonic acoustic rarefaction (characteristic speed
      // negative on its left, positive on its right) contributes
      // lam_l (lam_r - s) / (lam_r - lam_l) W to A^-dQ.  The middle state's
      // speed is formed only when a cheap exact test (u_m > c_m, i.e.
      // m_n > 0 and m_n^2 > gamma p_m rho_m) says the wave is transonic.
      {
        const R lam_l = unl - cl.c;
        R qm[M];
#pragma unroll
        for (int k = 0; k < M; ++k) qm[k] = ql[k] + W[0][k];
        const R kin = qm[n] * qm[n] + (NDIM == 2 ? qm[t] * qm[t] : R(0));
        const R prho = g1 * (qm[EI] * qm[0] - R(0.5) * kin);   // p_m rho_m
        if (lam_l < R(0) && qm[0] > R(0) && prho > R(0) && qm[n] > R(0) &&
            qm[n] * qm[n] > gamma * prho) {
          R um, pm;
          prim<D>(qm, um, pm);
          const R lam_r = um - fsqrt(gamma * pm * frcp(qm[0]));
          if (R(0) < lam_r) coef[0] = lam_l * (lam_r - s[0]) * frcp(lam_r - lam_l);
        }
      }
      {
        const R lam_r = unr + cr.c;
        R qm[M];
#pragma unroll
        for (int k = 0; k < M; ++k) qm[k] = qr[k] - W[ACR][k];
        const R kin = qm[n] * qm[n] + (NDIM == 2 ? qm[t] * qm[t] : R(0));
        const R prho = g1 * (qm[EI] * qm[0] - R(0.5) * kin);
        if (lam_r > R(0) && qm[0] > R(0) && prho > R(0) && qm[n] < R(0) &&
            qm[n] * qm[n] > gamma * prho) {
          R um, pm;
          prim<D>(qm, um, pm);
          const R lam_l = um + fsqrt(gamma * pm * frcp(qm[0]));
          if (lam_l < R(0)) coef[ACR] = lam_l * (lam_r - s[ACR]) * frcp(lam_r - lam_l);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
      R a = R(0), sw = R(0);
#pragma unroll
      for (int p = 0; p < MW; ++p) {
        if (!nz<D>(p, k)) continue;
        a += coef[p] * W[p][k];
        sw += s[p] * W[p][k];
      }
      am[k] = a;
      ap[k] = sw - a;
    }
  }

  // Split a fluctuation from a face normal to D in the transverse direction
  // with the face's Roe averages: speeds v-c, v, v, v+c (and v for the
  // tracer), v being the velocity along the transverse direction.
  template <int D>
  __device__ __forceinline__ void transverse(const Face& f, const Cell&, const Cell&, const Cell&,
                                             const R* d, R* bm, R* bp) const {
    if constexpr (NDIM == 2) {
      constexpr int n = 1 + D, t = 2 - D;
      const R b3 = d[n] - f.un * d[0];
      const R b2 = f.g1c2 * ((f.H - f.q2) * d[0] + f.un * d[n] + f.ut * d[t] - d[EI]);
      const R b4 = (d[t] + (f.c - f.ut) * d[0] - f.c * b2) * f.i2c;
      const R b1 = d[0] - b2 - b4;
      const R l1 = f.ut - f.c, l2 = f.ut, l4 = f.ut + f.c;
      const R m1 = rmin(l1, R(0)) * b1, m2 = rmin(l2, R(0)) * b2, m3 = rmin(l2, R(0)) * b3,
              m4 = rmin(l4, R(0)) * b4;
      const R p1 = rmax(l1, R(0)) * b1, p2 = rmax(l2, R(0)) * b2, p3 = rmax(l2, R(0)) * b3,
              p4 = rmax(l4, R(0)) * b4;
      // eigenvectors (rho, across, along, E): (1, u, v-c, H - v c), (1, u, v, q2/2),
      // (0, 1, 0, u), (1, u, v+c, H + v c)
      const R hq = R(0.5) * f.q2;
      bm[0] = m1 + m2 + m4;
      bm[n] = (m1 + m2 + m4) * f.un + m3;
      bm[t] = m1 * l1 + m2 * l2 + m4 * l4;
      bm[EI] = m1 * (f.H - f.ut * f.c) + m2 * hq + m3 * f.un + m4 * (f.H + f.ut * f.c);
      bp[0] = p1 + p2 + p4;
      bp[n] = (p1 + p2 + p4) * f.un + p3;
      bp[t] = p1 * l1 + p2 * l2 + p4 * l4;
      bp[EI] = p1 * (f.H - f.ut * f.c) + p2 * hq + p3 * f.un + p4 * (f.H + f.ut * f.c);
      if constexpr (TRACER) {
        bm[PHI] = rmin(l2, R(0)) * d[PHI];
        bp[PHI] = rmax(l2, R(0)) * d[PHI];
      }
    }
  }

  // Axisymmetric geometric source -(v/r)(rho, rho u, rho v, E + p) (tracer 0)
  // over dt by Heun's method: the increment dt/2 (psi(q) + psi(q + dt psi(q))).
  __device__ __forceinline__ void psi(const R* q, R ir, R* out) const {
    const R irho = frcp(q[0]);
    const R v = q[2] * irho;
    const R p = g1 * (q[3] - R(0.5) * (q[1] * q[1] + q[2] * q[2]) * irho);
    const R w = -v * ir;
    out[0] = w * q[0];
    out[1] = w * q[1];
    out[2] = w * q[2];
    out[3] = w * (q[3] + p);
  }
  __device__ __forceinline__ void source_increment(const R* q, R ir, R dt, R* inc) const {
    R f0[4], f1[4], qs[4];
    psi(q, ir, f0);
#pragma unroll
    for (int k = 0; k < 4; ++k) qs[k] = q[k] + dt * f0[k];
    psi(qs, ir, f1);
#pragma unroll
    for (int k = 0; k < 4; ++k) inc[k] = R(0.5) * dt * (f0[k] + f1[k]);
  }

  __device__ __forceinline__ double cell_speed(const R* q, const R*, double rdx, double rdy) const {
    const double rho = q[0], u = (double)q[1] / rho;
    const double v = NDIM == 2 ? (double)q[2] / rho : 0.0;
    const double p = ((double)gamma - 1.0) * ((double)q[EI] - 0.5 * rho * (u * u + v * v));
    const double c = sqrt((double)gamma * p / rho);
    double s = (fabs(u) + c) * rdx;
    if (NDIM == 2) s = fmax(s, (fabs(v) + c) * rdy);
    return s;
  }
};

// ===========================================================================
// SharpClaw: numerical fluxes at an interface from reconstructed edge values.
// ===========================================================================

// Upwind flux for scalar advection.
template <typename R, int NDIM>
struct AdvectionFlux {
  static constexpr int M = 1, NA = 0;
  R u, v;
  __device__ explicit AdvectionFlux(const GridDesc& G) : u((R)G.pd[0]), v((R)G.pd[1]) {}
  static constexpr bool odd(int, int) { return false; }
  template <int D>
  __device__ __forceinline__ R flux(const R* ql, const R* qr, R* F) const {
    const R un = D == 0 ? u : v;
    F[0] = un > R(0) ? un * ql[0] : un * qr[0];
    return rabs(un);
  }
  __device__ __forceinline__ double cell_speed(const R*, const R*, double rdx, double rdy) const {
    double s = fabs((double)u) * rdx;
    if (NDIM == 2) s = fmax(s, fabs((double)v) * rdy);
    return s;
  }
};

// Euler equations, HLLE flux (Einfeldt) with Roe-average wave-speed bounds.
// q = (rho, rho u, E) in 1D, (rho, rho u, rho v, E) in 2D.
template <typename R, int NDIM>
struct EulerHLLE {
  static constexpr int M = NDIM == 1 ? 3 : 4, NA = 0;
  R gamma, gm1;
  __device__ explicit EulerHLLE(const GridDesc& G) : gamma((R)G.pd[0]), gm1((R)G.pd[0] - R(1)) {}
  static constexpr bool odd(int d, int k) { return k == 1 + d; }

  template <int D>
  __device__ __forceinline__ R flux(const R* ql, const R* qr, R* F) const {
    constexpr int E = M - 1;
    const R rl = ql[0], rr = qr[0];
    // 1/sqrt(rho) gives sqrt(rho) and 1/rho together
    const R isl = frsq(rl), isr = frsq(rr);
    const R wl = rl * isl, wr = rr * isr;
    const R irl = isl * isl, irr = isr * isr;
    const R ul = ql[1] * irl, ur = qr[1] * irr;
    const R vl = NDIM == 2 ? ql[2] * irl : R(0);
    const R vr = NDIM == 2 ? qr[2] * irr : R(0);
    const R pl = gm1 * (ql[E] - R(0.5) * rl * (ul * ul + vl * vl));
    const R pr = gm1 * (qr[E] - R(0.5) * rr * (ur * ur + vr * vr));
    const R cl = fsqrt(gamma * pl * irl), cr = fsqrt(gamma * pr * irr);
    const R unl = D == 0 ? ul : vl, unr = D == 0 ? ur : vr;
    const R iw = frcp(wl + wr);
    const R ut = (wl * ul + wr * ur) * iw;
    const R vt = (wl * vl + wr * vr) * iw;
    const R Ht = (wl * ((ql[E] + pl) * irl) + wr * ((qr[E] + pr) * irr)) * iw;
    const R ct = fsqrt(gm1 * (Ht - R(0.5) * (ut * ut + vt * vt)));
    const R unt = D == 0 ? ut : vt;
    const R s1 = rmin(unl - cl, unt - ct);
    const R s2 = rmax(unr + cr, unt + ct);
    R fl[M], fr[M];
    fl[0] = rl * unl;
    fr[0] = rr * unr;
    fl[1] = ql[1] * unl;
    fr[1] = qr[1] * unr;
    if constexpr (NDIM == 2) {
      fl[2] = ql[2] * unl;
      fr[2] = qr[2] * unr;
    }
    fl[1 + D] += pl;
    fr[1 + D] += pr;
    fl[E] = (ql[E] + pl) * unl;
    fr[E] = (qr[E] + pr) * unr;
    if (s1 >= R(0)) {
#pragma unroll
      for (int k = 0; k < M; ++k) F[k] = fl[k];
    } else if (s2 <= R(0)) {
#pragma unroll
      for (int k = 0; k < M; ++k) F[k] = fr[k];
    } else {
      const R inv = frcp(s2 - s1);
      const R s12 = s1 * s2;
#pragma unroll
      for (int k = 0; k < M; ++k)
        F[k] = mul_rounded(s2 * fl[k] - s1 * fr[k] + s12 * (qr[k] - ql[k]), inv);
    }
    return max_nan(rabs(s1), rabs(s2));
  }

  __device__ __forceinline__ double cell_speed(const R* q, const R*, double rdx, double rdy) const {
    const double rho = q[0], u = (double)q[1] / rho;
    const double v = NDIM == 2 ? (double)q[2] / rho : 0.0;
    const double p = ((double)gamma - 1.0) * ((double)q[M - 1] - 0.5 * rho * (u * u + v * v));
    const double c = sqrt((double)gamma * p / rho);
    double s = (fabs(u) + c) * rdx;
    if (NDIM == 2) s = fmax(s, (fabs(v) + c) * rdy);
    return s;
  }
};

// Nonlinear p-system with spatially varying coefficients (Section 7.3,
// eq. p-system), q = (strain eps, rho u[, rho v]), aux = (K, rho) per cell,
// stress sigma = exp(K eps) - 1.  Interface flux from the f-wave split of
// the flux jump (left-going wave on the left material's eigenvector
// (1, Z_l e_n), right-going on the right's (1, -Z_r e_n), Z = rho c,
// c = sqrt(K exp(K eps) / rho)), written in its symmetric closed form:
//   F_0 = -(Z_l u_l + Z_r u_r + sigma_r - sigma_l) / (Z_l + Z_r)
//   F_n = -(Z_r sigma_l + Z_l sigma_r + Z_l Z_r (u_r - u_l)) / (Z_l + Z_r)
// (the interface velocity and stress of the linearised impedance problem),
// the transverse momentum's flux 0.  Speed max(c_l, c_r).
template <typename R, int NDIM>
struct PSystem {
  static constexpr int M = NDIM == 1 ? 2 : 3, NA = 2;
  __device__ explicit PSystem(const GridDesc&) {}
  static constexpr bool odd(int d, int k) { return k == 1 + d; }

  __device__ __forceinline__ static R em1(R x) {
    if constexpr (sizeof(R) == 8) return expm1(x);
    else return expm1f(x);
  }

  template <int D>
  __device__ __forceinline__ R flux(const R* ql, const R* qr, const R* al, const R* ar,
                                    R* F) const {
    constexpr int N = 1 + D;
    const R Kl = al[0], rl = al[1], Kr = ar[0], rr = ar[1];
    const R sl = em1(Kl * ql[0]), sr = em1(Kr * qr[0]);
    // Z = rho c = sqrt(K exp(K eps) rho), c = Z / rho
    const R irl = frcp(rl), irr = frcp(rr);
    const R Zl = fsqrt(Kl * (sl + R(1)) * rl), Zr = fsqrt(Kr * (sr + R(1)) * rr);
    const R ul = ql[N] * irl, ur = qr[N] * irr;
    const R iz = frcp(Zl + Zr);
    F[0] = mul_rounded(-(Zl * ul + Zr * ur + (sr - sl)), iz);
    F[N] = mul_rounded(-(Zr * sl + Zl * sr + Zl * Zr * (ur - ul)), iz);
    if constexpr (NDIM == 2) F[3 - N] = R(0);
    return rmax(Zl * irl, Zr * irr);
  }

  __device__ __forceinline__ double cell_speed(const R* q, const R* a, double rdx,
                                               double rdy) const {
    const double K = a[0], rho = a[1];
    const double c = sqrt(K * exp(K * (double)q[0]) / rho);
    return NDIM == 2 ? fmax(c * rdx, c * rdy) : c * rdx;
  }
};

// WENO5 (Jiang-Shu), component-wise: from the five cell averages centred on
// cell i, the value at its right edge (qL, the left state of face i+1/2) and
// at its left edge (qR, the right state of face i-1/2).  Everything is
// written in the first differences da..dd of the window:
//  - smoothness indicators: 13/12 t^2 + 1/4 u^2 with t the stencil's second
//    difference and u its one-sided derivative term; the weights use
//    4 (eps + beta_k) = 4 eps + 13/3 t^2 + u^2, which leaves the normalised
//    weights unchanged;
//  - with D_k = (4 eps + 4 beta_k)^2, the weights d_k/D_k / sum_j d_j/D_j
//    equal d_k P_k / sum_j d_j P_j, P_k = prod_{j != k} D_j, so each edge
//    needs one reciprocal; the linear weights (1, 6, 3)/10 of the right edge
//    and (3, 6, 1)/10 of the left share 6 P_1 and are not normalised;
//  - the three candidate edge values, times 6, relative to the centre value:
//    the result is v0 plus a weighted correction, so the differences, not
//    the values, carry the rounding.
// The same from the centre value and the window's four first differences
// da = v(-1) - v(-2), db = v(0) - v(-1), dc = v(1) - v(0), dd = v(2) - v(1)
// (a caller that has them from its neighbours passes them directly).
template <typename R>
__device__ __forceinline__ void weno5_edges_d(R v0, R da, R db, R dc, R dd, R eps, R& qL, R& qR) {
  const R t0 = db - da, t1 = dc - db, t2 = dd - dc;
  const R u0 = R(3) * db - da, u1 = db + dc, u2 = dd - R(3) * dc;
  const R c = R(13.0 / 3.0), e4 = R(4) * eps;
  const R e0 = (c * t0) * t0 + (u0 * u0 + e4);
  const R e1 = (c * t1) * t1 + (u1 * u1 + e4);
  const R e2 = (c * t2) * t2 + (u2 * u2 + e4);
  const R D0 = e0 * e0, D1 = e1 * e1, D2 = e2 * e2;
  const R P0 = D1 * D2, A1 = R(6) * (D0 * D2), P2 = D0 * D1;
  const R A2 = R(3) * P2, B0 = R(3) * P0;
  // 6 (candidate - v0): right edge l0..l2, left edge r0..r2
  const R l0 = R(5) * db - R(2) * da, l1 = db + R(2) * dc, l2 = R(4) * dc - dd;
  const R r0 = da - R(4) * db, r1 = -(R(2) * db + dc), r2 = R(2) * dd - R(5) * dc;
  const R nL = P0 * l0 + A1 * l1 + A2 * l2, sL = P0 + A1 + A2;
  const R nR = B0 * r0 + A1 * r1 + P2 * r2, sR = B0 + A1 + P2;
  qL = v0 + nL * (R(1.0 / 6.0) * frcp(sL));
  qR = v0 + nR * (R(1.0 / 6.0) * frcp(sR));
}

template <typename R>
__device__ __forceinline__ void weno5_edges(R vm2, R vm1, R v0, R vp1, R vp2, R eps, R& qL, R& qR) {
  weno5_edges_d(v0, vm1 - vm2, v0 - vm1, vp1 - v0, vp2 - vp1, eps, qL, qR);
}

}  // namespace claw
