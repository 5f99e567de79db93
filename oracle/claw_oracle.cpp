// claw_oracle.cpp -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 CPU implementation of one finite-volume time step for
// q_t + f(q)_x + g(q)_y = 0 on a uniform Cartesian grid, in the two forms the
// PyClaw paper describes (Section 2, "Finite Volume Hyperbolic PDE solvers",
// and Section 2.1, "Clawpack and SharpClaw"):
//
//   * classic Clawpack wave propagation (Riemann solvers: advection, shallow
//     water Roe, Euler Roe with an optional tracer, elasticity): a Riemann
//     solve at every interface,
//     waves limited by the upwind neighbour, a second-order correction flux
//     (eq. lwflux: F = F_upwind + F_correction, first-order part written as
//     fluctuations) and, in 2D, the unsplit transverse corrections computed by
//     a secondary "transverse" Riemann solver; a geometric source term (the
//     axisymmetric Euler equations, eq. euler-rz) is applied by a fractional
//     step after the hyperbolic update (Section 2.1, source terms by
//     operator splitting);
//   * SharpClaw method of lines: WENO edge values (fifth order, or any odd
//     order 2r-1 from the general definition), an interface Riemann flux and
//     flux differencing (eq. fluxdiff), inside SSP Runge-Kutta stages
//     (Shu-Osher SSPRK(3,3), or the ten-stage fourth-order SSP method with a
//     two-register implementation that SharpClaw uses by default).
//
// The paper prints none of the Riemann solvers, limiters, WENO weights or RK
// coefficients; it defers to LeVeque (1997, 2002), Jiang-Shu and Shu-Osher.
// The formulas below are those published definitions written out plainly.
// Every choice the paper leaves open is fixed once here and listed in the
// design notes of the repository (entropy fix form, transverse factor, WENO
// epsilon, Courant number definition, step controller).
//
// Nothing in the GPU library may include, link or call this file; it exists
// so tests and the CPU baseline can check the GPU results against it.  It is
// compiled with -O2 -ffp-contract=off and no fast-math.
//
// Layout of every array: component-major, x fastest: q[k][j][i],
// k = component, j = row (y), i = column (x); interior cells only.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

extern "C" {

// Problem description (the oracle's own struct; the GPU library has its own).
struct OCfg {
  int ndim;            // 1 or 2
  int nx, ny;          // interior cells (ny = 1 in 1D)
  double xlo, xhi, ylo, yhi;
  int scheme;          // 1 classic wave propagation, 2 SharpClaw (WENO5 + SSPRK(3,3))
  int solver;          // 1 advection, 2 shallow water Roe, 3 Euler HLLE, 4 elasticity (variable coeff.)
  int limiter;         // 0 none (Lax-Wendroff), 1 minmod, 2 MC
  int transverse;      // 0 none, 1 fluctuations, 2 full (fluctuations -/+ second-order term)
  int efix;            // 1: Harten-Hyman entropy fix in the shallow-water Roe solver
  int bc[4];           // x-lower, x-upper, y-lower, y-upper: 1 extrap, 2 periodic, 3 wall, 4 Dirichlet
  double bcstate[4][8];// Dirichlet state per side
  double weno_eps;     // WENO epsilon
  double pd[8];        // problem data: advection (u, v); shallow water (g); Euler (gamma)
  int integrator;      // SharpClaw: 0/1 SSPRK(3,3), 2 SSPRK(10,4)
  int weno_order;      // SharpClaw: 0/5 WENO5, or 2r-1 for r = 3..9
  int tracer;          // Euler Roe: 1 = one passive tracer advected with the flow
  int source;          // classic 2D Euler Roe: 1 = axisymmetric about y = 0 (r = y)
  int split;           // classic 2D: 0 unsplit, 1 Godunov (x then y), 2 Strang (x/2, y, x/2)
  double cfl_max;      // split steps: a sweep above it ends the step's Courant reading
};

}  // extern "C"

namespace {

enum { S_ADV = 1, S_SW = 2, S_EULER = 3, S_ELASTIC = 4, S_EULER_ROE = 5, S_PSYS = 6 };
enum { BC_EXTRAP = 1, BC_PERIODIC = 2, BC_WALL = 3, BC_DIRICHLET = 4 };

int num_eqn(const OCfg& c) {
  switch (c.solver) {
    case S_ADV: return 1;
    case S_SW: return c.ndim == 1 ? 2 : 3;
    case S_EULER: return c.ndim == 1 ? 3 : 4;
    case S_ELASTIC: return 5;
    case S_EULER_ROE: return (c.ndim == 1 ? 3 : 4) + (c.tracer ? 1 : 0);
    case S_PSYS: return c.ndim == 1 ? 2 : 3;
  }
  return 0;
}
int num_waves(const OCfg& c) {
  switch (c.solver) {
    case S_ADV: return 1;
    case S_SW: return c.ndim == 1 ? 2 : 3;
    case S_EULER: return 2;
    case S_ELASTIC: return 4;
    case S_EULER_ROE: return (c.ndim == 1 ? 3 : 4) + (c.tracer ? 1 : 0);
    case S_PSYS: return 2;
  }
  return 0;
}
int num_aux(const OCfg& c) { return c.solver == S_ELASTIC ? 3 : (c.solver == S_PSYS ? 2 : 0); }

double dx_of(const OCfg& c) { return (c.xhi - c.xlo) / c.nx; }
double dy_of(const OCfg& c) { return c.ndim == 2 ? (c.yhi - c.ylo) / c.ny : 1.0; }

// Components whose sign flips under reflection through a wall normal to
// direction d (the "normal-odd" components).
bool odd_under_reflection(const OCfg& c, int d, int k) {
  switch (c.solver) {
    case S_SW:
    case S_EULER:
    case S_EULER_ROE:
    case S_PSYS: return k == 1 + d;                  // normal momentum
    case S_ELASTIC: return k == 2 || k == 3 + d;      // shear stress and normal velocity
  }
  return false;
}

// Ghost-padded field: g ghost layers in x, and in y when ndim == 2.
struct Field {
  int m = 0, nx = 0, ny = 0, g = 0, gy = 0, NX = 0, NY = 0;
  std::vector<double> v;
  void init(int m_, int nx_, int ny_, int g_, int ndim) {
    m = m_; nx = nx_; ny = ny_; g = g_; gy = ndim == 2 ? g_ : 0;
    NX = nx + 2 * g; NY = ny + 2 * gy;
    v.assign((size_t)std::max(m, 1) * NX * NY, 0.0);
  }
  double& at(int k, int j, int i) { return v[((size_t)k * NY + (j + gy)) * NX + (i + g)]; }
  double at(int k, int j, int i) const { return v[((size_t)k * NY + (j + gy)) * NX + (i + g)]; }
};

// Ghost cells (Section 4, "Parallelization": ghost layers set from the boundary
// conditions before each step).  x ghosts are filled for interior rows first;
// then y ghosts for every column, ghost columns included, so a corner ghost is
// the y-boundary image of an x-ghost.
void fill_ghosts(const OCfg& c, Field& f, bool is_aux) {
  const int nx = f.nx, ny = f.ny, g = f.g;
  auto bc_of = [&](int side) {
    int b = c.bc[side];
    if (is_aux && b == BC_DIRICHLET) b = BC_EXTRAP;   // material data: copy the edge
    return b;
  };
  for (int j = 0; j < ny; ++j)
    for (int kk = 1; kk <= g; ++kk)
      for (int k = 0; k < f.m; ++k) {
        // lower x side, ghost column i = -kk
        switch (bc_of(0)) {
          case BC_EXTRAP: f.at(k, j, -kk) = f.at(k, j, 0); break;
          case BC_PERIODIC: f.at(k, j, -kk) = f.at(k, j, nx - kk); break;
          case BC_WALL: {
            double s = (!is_aux && odd_under_reflection(c, 0, k)) ? -1.0 : 1.0;
            f.at(k, j, -kk) = s * f.at(k, j, kk - 1);
          } break;
          case BC_DIRICHLET: f.at(k, j, -kk) = c.bcstate[0][k]; break;
        }
        // upper x side, ghost column i = nx - 1 + kk
        switch (bc_of(1)) {
          case BC_EXTRAP: f.at(k, j, nx - 1 + kk) = f.at(k, j, nx - 1); break;
          case BC_PERIODIC: f.at(k, j, nx - 1 + kk) = f.at(k, j, kk - 1); break;
          case BC_WALL: {
            double s = (!is_aux && odd_under_reflection(c, 0, k)) ? -1.0 : 1.0;
            f.at(k, j, nx - 1 + kk) = s * f.at(k, j, nx - kk);
          } break;
          case BC_DIRICHLET: f.at(k, j, nx - 1 + kk) = c.bcstate[1][k]; break;
        }
      }
  if (c.ndim != 2) return;
  for (int i = -g; i < nx + g; ++i)
    for (int kk = 1; kk <= g; ++kk)
      for (int k = 0; k < f.m; ++k) {
        switch (bc_of(2)) {
          case BC_EXTRAP: f.at(k, -kk, i) = f.at(k, 0, i); break;
          case BC_PERIODIC: f.at(k, -kk, i) = f.at(k, ny - kk, i); break;
          case BC_WALL: {
            double s = (!is_aux && odd_under_reflection(c, 1, k)) ? -1.0 : 1.0;
            f.at(k, -kk, i) = s * f.at(k, kk - 1, i);
          } break;
          case BC_DIRICHLET: f.at(k, -kk, i) = c.bcstate[2][k]; break;
        }
        switch (bc_of(3)) {
          case BC_EXTRAP: f.at(k, ny - 1 + kk, i) = f.at(k, ny - 1, i); break;
          case BC_PERIODIC: f.at(k, ny - 1 + kk, i) = f.at(k, kk - 1, i); break;
          case BC_WALL: {
            double s = (!is_aux && odd_under_reflection(c, 1, k)) ? -1.0 : 1.0;
            f.at(k, ny - 1 + kk, i) = s * f.at(k, ny - kk, i);
          } break;
          case BC_DIRICHLET: f.at(k, ny - 1 + kk, i) = c.bcstate[3][k]; break;
        }
      }
}

void load_field(const OCfg& c, Field& f, const double* src, int m, int g, bool is_aux) {
  f.init(m, c.nx, c.ny, g, c.ndim);
  if (m == 0) return;
  for (int k = 0; k < m; ++k)
    for (int j = 0; j < c.ny; ++j)
      for (int i = 0; i < c.nx; ++i) f.at(k, j, i) = src[((size_t)k * c.ny + j) * c.nx + i];
  fill_ghosts(c, f, is_aux);
}

// ---------------------------------------------------------------------------
// Riemann solvers (the problem-specific kernels of Section 2.1).  A solve at
// a face normal to direction d takes the left state ql (lower index side) and
// right state qr, and returns waves W^p, speeds s^p and the fluctuations
// A^-dQ, A^+dQ.
// ---------------------------------------------------------------------------

struct FaceSol {
  double W[5][5];
  double s[5];
  double amdq[5], apdq[5];
};

// Scalar advection q_t + u q_x + v q_y = 0: one wave, the jump.
void rp_advection(const OCfg& c, int d, const double* ql, const double* qr, FaceSol& r) {
  const double u = c.pd[d];
  const double dq = qr[0] - ql[0];
  r.W[0][0] = dq;
  r.s[0] = u;
  r.amdq[0] = std::min(u, 0.0) * dq;
  r.apdq[0] = std::max(u, 0.0) * dq;
}

// Shallow water, Roe linearisation (LeVeque 2002, ch. 15; the "Roe solver
// with an entropy fix" of the paper's serial timing study, Section 5).
// q = (h, hu) in 1D, (h, hu, hv) in 2D.  Components: 0 depth, n normal
// momentum, t tangential momentum.
struct RoeSW {
  double ubar, vbar, cbar;   // normal velocity, tangential velocity, celerity
};

RoeSW sw_roe_avg(const OCfg& c, int d, const double* ql, const double* qr) {
  const double gr = c.pd[0];
  const int n = 1 + d, t = 2 - d;
  const double hl = ql[0], hr = qr[0];
  const double sl = std::sqrt(hl), sr = std::sqrt(hr);
  RoeSW a;
  a.ubar = (sl * (ql[n] / hl) + sr * (qr[n] / hr)) / (sl + sr);
  a.vbar = c.ndim == 2 ? (sl * (ql[t] / hl) + sr * (qr[t] / hr)) / (sl + sr) : 0.0;
  a.cbar = std::sqrt(gr * 0.5 * (hl + hr));
  return a;
}

void rp_sw_roe(const OCfg& c, int d, const double* ql, const double* qr, FaceSol& r) {
  const double gr = c.pd[0];
  const int m = num_eqn(c);
  const int n = 1 + d, t = 2 - d;
  const RoeSW a = sw_roe_avg(c, d, ql, qr);
  double dq[3];
  for (int k = 0; k < m; ++k) dq[k] = qr[k] - ql[k];
  const double a1 = ((a.ubar + a.cbar) * dq[0] - dq[n]) / (2.0 * a.cbar);
  const double a3 = (-(a.ubar - a.cbar) * dq[0] + dq[n]) / (2.0 * a.cbar);
  std::memset(r.W, 0, sizeof(r.W));
  // family "first" (left-going acoustic) and "last" (right-going acoustic)
  const int last = m == 2 ? 1 : 2;
  r.W[0][0] = a1; r.W[0][n] = a1 * (a.ubar - a.cbar);
  r.s[0] = a.ubar - a.cbar;
  r.W[last][0] = a3; r.W[last][n] = a3 * (a.ubar + a.cbar);
  r.s[last] = a.ubar + a.cbar;
  if (m == 3) {
    r.W[0][t] = a1 * a.vbar;
    r.W[2][t] = a3 * a.vbar;
    r.W[1][t] = dq[t] - a.vbar * dq[0];   // shear wave
    r.s[1] = a.ubar;
  }
  const int mw = m;
  for (int k = 0; k < m; ++k) { r.amdq[k] = 0.0; r.apdq[k] = 0.0; }
  if (!c.efix) {
    for (int p = 0; p < mw; ++p)
      for (int k = 0; k < m; ++k) {
        r.amdq[k] += std::min(r.s[p], 0.0) * r.W[p][k];
        r.apdq[k] += std::max(r.s[p], 0.0) * r.W[p][k];
      }
    return;
  }
  // Harten-Hyman entropy fix: a transonic rarefaction in an acoustic family
  // splits that wave's contribution between A^- and A^+.
  double coef[3];
  {  // first family: characteristic speed left of and right of the wave
    const double lam_l = ql[n] / ql[0] - std::sqrt(gr * ql[0]);
    const double hm = ql[0] + r.W[0][0], hum = ql[n] + r.W[0][n];
    const double lam_r = hum / hm - std::sqrt(gr * hm);
    if (lam_l < 0.0 && 0.0 < lam_r)
      coef[0] = lam_l * (lam_r - r.s[0]) / (lam_r - lam_l);
    else
      coef[0] = std::min(r.s[0], 0.0);
  }
  if (m == 3) coef[1] = std::min(r.s[1], 0.0);
  {  // last family
    const double hm = qr[0] - r.W[last][0], hum = qr[n] - r.W[last][n];
    const double lam_l = hum / hm + std::sqrt(gr * hm);
    const double lam_r = qr[n] / qr[0] + std::sqrt(gr * qr[0]);
    if (lam_l < 0.0 && 0.0 < lam_r)
      coef[last] = lam_l * (lam_r - r.s[last]) / (lam_r - lam_l);
    else
      coef[last] = std::min(r.s[last], 0.0);
  }
  for (int p = 0; p < mw; ++p)
    for (int k = 0; k < m; ++k) r.amdq[k] += coef[p] * r.W[p][k];
  for (int k = 0; k < m; ++k) {
    double sw = 0.0;
    for (int p = 0; p < mw; ++p) sw += r.s[p] * r.W[p][k];
    r.apdq[k] = sw - r.amdq[k];
  }
}

// Linear elasticity with variable coefficients (LeVeque 2002, ch. 22 system,
// decomposed as for variable-coefficient acoustics, ch. 9).
// q = (s11, s22, s12, u, v); aux = (rho, lambda, mu).
struct Mat {
  double rho, lam, mu, a, cp, cs;
};
Mat material(const double* aux) {
  Mat t;
  t.rho = aux[0]; t.lam = aux[1]; t.mu = aux[2];
  t.a = t.lam + 2.0 * t.mu;
  t.cp = std::sqrt(t.a / t.rho);
  t.cs = std::sqrt(t.mu / t.rho);
  return t;
}
// Index map for direction d: sn normal stress, so other normal stress,
// sh shear stress, vn normal velocity, vt tangential velocity.
struct EIdx { int sn, so, sh, vn, vt; };
EIdx eidx(int d) { return d == 0 ? EIdx{0, 1, 2, 3, 4} : EIdx{1, 0, 2, 4, 3}; }

void rp_elastic(int d, const double* ql, const double* qr, const double* auxl,
                const double* auxr, FaceSol& r) {
  const EIdx e = eidx(d);
  const Mat L = material(auxl), R = material(auxr);
  double dq[5];
  for (int k = 0; k < 5; ++k) dq[k] = qr[k] - ql[k];
  const double D = L.a * R.cp + R.a * L.cp;
  const double a1 = (R.cp * dq[e.sn] + R.a * dq[e.vn]) / D;
  const double a4 = (L.cp * dq[e.sn] - L.a * dq[e.vn]) / D;
  const double Ds = L.mu * R.cs + R.mu * L.cs;
  const double a2 = (R.cs * dq[e.sh] + R.mu * dq[e.vt]) / Ds;
  const double a3 = (L.cs * dq[e.sh] - L.mu * dq[e.vt]) / Ds;
  std::memset(r.W, 0, sizeof(r.W));
  r.W[0][e.sn] = a1 * L.a; r.W[0][e.so] = a1 * L.lam; r.W[0][e.vn] = a1 * L.cp;
  r.s[0] = -L.cp;
  r.W[1][e.sh] = a2 * L.mu; r.W[1][e.vt] = a2 * L.cs;
  r.s[1] = -L.cs;
  r.W[2][e.sh] = a3 * R.mu; r.W[2][e.vt] = -a3 * R.cs;
  r.s[2] = R.cs;
  r.W[3][e.sn] = a4 * R.a; r.W[3][e.so] = a4 * R.lam; r.W[3][e.vn] = -a4 * R.cp;
  r.s[3] = R.cp;
  for (int k = 0; k < 5; ++k) {
    r.amdq[k] = r.s[0] * r.W[0][k] + r.s[1] * r.W[1][k];
    r.apdq[k] = r.s[2] * r.W[2][k] + r.s[3] * r.W[3][k];
  }
}

// Euler equations, Roe solver (LeVeque 2002, ch. 15 for the 1D system; in 2D
// the tangential momentum adds a shear wave).  q = (rho, rho u, [rho v,] E
// [, phi]) with an optional passive tracer phi (q_t + u phi_x = 0 form,
// advected at the Roe velocity).  For a face normal to d, n = normal
// momentum, t = tangential momentum, e = energy.
//   Roe averages with sqrt(rho) weights: u~ (normal), v~ (tangential), H~;
//   c~^2 = (gamma-1)(H~ - (u~^2 + v~^2)/2).
//   Waves and speeds:
//     acoustic  a1 (1, u~-c~, v~, H~ - u~ c~)          at u~ - c~
//     entropy   a2 (1, u~,    v~, (u~^2+v~^2)/2)       at u~
//     shear     a3 (0, 0,     1,  v~)          [2D]    at u~
//     acoustic  a4 (1, u~+c~, v~, H~ + u~ c~)          at u~ + c~
//     tracer    d_phi e_phi                    [opt]   at u~
//   with a3 = d_t - v~ d_rho,
//        a2 = (gamma-1)/c~^2 ((H~ - u~^2 - v~^2) d_rho + u~ d_n + v~ d_t - d_e),
//        a4 = (d_n + (c~ - u~) d_rho - c~ a2) / (2 c~),  a1 = d_rho - a2 - a4.
//   A^-dQ = sum min(s,0) W (Harten-Hyman fix on the acoustic waves when
//   entropy_fix is set), A^+dQ = sum s W - A^-dQ.
struct RoeEuler {
  double un, ut, H, c, q2;
};
struct EIdxE { int n, t, e, phi; };
EIdxE euler_idx(const OCfg& c, int d) {
  if (c.ndim == 1) return EIdxE{1, -1, 2, c.tracer ? 3 : -1};
  return EIdxE{1 + d, 2 - d, 3, c.tracer ? 4 : -1};
}
// pressure and velocities of a state in the face frame
static void euler_prim(const OCfg& c, const EIdxE& x, const double* q, double* un, double* ut,
                       double* p) {
  const double rho = q[0];
  *un = q[x.n] / rho;
  *ut = x.t >= 0 ? q[x.t] / rho : 0.0;
  *p = (c.pd[0] - 1.0) * (q[x.e] - 0.5 * rho * (*un * *un + *ut * *ut));
}
RoeEuler euler_roe_avg(const OCfg& c, const EIdxE& x, const double* ql, const double* qr) {
  double unl, utl, pl, unr, utr, pr;
  euler_prim(c, x, ql, &unl, &utl, &pl);
  euler_prim(c, x, qr, &unr, &utr, &pr);
  const double wl = std::sqrt(ql[0]), wr = std::sqrt(qr[0]);
  const double Hl = (ql[x.e] + pl) / ql[0], Hr = (qr[x.e] + pr) / qr[0];
  RoeEuler a;
  a.un = (wl * unl + wr * unr) / (wl + wr);
  a.ut = (wl * utl + wr * utr) / (wl + wr);
  a.H = (wl * Hl + wr * Hr) / (wl + wr);
  a.q2 = a.un * a.un + a.ut * a.ut;
  a.c = std::sqrt((c.pd[0] - 1.0) * (a.H - 0.5 * a.q2));
  return a;
}

void rp_euler_roe(const OCfg& c, int d, const double* ql, const double* qr, FaceSol& r) {
  const int m = num_eqn(c), mw = num_waves(c);
  const double g1 = c.pd[0] - 1.0;
  const EIdxE x = euler_idx(c, d);
  const RoeEuler a = euler_roe_avg(c, x, ql, qr);
  double dq[5];
  for (int k = 0; k < m; ++k) dq[k] = qr[k] - ql[k];
  const double dt_ = x.t >= 0 ? dq[x.t] : 0.0;
  const double a2 = g1 / (a.c * a.c) *
                    ((a.H - a.q2) * dq[0] + a.un * dq[x.n] + a.ut * dt_ - dq[x.e]);
  const double a4 = (dq[x.n] + (a.c - a.un) * dq[0] - a.c * a2) / (2.0 * a.c);
  const double a1 = dq[0] - a2 - a4;
  std::memset(r.W, 0, sizeof(r.W));
  int p = 0;
  const int p1 = p++;
  r.W[p1][0] = a1; r.W[p1][x.n] = a1 * (a.un - a.c); r.W[p1][x.e] = a1 * (a.H - a.un * a.c);
  if (x.t >= 0) r.W[p1][x.t] = a1 * a.ut;
  r.s[p1] = a.un - a.c;
  const int p2 = p++;
  r.W[p2][0] = a2; r.W[p2][x.n] = a2 * a.un; r.W[p2][x.e] = a2 * 0.5 * a.q2;
  if (x.t >= 0) r.W[p2][x.t] = a2 * a.ut;
  r.s[p2] = a.un;
  if (x.t >= 0) {
    const int p3 = p++;
    const double a3 = dq[x.t] - a.ut * dq[0];
    r.W[p3][x.t] = a3; r.W[p3][x.e] = a3 * a.ut;
    r.s[p3] = a.un;
  }
  const int p4 = p++;
  r.W[p4][0] = a4; r.W[p4][x.n] = a4 * (a.un + a.c); r.W[p4][x.e] = a4 * (a.H + a.un * a.c);
  if (x.t >= 0) r.W[p4][x.t] = a4 * a.ut;
  r.s[p4] = a.un + a.c;
  if (x.phi >= 0) {
    const int p5 = p++;
    r.W[p5][x.phi] = dq[x.phi];
    r.s[p5] = a.un;
  }
  (void)mw;
  double coef[5];
  for (int q = 0; q < p; ++q) coef[q] = std::min(r.s[q], 0.0);
  if (c.efix) {
    // Harten-Hyman: a transonic acoustic rarefaction splits its A^- part
    const double gam = c.pd[0];
    double unl, utl, pl, unr, utr, pr;
    euler_prim(c, x, ql, &unl, &utl, &pl);
    euler_prim(c, x, qr, &unr, &utr, &pr);
    {
      double qm[5];
      for (int k = 0; k < m; ++k) qm[k] = ql[k] + r.W[p1][k];
      double um, utm, pm;
      euler_prim(c, x, qm, &um, &utm, &pm);
      const double lam_l = unl - std::sqrt(gam * pl / ql[0]);
      const double lam_r = um - std::sqrt(gam * pm / qm[0]);
      if (lam_l < 0.0 && 0.0 < lam_r) coef[p1] = lam_l * (lam_r - r.s[p1]) / (lam_r - lam_l);
    }
    {
      double qm[5];
      for (int k = 0; k < m; ++k) qm[k] = qr[k] - r.W[p4][k];
      double um, utm, pm;
      euler_prim(c, x, qm, &um, &utm, &pm);
      const double lam_l = um + std::sqrt(gam * pm / qm[0]);
      const double lam_r = unr + std::sqrt(gam * pr / qr[0]);
      if (lam_l < 0.0 && 0.0 < lam_r) coef[p4] = lam_l * (lam_r - r.s[p4]) / (lam_r - lam_l);
    }
  }
  for (int k = 0; k < m; ++k) {
    double am = 0.0, sw = 0.0;
    for (int q = 0; q < p; ++q) {
      am += coef[q] * r.W[q][k];
      sw += r.s[q] * r.W[q][k];
    }
    r.amdq[k] = am;
    r.apdq[k] = sw - am;
  }
}

void rp_normal(const OCfg& c, int d, const double* ql, const double* qr, const double* auxl,
               const double* auxr, FaceSol& r) {
  switch (c.solver) {
    case S_ADV: rp_advection(c, d, ql, qr, r); break;
    case S_SW: rp_sw_roe(c, d, ql, qr, r); break;
    case S_ELASTIC: rp_elastic(d, ql, qr, auxl, auxr, r); break;
    case S_EULER_ROE: rp_euler_roe(c, d, ql, qr, r); break;
    default: std::memset(&r, 0, sizeof(r)); break;
  }
}

// Transverse Riemann solver (Section 2.1: the secondary solver of the unsplit
// multidimensional algorithms).  A fluctuation asdq produced at a face normal
// to direction d lives in one cell; split it into the parts propagating toward
// lower (bm) and higher (bp) index in the other direction.  ql, qr are the
// states of the face where asdq was produced; aux_m, aux_c, aux_p are the
// materials of that cell's lower neighbour, the cell, and its upper neighbour
// in the transverse direction.
void rp_transverse(const OCfg& c, int d, const double* ql, const double* qr, const double* aux_m,
                   const double* aux_c, const double* aux_p, const double* asdq, double* bm,
                   double* bp) {
  const int m = num_eqn(c);
  if (c.solver == S_ADV) {
    const double v = c.pd[1 - d];
    bm[0] = std::min(v, 0.0) * asdq[0];
    bp[0] = std::max(v, 0.0) * asdq[0];
    return;
  }
  if (c.solver == S_SW) {
    // eigen-decomposition in the transverse direction with the face's Roe averages
    const RoeSW a = sw_roe_avg(c, d, ql, qr);
    const int n = 1 + d, t = 2 - d;
    const double b1 = ((a.vbar + a.cbar) * asdq[0] - asdq[t]) / (2.0 * a.cbar);
    const double b3 = (-(a.vbar - a.cbar) * asdq[0] + asdq[t]) / (2.0 * a.cbar);
    const double b2 = asdq[n] - a.ubar * asdq[0];
    const double l1 = a.vbar - a.cbar, l2 = a.vbar, l3 = a.vbar + a.cbar;
    double r1[3], r2[3], r3[3];
    r1[0] = 1.0; r1[n] = a.ubar; r1[t] = a.vbar - a.cbar;
    r2[0] = 0.0; r2[n] = 1.0;    r2[t] = 0.0;
    r3[0] = 1.0; r3[n] = a.ubar; r3[t] = a.vbar + a.cbar;
    for (int k = 0; k < 3; ++k) {
      bm[k] = std::min(l1, 0.0) * b1 * r1[k] + std::min(l2, 0.0) * b2 * r2[k] +
              std::min(l3, 0.0) * b3 * r3[k];
      bp[k] = std::max(l1, 0.0) * b1 * r1[k] + std::max(l2, 0.0) * b2 * r2[k] +
              std::max(l3, 0.0) * b3 * r3[k];
    }
    (void)m;
    return;
  }
  if (c.solver == S_EULER_ROE) {
    // eigen-decomposition in the transverse direction with the face's Roe
    // averages: velocity along it v~ = a.ut, across it u~ = a.un
    const EIdxE x = euler_idx(c, d);
    const RoeEuler a = euler_roe_avg(c, x, ql, qr);
    const double g1 = c.pd[0] - 1.0;
    const double* dq = asdq;
    const double b3 = dq[x.n] - a.un * dq[0];   // shear wave (momentum across the transverse dir.)
    const double b2 = g1 / (a.c * a.c) *
                      ((a.H - a.q2) * dq[0] + a.un * dq[x.n] + a.ut * dq[x.t] - dq[x.e]);
    const double b4 = (dq[x.t] + (a.c - a.ut) * dq[0] - a.c * b2) / (2.0 * a.c);
    const double b1 = dq[0] - b2 - b4;
    double R[5][5] = {{0}}, lam[5], beta[5];
    int np = 0;
    R[np][0] = 1.0; R[np][x.n] = a.un; R[np][x.t] = a.ut - a.c; R[np][x.e] = a.H - a.ut * a.c;
    lam[np] = a.ut - a.c; beta[np++] = b1;
    R[np][0] = 1.0; R[np][x.n] = a.un; R[np][x.t] = a.ut; R[np][x.e] = 0.5 * a.q2;
    lam[np] = a.ut; beta[np++] = b2;
    R[np][x.n] = 1.0; R[np][x.e] = a.un;
    lam[np] = a.ut; beta[np++] = b3;
    R[np][0] = 1.0; R[np][x.n] = a.un; R[np][x.t] = a.ut + a.c; R[np][x.e] = a.H + a.ut * a.c;
    lam[np] = a.ut + a.c; beta[np++] = b4;
    if (x.phi >= 0) {
      R[np][x.phi] = 1.0;
      lam[np] = a.ut; beta[np++] = dq[x.phi];
    }
    for (int k = 0; k < m; ++k) {
      bm[k] = 0.0;
      bp[k] = 0.0;
      for (int q = 0; q < np; ++q) {
        bm[k] += std::min(lam[q], 0.0) * beta[q] * R[q][k];
        bp[k] += std::max(lam[q], 0.0) * beta[q] * R[q][k];
      }
    }
    return;
  }
  if (c.solver == S_ELASTIC) {
    const int t = 1 - d;   // transverse direction
    const EIdx e = eidx(t);
    const Mat M = material(aux_m), C = material(aux_c), P = material(aux_p);
    // down-going: the face between the lower neighbour (left) and the cell (right)
    const double b1 = (C.cp * asdq[e.sn] + C.a * asdq[e.vn]) / (M.a * C.cp + C.a * M.cp);
    const double b2 = (C.cs * asdq[e.sh] + C.mu * asdq[e.vt]) / (M.mu * C.cs + C.mu * M.cs);
    // up-going: the face between the cell (left) and the upper neighbour (right)
    const double b3 = (C.cs * asdq[e.sh] - C.mu * asdq[e.vt]) / (C.mu * P.cs + P.mu * C.cs);
    const double b4 = (C.cp * asdq[e.sn] - C.a * asdq[e.vn]) / (C.a * P.cp + P.a * C.cp);
    for (int k = 0; k < 5; ++k) { bm[k] = 0.0; bp[k] = 0.0; }
    // bm = -cp_m b1 r1(m) - cs_m b2 r2(m)
    bm[e.sn] += -M.cp * b1 * M.a;
    bm[e.so] += -M.cp * b1 * M.lam;
    bm[e.vn] += -M.cp * b1 * M.cp;
    bm[e.sh] += -M.cs * b2 * M.mu;
    bm[e.vt] += -M.cs * b2 * M.cs;
    // bp = cs_p b3 r3(p) + cp_p b4 r4(p)
    bp[e.sh] += P.cs * b3 * P.mu;
    bp[e.vt] += P.cs * b3 * (-P.cs);
    bp[e.sn] += P.cp * b4 * P.a;
    bp[e.so] += P.cp * b4 * P.lam;
    bp[e.vn] += P.cp * b4 * (-P.cp);
    return;
  }
  for (int k = 0; k < m; ++k) { bm[k] = 0.0; bp[k] = 0.0; }
}

// Wave limiter (Section 2: the limiter acts on waves, not fluxes; LeVeque 2002,
// ch. 6 and 9).  theta = (W_upwind . W) / (W . W); the upwind face is the
// lower-index neighbour when s > 0, else the higher-index one.
double limiter_phi(int lim, double th) {
  switch (lim) {
    case 0: return 1.0;
    case 1: return std::max(0.0, std::min(1.0, th));                                // minmod
    case 2: return std::max(0.0, std::min(std::min((1.0 + th) / 2.0, 2.0), 2.0 * th));  // MC
  }
  return 1.0;
}

void limit_waves(const OCfg& c, int m, int mw, const FaceSol& lo, const FaceSol& me,
                 const FaceSol& hi, double Wl[5][5]) {
  for (int p = 0; p < mw; ++p) {
    double nrm = 0.0, dlo = 0.0, dhi = 0.0;
    for (int k = 0; k < m; ++k) {
      nrm += me.W[p][k] * me.W[p][k];
      dlo += lo.W[p][k] * me.W[p][k];
      dhi += hi.W[p][k] * me.W[p][k];
    }
    double phi = 0.0;
    if (nrm != 0.0) {
      const double th = (me.s[p] > 0.0 ? dlo : dhi) / nrm;
      phi = limiter_phi(c.limiter, th);
    }
    for (int k = 0; k < m; ++k) Wl[p][k] = phi * me.W[p][k];
  }
}

// ---------------------------------------------------------------------------
// Classic Clawpack step (Section 2, eq. lwflux and eq. fluxdiff; Section 2.1,
// transverse corrections; LeVeque 1997).
// ---------------------------------------------------------------------------

double classic_1d(const OCfg& c, const double* qin, double* qout, double dt) {
  const int m = num_eqn(c), mw = num_waves(c), nx = c.nx;
  const double dx = dx_of(c), dtdx = dt / dx;
  Field Q;
  load_field(c, Q, qin, m, 2, false);
  // faces f = -1 .. nx+1 ; face f lies between cells f-1 and f
  std::vector<FaceSol> F(nx + 3);
  for (int f = -1; f <= nx + 1; ++f) {
    double ql[5], qr[5];
    for (int k = 0; k < m; ++k) { ql[k] = Q.at(k, 0, f - 1); qr[k] = Q.at(k, 0, f); }
    rp_normal(c, 0, ql, qr, nullptr, nullptr, F[f + 1]);
  }
  double smax = 0.0;
  std::vector<double> Ft((size_t)(nx + 1) * m, 0.0);
  for (int f = 0; f <= nx; ++f) {
    const FaceSol& me = F[f + 1];
    double Wl[5][5];
    limit_waves(c, m, mw, F[f], me, F[f + 2], Wl);
    for (int p = 0; p < mw; ++p) {
      const double as = std::fabs(me.s[p]);
      smax = std::max(smax, as / dx);
      for (int k = 0; k < m; ++k) Ft[(size_t)f * m + k] += 0.5 * as * (1.0 - dtdx * as) * Wl[p][k];
    }
  }
  for (int k = 0; k < m; ++k)
    for (int i = 0; i < nx; ++i) {
      const FaceSol& lo = F[i + 1];   // face i   (left of cell i)
      const FaceSol& hi = F[i + 2];   // face i+1 (right of cell i)
      qout[(size_t)k * nx + i] =
          Q.at(k, 0, i) - dtdx * (lo.apdq[k] + hi.amdq[k]) -
          dtdx * (Ft[(size_t)(i + 1) * m + k] - Ft[(size_t)i * m + k]);
    }
  return smax;
}

double classic_2d(const OCfg& c, const double* qin, const double* auxin, double* qout, double dt) {
  const int m = num_eqn(c), mw = num_waves(c), na = num_aux(c);
  const int nx = c.nx, ny = c.ny;
  const double dx = dx_of(c), dy = dy_of(c);
  const double dtdx = dt / dx, dtdy = dt / dy;
  Field Q, A;
  load_field(c, Q, qin, m, 2, false);
  load_field(c, A, auxin, na, 2, true);
  static const double zero_aux[3] = {0.0, 0.0, 0.0};
  auto auxp = [&](int j, int i, double* buf) -> const double* {
    if (na == 0) return zero_aux;
    for (int k = 0; k < na; ++k) buf[k] = A.at(k, j, i);
    return buf;
  };

  // x-faces: face (f, j) between cells (f-1, j) and (f, j); f in [-1, nx+1], j in [-1, ny]
  const int XW = nx + 3, XH = ny + 2;
  std::vector<FaceSol> XF((size_t)XW * XH);
  auto xf = [&](int f, int j) -> FaceSol& { return XF[(size_t)(j + 1) * XW + (f + 1)]; };
  // y-faces: face (i, g) between cells (i, g-1) and (i, g); g in [-1, ny+1], i in [-1, nx]
  const int YW = nx + 2, YH = ny + 3;
  std::vector<FaceSol> YF((size_t)YW * YH);
  auto yf = [&](int i, int g) -> FaceSol& { return YF[(size_t)(g + 1) * YW + (i + 1)]; };

#pragma omp parallel for schedule(static)
  for (int j = -1; j <= ny; ++j)
    for (int f = -1; f <= nx + 1; ++f) {
      double ql[5], qr[5], al[3], ar[3];
      for (int k = 0; k < m; ++k) { ql[k] = Q.at(k, j, f - 1); qr[k] = Q.at(k, j, f); }
      rp_normal(c, 0, ql, qr, auxp(j, f - 1, al), auxp(j, f, ar), xf(f, j));
    }
#pragma omp parallel for schedule(static)
  for (int g = -1; g <= ny + 1; ++g)
    for (int i = -1; i <= nx; ++i) {
      double ql[5], qr[5], al[3], ar[3];
      for (int k = 0; k < m; ++k) { ql[k] = Q.at(k, g - 1, i); qr[k] = Q.at(k, g, i); }
      rp_normal(c, 1, ql, qr, auxp(g - 1, i, al), auxp(g, i, ar), yf(i, g));
    }

  // Correction fluxes: Fx at x-faces (f in [0,nx], j in [0,ny)), Gy at y-faces
  // (i in [0,nx), g in [0,ny]).  Each holds the limited second-order term plus
  // the transverse contributions from faces of the other direction.
  std::vector<double> Fc((size_t)(nx + 1) * ny * m, 0.0), Gc((size_t)nx * (ny + 1) * m, 0.0);
  auto fc = [&](int f, int j, int k) -> double& { return Fc[((size_t)j * (nx + 1) + f) * m + k]; };
  auto gc = [&](int i, int g, int k) -> double& { return Gc[((size_t)g * nx + i) * m + k]; };

  double smax = 0.0;
  // x sweep: limiter, correction flux, transverse split into G (serial: scatter)
  for (int j = -1; j <= ny; ++j)
    for (int f = 0; f <= nx; ++f) {
      const FaceSol& me = xf(f, j);
      double Wl[5][5], cq[5] = {0, 0, 0, 0, 0};
      limit_waves(c, m, mw, xf(f - 1, j), me, xf(f + 1, j), Wl);
      for (int p = 0; p < mw; ++p) {
        const double as = std::fabs(me.s[p]);
        if (j >= 0 && j < ny) smax = std::max(smax, as / dx);
        for (int k = 0; k < m; ++k) cq[k] += as * (1.0 - dtdx * as) * Wl[p][k];
      }
      if (j >= 0 && j < ny)
        for (int k = 0; k < m; ++k) fc(f, j, k) += 0.5 * cq[k];
      if (c.transverse == 0) continue;
      double am[5], ap[5];
      for (int k = 0; k < m; ++k) {
        am[k] = me.amdq[k] + (c.transverse == 2 ? cq[k] : 0.0);
        ap[k] = me.apdq[k] - (c.transverse == 2 ? cq[k] : 0.0);
      }
      double ql[5], qr[5];
      for (int k = 0; k < m; ++k) { ql[k] = Q.at(k, j, f - 1); qr[k] = Q.at(k, j, f); }
      double bm[5], bp[5], a0[3], a1[3], a2[3];
      // A^+ part lives in cell (f, j): feeds G at y-faces (f, j) and (f, j+1)
      rp_transverse(c, 0, ql, qr, auxp(j - 1, f, a0), auxp(j, f, a1), auxp(j + 1, f, a2), ap, bm, bp);
      if (f < nx) {
        if (j + 1 >= 0 && j + 1 <= ny)
          for (int k = 0; k < m; ++k) gc(f, j + 1, k) -= 0.5 * dtdx * bp[k];
        if (j >= 0 && j <= ny)
          for (int k = 0; k < m; ++k) gc(f, j, k) -= 0.5 * dtdx * bm[k];
      }
      // A^- part lives in cell (f-1, j)
      rp_transverse(c, 0, ql, qr, auxp(j - 1, f - 1, a0), auxp(j, f - 1, a1), auxp(j + 1, f - 1, a2),
                    am, bm, bp);
      if (f - 1 >= 0) {
        if (j + 1 >= 0 && j + 1 <= ny)
          for (int k = 0; k < m; ++k) gc(f - 1, j + 1, k) -= 0.5 * dtdx * bp[k];
        if (j >= 0 && j <= ny)
          for (int k = 0; k < m; ++k) gc(f - 1, j, k) -= 0.5 * dtdx * bm[k];
      }
    }
  // y sweep
  for (int g = 0; g <= ny; ++g)
    for (int i = -1; i <= nx; ++i) {
      const FaceSol& me = yf(i, g);
      double Wl[5][5], cq[5] = {0, 0, 0, 0, 0};
      limit_waves(c, m, mw, yf(i, g - 1), me, yf(i, g + 1), Wl);
      for (int p = 0; p < mw; ++p) {
        const double as = std::fabs(me.s[p]);
        if (i >= 0 && i < nx) smax = std::max(smax, as / dy);
        for (int k = 0; k < m; ++k) cq[k] += as * (1.0 - dtdy * as) * Wl[p][k];
      }
      if (i >= 0 && i < nx)
        for (int k = 0; k < m; ++k) gc(i, g, k) += 0.5 * cq[k];
      if (c.transverse == 0) continue;
      double bmq[5], bpq[5];
      for (int k = 0; k < m; ++k) {
        bmq[k] = me.amdq[k] + (c.transverse == 2 ? cq[k] : 0.0);
        bpq[k] = me.apdq[k] - (c.transverse == 2 ? cq[k] : 0.0);
      }
      double ql[5], qr[5];
      for (int k = 0; k < m; ++k) { ql[k] = Q.at(k, g - 1, i); qr[k] = Q.at(k, g, i); }
      double lm[5], lp[5], a0[3], a1[3], a2[3];
      // B^+ part lives in cell (i, g): feeds F at x-faces (i, g) and (i+1, g)
      rp_transverse(c, 1, ql, qr, auxp(g, i - 1, a0), auxp(g, i, a1), auxp(g, i + 1, a2), bpq, lm, lp);
      if (g < ny) {
        if (i + 1 >= 0 && i + 1 <= nx)
          for (int k = 0; k < m; ++k) fc(i + 1, g, k) -= 0.5 * dtdy * lp[k];
        if (i >= 0 && i <= nx)
          for (int k = 0; k < m; ++k) fc(i, g, k) -= 0.5 * dtdy * lm[k];
      }
      // B^- part lives in cell (i, g-1)
      rp_transverse(c, 1, ql, qr, auxp(g - 1, i - 1, a0), auxp(g - 1, i, a1), auxp(g - 1, i + 1, a2),
                    bmq, lm, lp);
      if (g - 1 >= 0) {
        if (i + 1 >= 0 && i + 1 <= nx)
          for (int k = 0; k < m; ++k) fc(i + 1, g - 1, k) -= 0.5 * dtdy * lp[k];
        if (i >= 0 && i <= nx)
          for (int k = 0; k < m; ++k) fc(i, g - 1, k) -= 0.5 * dtdy * lm[k];
      }
    }

  // cell update, eq. fluxdiff with fluctuations and correction fluxes
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < m; ++k) {
        const double xs = xf(i, j).apdq[k] + xf(i + 1, j).amdq[k] + fc(i + 1, j, k) - fc(i, j, k);
        const double ys = yf(i, j).apdq[k] + yf(i, j + 1).amdq[k] + gc(i, j + 1, k) - gc(i, j, k);
        qout[((size_t)k * ny + j) * nx + i] = Q.at(k, j, i) - dtdx * xs - dtdy * ys;
      }
  return smax;
}

// ---------------------------------------------------------------------------
// Dimensionally split classic step (the paper names both dimensionally-split
// and fully multidimensional algorithms, Section 2.1): each sweep applies the
// 1D wave-propagation update (normal solves, limited correction fluxes, no
// transverse terms) along x to every row, or along y to every column, of the
// 2D state.  Godunov splitting: x sweep over dt, then y sweep over dt.
// Strang splitting: x over dt/2, y over dt, x over dt/2.
// Courant number (the paper is silent on split steps): the step's dt times
// the running maximum of the sweeps' largest speed / spacing, taken in sweep
// order and stopped at the first sweep whose own value (step dt times its
// speed) exceeds cfl_max or is not finite: that sweep rejects the step (or
// flags it non-physical), and the sweeps after it, which act on an unstable
// intermediate, do not count.  A sweep's speed is NaN if any of its faces'
// is.
// ---------------------------------------------------------------------------
double classic_sweep(const OCfg& c, int d, const double* qin, const double* auxin, double* qout,
                     double dt) {
  const int m = num_eqn(c), mw = num_waves(c), na = num_aux(c);
  const int nx = c.nx, ny = c.ny;
  const double h = d == 0 ? dx_of(c) : dy_of(c), dth = dt / h;
  Field Q, A;
  load_field(c, Q, qin, m, 2, false);
  load_field(c, A, auxin, na, 2, true);
  const int n = d == 0 ? nx : ny, lines = d == 0 ? ny : nx;
  double smax = 0.0;
  int nan_seen = 0;
#pragma omp parallel for schedule(static) reduction(max : smax) reduction(| : nan_seen)
  for (int L = 0; L < lines; ++L) {
    auto at = [&](int k, int s) { return d == 0 ? Q.at(k, L, s) : Q.at(k, s, L); };
    auto aux_at = [&](int k, int s) { return d == 0 ? A.at(k, L, s) : A.at(k, s, L); };
    // faces f = -1 .. n+1 along the line; face f lies between cells f-1 and f
    std::vector<FaceSol> F(n + 3);
    for (int f = -1; f <= n + 1; ++f) {
      double ql[5], qr[5], al[3] = {0, 0, 0}, ar[3] = {0, 0, 0};
      for (int k = 0; k < m; ++k) { ql[k] = at(k, f - 1); qr[k] = at(k, f); }
      for (int k = 0; k < na; ++k) { al[k] = aux_at(k, f - 1); ar[k] = aux_at(k, f); }
      rp_normal(c, d, ql, qr, al, ar, F[f + 1]);
    }
    std::vector<double> Ft((size_t)(n + 1) * m, 0.0);
    for (int f = 0; f <= n; ++f) {
      const FaceSol& me = F[f + 1];
      double Wl[5][5];
      limit_waves(c, m, mw, F[f], me, F[f + 2], Wl);
      for (int p = 0; p < mw; ++p) {
        const double as = std::fabs(me.s[p]);
        if (std::isnan(as)) nan_seen = 1;
        else smax = std::max(smax, as / h);
        for (int k = 0; k < m; ++k) Ft[(size_t)f * m + k] += 0.5 * as * (1.0 - dth * as) * Wl[p][k];
      }
    }
    for (int s = 0; s < n; ++s)
      for (int k = 0; k < m; ++k) {
        const size_t idx = d == 0 ? ((size_t)k * ny + L) * nx + s : ((size_t)k * ny + s) * nx + L;
        qout[idx] = at(k, s) - dth * (F[s + 1].apdq[k] + F[s + 2].amdq[k]) -
                    dth * (Ft[(size_t)(s + 1) * m + k] - Ft[(size_t)s * m + k]);
      }
  }
  return nan_seen ? std::numeric_limits<double>::quiet_NaN() : smax;
}

double classic_2d_split(const OCfg& c, const double* qin, const double* auxin, double* qout,
                        double dt) {
  const size_t N = (size_t)num_eqn(c) * c.nx * c.ny;
  std::vector<double> a(N), b(N);
  double s = 0.0;
  bool open = true;   // no sweep has ended the Courant reading yet
  auto fold = [&](double sk) {
    if (!open) return;
    s = std::isnan(sk) ? sk : std::max(s, sk);
    if (!(dt * sk <= c.cfl_max)) open = false;
  };
  if (c.split == 2) {
    fold(classic_sweep(c, 0, qin, auxin, a.data(), 0.5 * dt));
    fold(classic_sweep(c, 1, a.data(), auxin, b.data(), dt));
    fold(classic_sweep(c, 0, b.data(), auxin, qout, 0.5 * dt));
  } else {
    fold(classic_sweep(c, 0, qin, auxin, a.data(), dt));
    fold(classic_sweep(c, 1, a.data(), auxin, qout, dt));
  }
  return s;
}

// ---------------------------------------------------------------------------
// SharpClaw (Section 2, method of lines; Section 2.1: WENO5 in space, SSP
// Runge-Kutta in time, normal Riemann problems only in multi-D).
// ---------------------------------------------------------------------------

// WENO5 (Jiang-Shu) from five cell averages v[0..4] centred on cell i = v[2]:
// qL = value at the right edge of cell i (x_{i+1/2}, seen from the left),
// qR = value at the left edge of cell i (x_{i-1/2}, seen from the right).
void weno5(const double* v, double eps, double* qL, double* qR) {
  const double vm2 = v[0], vm1 = v[1], v0 = v[2], vp1 = v[3], vp2 = v[4];
  const double b0 = 13.0 / 12.0 * (vm2 - 2.0 * vm1 + v0) * (vm2 - 2.0 * vm1 + v0) +
                    0.25 * (vm2 - 4.0 * vm1 + 3.0 * v0) * (vm2 - 4.0 * vm1 + 3.0 * v0);
  const double b1 = 13.0 / 12.0 * (vm1 - 2.0 * v0 + vp1) * (vm1 - 2.0 * v0 + vp1) +
                    0.25 * (vm1 - vp1) * (vm1 - vp1);
  const double b2 = 13.0 / 12.0 * (v0 - 2.0 * vp1 + vp2) * (v0 - 2.0 * vp1 + vp2) +
                    0.25 * (3.0 * v0 - 4.0 * vp1 + vp2) * (3.0 * v0 - 4.0 * vp1 + vp2);
  // right edge of cell i
  {
    const double p0 = (2.0 * vm2 - 7.0 * vm1 + 11.0 * v0) / 6.0;
    const double p1 = (-vm1 + 5.0 * v0 + 2.0 * vp1) / 6.0;
    const double p2 = (2.0 * v0 + 5.0 * vp1 - vp2) / 6.0;
    const double a0 = 0.1 / ((eps + b0) * (eps + b0));
    const double a1 = 0.6 / ((eps + b1) * (eps + b1));
    const double a2 = 0.3 / ((eps + b2) * (eps + b2));
    *qL = (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
  }
  // left edge of cell i: mirror image (stencils reversed, linear weights reversed)
  {
    const double p0 = (-vm2 + 5.0 * vm1 + 2.0 * v0) / 6.0;
    const double p1 = (2.0 * vm1 + 5.0 * v0 - vp1) / 6.0;
    const double p2 = (11.0 * v0 - 7.0 * vp1 + 2.0 * vp2) / 6.0;
    const double a0 = 0.3 / ((eps + b0) * (eps + b0));
    const double a1 = 0.6 / ((eps + b1) * (eps + b1));
    const double a2 = 0.1 / ((eps + b2) * (eps + b2));
    *qR = (a0 * p0 + a1 * p1 + a2 * p2) / (a0 + a1 + a2);
  }
}

// ---------------------------------------------------------------------------
// WENO of order 2r-1 (Jiang-Shu construction for any r; PyWENO generates the
// same tables symbolically), written from its definition with cell width 1
// and cell i = [-1/2, 1/2]:
//   * candidate k = 0..r-1 is the polynomial of degree r-1 whose averages over
//     cells i-r+1+k .. i+k equal the data; its values at x = +1/2 and -1/2
//     are linear in the data (coefficient tables cR, cL);
//   * the linear weights d_k make sum_k d_k p_k(+1/2) equal the value of the
//     degree-(2r-2) polynomial through all 2r-1 averages (consistency);
//     the left edge uses the mirrored weights d_{r-1-k};
//   * beta_k = sum_{l=1}^{r-1} integral over the cell of (d^l p_k / dx^l)^2,
//     evaluated from p_k's monomial coefficients a_1 .. a_{r-1} (the
//     constant a_0 does not enter): beta_k = sum_{n,m>=1} H_nm a_n a_m with
//     H_nm = sum_l (n!/(n-l)!) (m!/(m-l)!) integral of x^(n+m-2l);
//   * omega_k = alpha_k / sum alpha, alpha_k = d_k / (eps + beta_k)^2.
// The tables are computed once per r, in extended precision, by solving the
// small interpolation systems and integrating the squared derivatives exactly.
// ---------------------------------------------------------------------------
struct WenoTables {
  int r = 0;
  long double cR[9][9], cL[9][9];   // [k][j]: value at +1/2 / -1/2 from data of stencil k, j = 0..r-1
  double d[9];                      // linear weights, right edge
  long double A[9][9][9];           // [k][n][j]: monomial coefficient a_n of candidate k from its data
  long double H[9][9];              // [n][m]: beta = sum_{n,m >= 1} H a_n a_m
};

// The tables are built in binary128 (__float128, 113-bit significand): the
// monomial interpolation systems are ill-conditioned at high order (in
// long double the order-17 linear weights came out 3e-11 off their exact
// rational values); they are then stored in long double.
using Wide = __float128;
static Wide wabs(Wide x) { return x < 0 ? -x : x; }

// Coefficients a_n of p(x) = sum a_n x^n (n < r) from r cell averages at
// cells c0 .. c0+r-1 (cell j = [j-1/2, j+1/2]): returns the matrix M with
// a = M v.
static void interp_matrix(int r, int c0, Wide M[9][9]) {
  Wide A[9][18];
  for (int row = 0; row < r; ++row) {
    const Wide lo = c0 + row - Wide(0.5), hi = c0 + row + Wide(0.5);
    Wide plo = lo, phi = hi;   // lo^(n+1), hi^(n+1)
    for (int n = 0; n < r; ++n) {
      A[row][n] = (phi - plo) / (n + 1);
      plo *= lo;
      phi *= hi;
    }
    for (int n = 0; n < r; ++n) A[row][r + n] = row == n ? Wide(1) : Wide(0);
  }
  // Gauss-Jordan with partial pivoting: A = [V | I] -> [I | V^-1]
  for (int col = 0; col < r; ++col) {
    int piv = col;
    for (int row = col + 1; row < r; ++row)
      if (wabs(A[row][col]) > wabs(A[piv][col])) piv = row;
    for (int n = 0; n < 2 * r; ++n) std::swap(A[col][n], A[piv][n]);
    const Wide inv = Wide(1) / A[col][col];
    for (int n = 0; n < 2 * r; ++n) A[col][n] *= inv;
    for (int row = 0; row < r; ++row) {
      if (row == col) continue;
      const Wide f = A[row][col];
      for (int n = 0; n < 2 * r; ++n) A[row][n] -= f * A[col][n];
    }
  }
  for (int n = 0; n < r; ++n)
    for (int j = 0; j < r; ++j) M[n][j] = A[n][r + j];
}

static Wide poly_at(int r, const Wide* a, Wide x) {
  Wide s = Wide(0);
  for (int n = r - 1; n >= 0; --n) s = s * x + a[n];
  return s;
}

static const WenoTables& weno_tables(int r) {
  static WenoTables T[10];
  static bool done[10] = {false};
  WenoTables& t = T[r];
  if (done[r]) return t;
#pragma omp critical(weno_tables)
  if (!done[r]) {
    t.r = r;
    Wide cR[9][9], cL[9][9];
    for (int k = 0; k < r; ++k) {
      Wide M[9][9];
      interp_matrix(r, -(r - 1) + k, M);
      for (int j = 0; j < r; ++j) {
        Wide a[9];
        for (int n = 0; n < r; ++n) a[n] = M[n][j];
        cR[k][j] = poly_at(r, a, Wide(0.5));
        cL[k][j] = poly_at(r, a, -Wide(0.5));
        t.cR[k][j] = (long double)cR[k][j];
        t.cL[k][j] = (long double)cL[k][j];
      }
      for (int n = 0; n < r; ++n)
        for (int j = 0; j < r; ++j) t.A[k][n][j] = (long double)M[n][j];
    }
    // Gram matrix of the derivatives of the monomials: integral over the cell
    // of sum_l d^l x^n d^l x^m
    for (int n = 1; n < r; ++n)
      for (int m = 1; m < r; ++m) {
        Wide sum = Wide(0);
        for (int l = 1; l <= std::min(n, m); ++l) {
          Wide fn = Wide(1), fm = Wide(1);   // n!/(n-l)!, m!/(m-l)!
          for (int q = 0; q < l; ++q) { fn *= (n - q); fm *= (m - q); }
          const int e = (n - l) + (m - l);
          Wide h = Wide(1);   // (1/2)^(e+1); the integral of x^e over [-1/2, 1/2]
          for (int q = 0; q <= e; ++q) h *= Wide(0.5);
          sum += fn * fm * (e % 2 == 0 ? 2 * h : Wide(0)) / (e + 1);
        }
        t.H[n][m] = (long double)sum;
      }
    // big stencil: degree 2r-2 through the averages of cells -(r-1) .. r-1
    const int R2 = 2 * r - 1;
    Wide big[17];
    {
      Wide A[17][34];
      for (int row = 0; row < R2; ++row) {
        const Wide lo = -(r - 1) + row - Wide(0.5), hi = -(r - 1) + row + Wide(0.5);
        Wide plo = lo, phi = hi;
        for (int n = 0; n < R2; ++n) {
          A[row][n] = (phi - plo) / (n + 1);
          plo *= lo;
          phi *= hi;
        }
        for (int n = 0; n < R2; ++n) A[row][R2 + n] = row == n ? Wide(1) : Wide(0);
      }
      for (int col = 0; col < R2; ++col) {
        int piv = col;
        for (int row = col + 1; row < R2; ++row)
          if (wabs(A[row][col]) > wabs(A[piv][col])) piv = row;
        for (int n = 0; n < 2 * R2; ++n) std::swap(A[col][n], A[piv][n]);
        const Wide inv = Wide(1) / A[col][col];
        for (int n = 0; n < 2 * R2; ++n) A[col][n] *= inv;
        for (int row = 0; row < R2; ++row) {
          if (row == col) continue;
          const Wide f = A[row][col];
          for (int n = 0; n < 2 * R2; ++n) A[row][n] -= f * A[col][n];
        }
      }
      // value at +1/2 as a functional of the data: sum_n (1/2)^n M[n][j]
      for (int j = 0; j < R2; ++j) {
        Wide s = Wide(0), x = Wide(1);
        for (int n = 0; n < R2; ++n) { s += x * A[n][R2 + j]; x *= Wide(0.5); }
        big[j] = s;
      }
    }
    // consistency: sum_k d_k cR[k][j - k] = big[j]; data cell j of the big
    // stencil is cell j - k of candidate k.  Triangular in k for j < r.
    Wide dd[9];
    for (int j = 0; j < r; ++j) {
      Wide s = big[j];
      for (int k = 0; k < j; ++k) s -= dd[k] * cR[k][j - k];
      dd[j] = s / cR[j][0];
    }
    for (int k = 0; k < r; ++k) t.d[k] = (double)dd[k];
    done[r] = true;
  }
  return t;
}

// Candidate k's edge values and smoothness indicator from its r averages s[].
// Evaluated in long double: the monomial coefficients of a high-degree
// candidate are sums of large terms of both signs, and the quadratic form of
// the indicator loses further digits to cancellation (in double, about 4e-12
// of an edge value at order 17 against an exact evaluation).
static void weno_candidate(const WenoTables& t, int k, const double* s, double* pR, double* pL,
                           double* beta) {
  const int r = t.r;
  long double a = 0.0L, c = 0.0L, an[9];
  for (int i = 0; i < r; ++i) {
    a += t.cR[k][i] * s[i];
    c += t.cL[k][i] * s[i];
  }
  for (int n = 1; n < r; ++n) {
    an[n] = 0.0L;
    for (int i = 0; i < r; ++i) an[n] += t.A[k][n][i] * s[i];
  }
  long double b = 0.0L;
  for (int n = 1; n < r; ++n)
    for (int m = 1; m < r; ++m) b += t.H[n][m] * an[n] * an[m];
  *pR = (double)a;
  *pL = (double)c;
  *beta = (double)b;
}

// Edge values of cell i from the 2r-1 averages v[0..2r-2] centred on it
// (v[r-1] = cell i): qL at its right edge, qR at its left edge.
void weno_r(int r, const double* v, double eps, double* qL, double* qR) {
  const WenoTables& t = weno_tables(r);
  double beta[9], pR[9], pL[9];
  for (int k = 0; k < r; ++k) weno_candidate(t, k, v + k, &pR[k], &pL[k], &beta[k]);
  double sR = 0.0, sL = 0.0, nR = 0.0, nL = 0.0;
  for (int k = 0; k < r; ++k) {
    const double w = 1.0 / ((eps + beta[k]) * (eps + beta[k]));
    const double aR = t.d[k] * w, aL = t.d[r - 1 - k] * w;
    sR += aR; nR += aR * pR[k];
    sL += aL; nL += aL * pL[k];
  }
  *qL = nR / sR;
  *qR = nL / sL;
}

// Half-width of the reconstruction stencil (= ghost layers) of a config.
int weno_r_of(const OCfg& c) { return c.weno_order >= 7 ? (c.weno_order + 1) / 2 : 3; }

// Edge values of one cell from 2r-1 averages: WENO5 through its closed form,
// other orders through the general construction.
void weno_edges(const OCfg& c, const double* v, double* qL, double* qR) {
  const int r = weno_r_of(c);
  if (r == 3) weno5(v, c.weno_eps, qL, qR);
  else weno_r(r, v, c.weno_eps, qL, qR);
}

// Physical flux in direction d.
void euler_flux(const OCfg& c, int d, const double* q, double* f, double* un_out, double* cs_out) {
  const double gam = c.pd[0];
  const int m = num_eqn(c);
  const double rho = q[0];
  const double u = q[1] / rho;
  const double v = m == 4 ? q[2] / rho : 0.0;
  const double E = q[m - 1];
  const double p = (gam - 1.0) * (E - 0.5 * rho * (u * u + v * v));
  const double un = d == 0 ? u : v;
  f[0] = rho * un;
  f[1] = q[1] * un + (d == 0 ? p : 0.0);
  if (m == 4) f[2] = q[2] * un + (d == 1 ? p : 0.0);
  f[m - 1] = (E + p) * un;
  *un_out = un;
  *cs_out = std::sqrt(gam * p / rho);
}

// HLLE numerical flux (Einfeldt 1988) with Roe-average speed estimates.
double flux_hlle(const OCfg& c, int d, const double* ql, const double* qr, double* F) {
  const double gam = c.pd[0];
  const int m = num_eqn(c);
  double fl[4], fr[4], unl, unr, cl, cr;
  euler_flux(c, d, ql, fl, &unl, &cl);
  euler_flux(c, d, qr, fr, &unr, &cr);
  const double rl = ql[0], rr = qr[0];
  const double wl = std::sqrt(rl), wr = std::sqrt(rr);
  const double ul = ql[1] / rl, ur = qr[1] / rr;
  const double vl = m == 4 ? ql[2] / rl : 0.0, vr = m == 4 ? qr[2] / rr : 0.0;
  const double pl = (gam - 1.0) * (ql[m - 1] - 0.5 * rl * (ul * ul + vl * vl));
  const double pr = (gam - 1.0) * (qr[m - 1] - 0.5 * rr * (ur * ur + vr * vr));
  const double Hl = (ql[m - 1] + pl) / rl, Hr = (qr[m - 1] + pr) / rr;
  const double ut = (wl * ul + wr * ur) / (wl + wr);
  const double vt = (wl * vl + wr * vr) / (wl + wr);
  const double Ht = (wl * Hl + wr * Hr) / (wl + wr);
  const double ct = std::sqrt((gam - 1.0) * (Ht - 0.5 * (ut * ut + vt * vt)));
  const double unt = d == 0 ? ut : vt;
  const double s1 = std::min(unl - cl, unt - ct);
  const double s2 = std::max(unr + cr, unt + ct);
  for (int k = 0; k < m; ++k) {
    if (s1 >= 0.0)
      F[k] = fl[k];
    else if (s2 <= 0.0)
      F[k] = fr[k];
    else
      F[k] = (s2 * fl[k] - s1 * fr[k] + s1 * s2 * (qr[k] - ql[k])) / (s2 - s1);
  }
  return std::max(std::fabs(s1), std::fabs(s2));
}

// Upwind flux for scalar advection.
double flux_advection(const OCfg& c, int d, const double* ql, const double* qr, double* F) {
  const double u = c.pd[d];
  F[0] = u > 0.0 ? u * ql[0] : u * qr[0];
  return std::fabs(u);
}

// Nonlinear p-system with spatially varying coefficients (Section 7.3,
// eq. p-system): q = (strain eps, x-momentum rho u, y-momentum rho v), aux =
// (bulk modulus K, density rho) per cell, stress sigma(eps) = exp(K eps) - 1
// (eq. nonlinear const relation up to its additive constant, which cancels
// in every flux difference).  Flux normal to direction d: f = -(u_n, sigma
// e_n) with u_n = (rho u_n) / rho.  Its Jacobian has speeds -c, 0, +c with
// c = sqrt(sigma'(eps) / rho) = sqrt(K exp(K eps) / rho) and, for -c / +c,
// eigenvectors (1, Z e_n) / (1, -Z e_n), Z = rho c (impedance).
//
// Interface flux (f-wave decomposition for a flux that varies in space: the
// jump of the physical flux across the face, each side in its own material,
// is split into a left-going f-wave on the left material's eigenvector and a
// right-going one on the right material's):
//   f_r - f_l = b1 (1, Z_l e_n) + b2 (1, -Z_r e_n),
//   F = f_l + b1 (1, Z_l e_n)          (= f_r - b2 (1, -Z_r e_n)).
// Speed for the Courant number: max(c_l, c_r).
double flux_psystem(const OCfg& c, int d, const double* ql, const double* qr, const double* al,
                    const double* ar, double* F) {
  const int m = num_eqn(c), n = 1 + d;
  const double Kl = al[0], rl = al[1], Kr = ar[0], rr = ar[1];
  const double sl = std::expm1(Kl * ql[0]), sr = std::expm1(Kr * qr[0]);
  const double cl = std::sqrt(Kl * std::exp(Kl * ql[0]) / rl);
  const double cr = std::sqrt(Kr * std::exp(Kr * qr[0]) / rr);
  const double Zl = rl * cl, Zr = rr * cr;
  double fl[3] = {0.0, 0.0, 0.0}, fr[3] = {0.0, 0.0, 0.0};
  fl[0] = -ql[n] / rl;
  fl[n] = -sl;
  fr[0] = -qr[n] / rr;
  fr[n] = -sr;
  const double d0 = fr[0] - fl[0], dn = fr[n] - fl[n];
  const double b1 = (Zr * d0 + dn) / (Zl + Zr);
  for (int k = 0; k < m; ++k) F[k] = fl[k];
  F[0] += b1;
  F[n] += b1 * Zl;
  return std::max(cl, cr);
}

double num_flux(const OCfg& c, int d, const double* ql, const double* qr, const double* al,
                const double* ar, double* F) {
  if (c.solver == S_EULER) return flux_hlle(c, d, ql, qr, F);
  if (c.solver == S_PSYS) return flux_psystem(c, d, ql, qr, al, ar, F);
  return flux_advection(c, d, ql, qr, F);
}

// Semi-discrete operator L(Q) = -(F_{i+1/2}-F_{i-1/2})/dx - (G_{j+1/2}-G_{j-1/2})/dy.
// Returns the largest |speed|/spacing over faces bounding interior cells.
// A face flux sees the aux fields (material) of the two cells it separates.
double sharpclaw_L(const OCfg& c, const double* qin, const double* auxin, double* L) {
  const int m = num_eqn(c), nx = c.nx, ny = c.ny, na = num_aux(c);
  const double dx = dx_of(c), dy = dy_of(c);
  const int r = weno_r_of(c), w = 2 * r - 1;
  Field Q, A;
  load_field(c, Q, qin, m, r, false);
  load_field(c, A, auxin, na, r, true);
  auto aux_of = [&](int j, int i, double* a) {
    for (int k = 0; k < na; ++k) a[k] = A.at(k, j, i);
  };
  std::fill(L, L + (size_t)m * nx * ny, 0.0);
  double smax = 0.0;
  // x direction: one row at a time
#pragma omp parallel for schedule(static) reduction(max : smax)
  for (int j = 0; j < ny; ++j) {
    // edge values of cells -1 .. nx
    std::vector<double> eL((size_t)(nx + 2) * m), eR((size_t)(nx + 2) * m);
    for (int i = -1; i <= nx; ++i)
      for (int k = 0; k < m; ++k) {
        double v[17];
        for (int s = 0; s < w; ++s) v[s] = Q.at(k, j, i - (r - 1) + s);
        weno_edges(c, v, &eL[(size_t)(i + 1) * m + k], &eR[(size_t)(i + 1) * m + k]);
      }
    std::vector<double> Fx((size_t)(nx + 1) * m);
    for (int f = 0; f <= nx; ++f) {
      double ql[5], qr[5], al[3] = {0, 0, 0}, ar[3] = {0, 0, 0};
      for (int k = 0; k < m; ++k) {
        ql[k] = eL[(size_t)f * m + k];         // right edge of cell f-1
        qr[k] = eR[(size_t)(f + 1) * m + k];   // left edge of cell f
      }
      aux_of(j, f - 1, al);
      aux_of(j, f, ar);
      const double sp = num_flux(c, 0, ql, qr, al, ar, &Fx[(size_t)f * m]);
      smax = std::max(smax, sp / dx);
    }
    for (int i = 0; i < nx; ++i)
      for (int k = 0; k < m; ++k)
        L[((size_t)k * ny + j) * nx + i] -= (Fx[(size_t)(i + 1) * m + k] - Fx[(size_t)i * m + k]) / dx;
  }
  if (c.ndim == 2) {
#pragma omp parallel for schedule(static) reduction(max : smax)
    for (int i = 0; i < nx; ++i) {
      std::vector<double> eL((size_t)(ny + 2) * m), eR((size_t)(ny + 2) * m);
      for (int j = -1; j <= ny; ++j)
        for (int k = 0; k < m; ++k) {
          double v[17];
          for (int s = 0; s < w; ++s) v[s] = Q.at(k, j - (r - 1) + s, i);
          weno_edges(c, v, &eL[(size_t)(j + 1) * m + k], &eR[(size_t)(j + 1) * m + k]);
        }
      std::vector<double> Gy((size_t)(ny + 1) * m);
      for (int g = 0; g <= ny; ++g) {
        double ql[5], qr[5], al[3] = {0, 0, 0}, ar[3] = {0, 0, 0};
        for (int k = 0; k < m; ++k) {
          ql[k] = eL[(size_t)g * m + k];
          qr[k] = eR[(size_t)(g + 1) * m + k];
        }
        aux_of(g - 1, i, al);
        aux_of(g, i, ar);
        const double sp = num_flux(c, 1, ql, qr, al, ar, &Gy[(size_t)g * m]);
        smax = std::max(smax, sp / dy);
      }
      for (int j = 0; j < ny; ++j)
        for (int k = 0; k < m; ++k)
          L[((size_t)k * ny + j) * nx + i] -= (Gy[(size_t)(j + 1) * m + k] - Gy[(size_t)j * m + k]) / dy;
    }
  }
  return smax;
}

// SSP Runge-Kutta integrators over a semi-discrete operator Lop(q, out)
// (out = L(q); returns the largest speed/spacing, used from the first
// evaluation only: the Courant number is measured at Q^n).
//   SSPRK(3,3) (Shu-Osher):  Q1 = Q + dt L(Q);  Q2 = 3/4 Q + 1/4 (Q1 + dt L(Q1));
//                            Q^{n+1} = 1/3 Q + 2/3 (Q2 + dt L(Q2)).
//   SSPRK(10,4) (Ketcheson 2008, two-register form, SSP coefficient 6):
//     q1 = q2 = Q;  five times q1 += dt/6 L(q1);  q2 = q2/25 + 9/25 q1;
//     q1 = 15 q2 - 5 q1;  four times q1 += dt/6 L(q1);
//     Q^{n+1} = q2 + 3/5 q1 + dt/10 L(q1).
template <class Op>
double ssp_step(int integrator, Op&& Lop, size_t N, const double* qin, double* qout, double dt) {
  std::vector<double> L(N);
  if (integrator == 2) {
    std::vector<double> q1(qin, qin + N), q2(qin, qin + N);
    double smax = 0.0;
    for (int s = 0; s < 5; ++s) {
      const double sp = Lop(q1.data(), L.data());
      if (s == 0) smax = sp;
      for (size_t n = 0; n < N; ++n) q1[n] = q1[n] + dt / 6.0 * L[n];
    }
    for (size_t n = 0; n < N; ++n) {
      q2[n] = q2[n] / 25.0 + 9.0 / 25.0 * q1[n];
      q1[n] = 15.0 * q2[n] - 5.0 * q1[n];
    }
    for (int s = 0; s < 4; ++s) {
      Lop(q1.data(), L.data());
      for (size_t n = 0; n < N; ++n) q1[n] = q1[n] + dt / 6.0 * L[n];
    }
    Lop(q1.data(), L.data());
    for (size_t n = 0; n < N; ++n) qout[n] = q2[n] + 3.0 / 5.0 * q1[n] + dt / 10.0 * L[n];
    return smax;
  }
  std::vector<double> Q1(N), Q2(N);
  const double smax = Lop(qin, L.data());
  for (size_t n = 0; n < N; ++n) Q1[n] = qin[n] + dt * L[n];
  Lop(Q1.data(), L.data());
  for (size_t n = 0; n < N; ++n) Q2[n] = 0.75 * qin[n] + 0.25 * (Q1[n] + dt * L[n]);
  Lop(Q2.data(), L.data());
  for (size_t n = 0; n < N; ++n) qout[n] = qin[n] / 3.0 + 2.0 / 3.0 * (Q2[n] + dt * L[n]);
  return smax;
}

double sharpclaw_step(const OCfg& c, const double* qin, const double* aux, double* qout,
                      double dt) {
  const size_t N = (size_t)num_eqn(c) * c.nx * c.ny;
  return ssp_step(c.integrator,
                  [&](const double* q, double* L) { return sharpclaw_L(c, q, aux, L); }, N, qin,
                  qout, dt);
}

// Geometric source of the axisymmetric Euler equations (eq. euler-rz with the
// axial coordinate z = x and the radius r = y): the right-hand sides are
//   psi(q) = -(v / r) (rho, rho u, rho v, rho E + p)   (tracer: 0),
// v the radial velocity.  It is applied after the hyperbolic step as a
// fractional step (Section 2.1; LeVeque 2002, ch. 17), integrated over dt by
// Heun's method (explicit trapezoidal rule, second order):
//   q* = q + dt psi(q),   q <- q + dt/2 (psi(q) + psi(q*)),
// with r the radius of the cell centre.
void euler_axisym_psi(const OCfg& c, const double* q, double r, double* out) {
  const double rho = q[0], u = q[1] / rho, v = q[2] / rho, E = q[3];
  const double p = (c.pd[0] - 1.0) * (E - 0.5 * rho * (u * u + v * v));
  out[0] = -rho * v / r;
  out[1] = -q[1] * v / r;
  out[2] = -q[2] * v / r;
  out[3] = -(E + p) * v / r;
  out[4] = 0.0;
}

void source_step(const OCfg& c, double* q, double dt) {
  const int m = num_eqn(c), nx = c.nx, ny = c.ny;
  const size_t N = (size_t)nx * ny;
  const double dy = dy_of(c);
#pragma omp parallel for schedule(static)
  for (int j = 0; j < ny; ++j) {
    const double r = c.ylo + (j + 0.5) * dy;
    for (int i = 0; i < nx; ++i) {
      const size_t n = (size_t)j * nx + i;
      double q0[5], qs[5], f0[5], f1[5];
      for (int k = 0; k < m; ++k) q0[k] = q[k * N + n];
      euler_axisym_psi(c, q0, r, f0);
      for (int k = 0; k < m; ++k) qs[k] = q0[k] + dt * f0[k];
      euler_axisym_psi(c, qs, r, f1);
      for (int k = 0; k < m; ++k) q[k * N + n] = q0[k] + 0.5 * dt * (f0[k] + f1[k]);
    }
  }
}

bool has_source(const OCfg& c) { return c.source == 1 && c.solver == S_EULER_ROE && c.ndim == 2; }

double one_step(const OCfg& c, const double* qin, const double* aux, double* qout, double dt) {
  if (c.scheme == 2) return sharpclaw_step(c, qin, aux, qout, dt);
  if (c.ndim == 1) return classic_1d(c, qin, qout, dt);
  const double s = c.split ? classic_2d_split(c, qin, aux, qout, dt) : classic_2d(c, qin, aux, qout, dt);
  if (has_source(c)) source_step(c, qout, dt);
  return s;
}

// Largest characteristic speed over spacing among the cells: used for the
// a-priori first time step when none is given.
double max_cell_speed(const OCfg& c, const double* q, const double* aux) {
  const size_t N = (size_t)c.nx * c.ny;
  const double dx = dx_of(c), dy = dy_of(c);
  double best = 0.0;
  for (size_t n = 0; n < N; ++n) {
    double s = 0.0;
    switch (c.solver) {
      case S_ADV:
        s = std::fabs(c.pd[0]) / dx;
        if (c.ndim == 2) s = std::max(s, std::fabs(c.pd[1]) / dy);
        break;
      case S_SW: {
        const double h = q[n], cel = std::sqrt(c.pd[0] * h);
        s = (std::fabs(q[N + n] / h) + cel) / dx;
        if (c.ndim == 2) s = std::max(s, (std::fabs(q[2 * N + n] / h) + cel) / dy);
      } break;
      case S_EULER:
      case S_EULER_ROE: {
        // energy follows the momenta; a tracer (Euler Roe) comes last
        const double rho = q[n], u = q[N + n] / rho;
        const double v = c.ndim == 2 ? q[2 * N + n] / rho : 0.0;
        const double E = q[(size_t)(1 + c.ndim) * N + n];
        const double p = (c.pd[0] - 1.0) * (E - 0.5 * rho * (u * u + v * v));
        const double cs = std::sqrt(c.pd[0] * p / rho);
        s = (std::fabs(u) + cs) / dx;
        if (c.ndim == 2) s = std::max(s, (std::fabs(v) + cs) / dy);
      } break;
      case S_ELASTIC: {
        const double cp = std::sqrt((aux[N + n] + 2.0 * aux[2 * N + n]) / aux[n]);
        s = std::max(cp / dx, cp / dy);
      } break;
      case S_PSYS: {
        const double K = aux[n], rho = aux[N + n];
        const double cs = std::sqrt(K * std::exp(K * q[n]) / rho);
        s = cs / dx;
        if (c.ndim == 2) s = std::max(s, cs / dy);
      } break;
    }
    best = std::max(best, s);
  }
  return best;
}

}  // namespace

// ---------------------------------------------------------------------------
// C entry points used by the Python test harness.
// ---------------------------------------------------------------------------
extern "C" {

int or_num_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Number of OpenMP threads used by later calls (n >= 1; timing of the
// single-thread baseline).  No effect without OpenMP.
void or_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int or_num_eqn(const OCfg* c) { return num_eqn(*c); }
int or_num_waves(const OCfg* c) { return num_waves(*c); }
int or_num_aux(const OCfg* c) { return num_aux(*c); }

// One step of size dt from qin to qout.  *speed receives the largest
// |wave speed|/spacing over faces bounding interior cells (the Courant number
// of the step is dt * speed).
int or_step(const OCfg* c, const double* qin, const double* aux, double* qout, double dt,
            double* speed) {
  *speed = one_step(*c, qin, aux, qout, dt);
  return 0;
}

double or_max_cell_speed(const OCfg* c, const double* q, const double* aux) {
  return max_cell_speed(*c, q, aux);
}

// Time-step controller (Section 4: after each step the Courant number is
// checked against the stability limit and the next step size is chosen).
//   dt_try = min(dt, t_end - t); step; C = dt_try * speed;
//   C <= cfl_max: accept (t = t_end exactly on the clipped step), else keep Q^n;
//   dt = min(dt_max, dt_try * cfl_desired / C)  (dt_max if C == 0).
// q is updated in place.  Logs (optional, capacity log_cap): dt tried and
// whether it was accepted.  Returns 0, or -5 on a non-finite Courant number,
// or -8 when max_steps attempts did not reach t_end.
int or_advance(const OCfg* c, double* q, const double* aux, double* t_io, double t_end,
               double* dt_io, double cfl_desired, double cfl_max, double dt_max, long max_steps,
               double* dt_log, int* acc_log, long log_cap, long* n_acc, long* n_rej,
               double* max_courant) {
  const size_t N = (size_t)num_eqn(*c) * c->nx * c->ny;
  std::vector<double> qn(N);
  double t = *t_io, dt = *dt_io;
  if (dt_max <= 0.0) dt_max = std::numeric_limits<double>::infinity();
  if (dt <= 0.0) {
    const double s = max_cell_speed(*c, q, aux);
    dt = s > 0.0 ? std::min(dt_max, cfl_desired / s) : dt_max;
  }
  long acc = 0, rej = 0, attempts = 0;
  double cmax = 0.0;
  int rc = 0;
  while (t < t_end) {
    if (attempts >= max_steps) { rc = -8; break; }
    const bool clipped = t + dt >= t_end;
    const double dt_try = clipped ? t_end - t : dt;
    const double speed = one_step(*c, q, aux, qn.data(), dt_try);
    const double C = dt_try * speed;
    if (!(C == C) || std::isinf(C)) { rc = -5; break; }
    const bool ok = C <= cfl_max;
    if (dt_log && attempts < log_cap) { dt_log[attempts] = dt_try; acc_log[attempts] = ok ? 1 : 0; }
    ++attempts;
    if (ok) {
      std::memcpy(q, qn.data(), N * sizeof(double));
      t = clipped ? t_end : t + dt_try;
      ++acc;
      cmax = std::max(cmax, C);
    } else {
      ++rej;
    }
    dt = C > 0.0 ? std::min(dt_max, dt_try * cfl_desired / C) : dt_max;
  }
  *t_io = t;
  *dt_io = dt;
  *n_acc = acc;
  *n_rej = rej;
  *max_courant = cmax;
  return rc;
}

// The source fractional step alone (q in place), for its pins.
int or_source_step(const OCfg* c, double* q, double dt) {
  if (!has_source(*c)) return -1;
  source_step(*c, q, dt);
  return 0;
}

// Per-face Riemann solve (exposed for algebraic identity tests).
int or_riemann(const OCfg* c, int d, const double* ql, const double* qr, const double* auxl,
               const double* auxr, double* W /*[5][5]*/, double* s /*[5]*/, double* amdq,
               double* apdq) {
  FaceSol r;
  std::memset(&r, 0, sizeof(r));
  rp_normal(*c, d, ql, qr, auxl, auxr, r);
  std::memcpy(W, r.W, sizeof(r.W));
  std::memcpy(s, r.s, sizeof(r.s));
  std::memcpy(amdq, r.amdq, sizeof(r.amdq));
  std::memcpy(apdq, r.apdq, sizeof(r.apdq));
  return 0;
}

int or_transverse(const OCfg* c, int d, const double* ql, const double* qr, const double* aux_m,
                  const double* aux_c, const double* aux_p, const double* asdq, double* bm,
                  double* bp) {
  rp_transverse(*c, d, ql, qr, aux_m, aux_c, aux_p, asdq, bm, bp);
  return 0;
}

double or_num_flux(const OCfg* c, int d, const double* ql, const double* qr, const double* al,
                   const double* ar, double* F) {
  const double z[3] = {0.0, 0.0, 0.0};
  return num_flux(*c, d, ql, qr, al ? al : z, ar ? ar : z, F);
}

void or_weno5(const double* v, double eps, double* qL, double* qR) { weno5(v, eps, qL, qR); }

// General WENO of order 2r-1 (3 <= r <= 9) from 2r-1 averages.
int or_weno_r(int r, const double* v, double eps, double* qL, double* qR) {
  if (r < 2 || r > 9) return -1;
  weno_r(r, v, eps, qL, qR);
  return 0;
}

// Smoothness indicators beta_0 .. beta_{r-1} of the candidates of WENO
// order 2r-1 from 2r-1 averages.
int or_weno_smoothness(int r, const double* v, double* beta) {
  if (r < 2 || r > 9) return -1;
  const WenoTables& t = weno_tables(r);
  for (int k = 0; k < r; ++k) {
    double a, c;
    weno_candidate(t, k, v + k, &a, &c, &beta[k]);
  }
  return 0;
}

// Linear weights of WENO order 2r-1 (right edge), r entries.
int or_weno_linear_weights(int r, double* d) {
  if (r < 2 || r > 9) return -1;
  const WenoTables& t = weno_tables(r);
  for (int k = 0; k < r; ++k) d[k] = t.d[k];
  return 0;
}

// The SSP integrator of the SharpClaw step applied to the scalar Riccati
// equation y' = 1 - y^2 (exact solution tanh(t + atanh(y0))): n steps of
// size T/n from y0.  Pins the integrators' order on a nonlinear problem.
double or_ssp_riccati(int integrator, double y0, double T, int n) {
  double y = y0;
  const double dt = T / n;
  for (int s = 0; s < n; ++s) {
    double out;
    ssp_step(integrator, [](const double* q, double* L) { L[0] = 1.0 - q[0] * q[0]; return 0.0; },
             1, &y, &out, dt);
    y = out;
  }
  return y;
}

double or_limiter(int lim, double theta) { return limiter_phi(lim, theta); }

// Conserved totals: sum over cells of q_k * dx * dy.
void or_totals(const OCfg* c, const double* q, double* tot) {
  const int m = num_eqn(*c);
  const size_t N = (size_t)c->nx * c->ny;
  const double cell = dx_of(*c) * dy_of(*c);
  for (int k = 0; k < m; ++k) {
    double s = 0.0;
    for (size_t n = 0; n < N; ++n) s += q[(size_t)k * N + n];
    tot[k] = s * cell;
  }
}

}  // extern "C"
