// dev_common.h -- device helpers for the gfx950 kernels: lane shuffles,
// boundary-condition index maps, Courant reduction and the device-side step
// controller.
#pragma once

#include "claw_internal.h"

namespace claw {

// ---------------------------------------------------------------------------
// Lane shifts inside one 64-lane wavefront.  x-neighbours of a cell live in
// adjacent lanes of the marching kernels; prev = value held by lane-1,
// next = value held by lane+1.  They are DPP wavefront shifts (wave_shr:1 /
// wave_shl:1, one VALU move per 32 bits, no LDS).  bound_ctrl makes the edge
// lanes (no source lane) receive 0 without a prior write of the destination;
// they are halo lanes whose results are discarded.
// ---------------------------------------------------------------------------
constexpr int kDppWaveShr1 = 0x138;   // lane l reads lane l-1
constexpr int kDppWaveShl1 = 0x130;   // lane l reads lane l+1

template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ float shfl_prev(float x) { return dpp_f<kDppWaveShr1>(x); }
__device__ __forceinline__ float shfl_next(float x) { return dpp_f<kDppWaveShl1>(x); }
__device__ __forceinline__ double shfl_prev(double x) { return dpp_d<kDppWaveShr1>(x); }
__device__ __forceinline__ double shfl_next(double x) { return dpp_d<kDppWaveShl1>(x); }

// Maximum that keeps a NaN (so a non-finite state reaches the Courant check).
template <typename R>
__device__ __forceinline__ R max_nan(R a, R b) { return (b > a || b != b) ? b : a; }

template <typename R>
__device__ __forceinline__ R wave_max(R v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max_nan(v, __shfl_xor(v, off, kLanes));
  return v;
}

// ---------------------------------------------------------------------------
// Reciprocal and reciprocal square root: the hardware estimate refined by one
// Newton step.  Measured on MI355X over 2^20 arguments spanning 2^-12..2^12:
// the FP64 estimates are within 4.6e-8 (rcp) and 5.2e-8 (rsq) relative, one
// step brings them to 2.1e-15 and 4.1e-15, a second to 1.1e-16 and 2.6e-16.
// One step is far inside the 1e-12 parity bar and saves two (rcp) or three
// (rsq) FP64 instructions per call on the kernels' instruction-issue-bound
// path.  FP32 uses the single-instruction estimates (about 1 ulp).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double frcp(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  const double e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frsq(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  return y * __builtin_fma(-0.5 * x, y * y, 1.5);
}
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
// sqrt(x) for x > 0
__device__ __forceinline__ double fsqrt(double x) { return x * frsq(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// ---------------------------------------------------------------------------
// Boundary conditions as index maps (ghost cells are never stored).  A ghost
// index outside [0, n) maps to the interior cell it copies, with a flag for a
// wall (normal-odd components flip sign) or a Dirichlet side.  Indices beyond
// the ghost width h are clamped first (they only occur in discarded lanes).
// ---------------------------------------------------------------------------
enum { kBcExtrap = 1, kBcPeriodic = 2, kBcWall = 3, kBcDirichlet = 4 };

struct AxisMap {
  int idx;    // interior index to read
  int kind;   // 0 plain, 1 wall (flip normal-odd components), 2 Dirichlet
  int side;   // 0 lower, 1 upper (for Dirichlet)
};

__device__ __forceinline__ AxisMap map_axis(int i, int n, int bc_lo, int bc_hi, int h) {
  // branch-free: every index maps to an interior cell (selects, no jumps)
  const bool lo = i < 0, hi = i >= n;
  i = i < -h ? -h : i;
  i = i > n - 1 + h ? n - 1 + h : i;
  const int bc = lo ? bc_lo : bc_hi;
  const int per = lo ? i + n : i - n;
  const int mir = lo ? -1 - i : 2 * n - 1 - i;
  const int edge = lo ? 0 : n - 1;
  const int gidx = bc == kBcPeriodic ? per : (bc == kBcWall ? mir : edge);
  AxisMap m;
  m.idx = (lo || hi) ? gidx : i;
  m.kind = (lo || hi) ? (bc == kBcWall ? 1 : (bc == kBcDirichlet ? 2 : 0)) : 0;
  m.side = hi ? 1 : 0;
  return m;
}

// Device arrays are addressed through global-address-space pointers: loads
// and stores then become global_* instructions, which count only against the
// vector-memory counter (flat_* ones also hold the scalar-memory counter and
// make every scalar load wait for them).
#define CLAW_GLOBAL __attribute__((address_space(1)))
template <typename T> using gconst = const CLAW_GLOBAL T*;
template <typename T> using gmut = CLAW_GLOBAL T*;
template <typename T>
__device__ __forceinline__ gconst<T> as_gconst(const void* p) { return (gconst<T>)p; }
template <typename T>
__device__ __forceinline__ gmut<T> as_gmut(void* p) { return (gmut<T>)p; }

// Ghost values that do not come from memory (Dirichlet sides), held in
// registers for the whole kernel instead of being re-read per row.
template <typename R, int M>
struct EdgeStates {
  R x[M];             // this lane's x side (used if its column is a Dirichlet ghost)
  R ylo[M], yhi[M];   // lower / upper y side
  bool xany;          // some lane of the wave maps a wall or Dirichlet ghost column
};
template <typename R, int M>
__device__ __forceinline__ EdgeStates<R, M> edge_states(const GridDesc& G, const AxisMap& mx) {
  EdgeStates<R, M> e;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    e.x[k] = (R)(mx.side ? G.bcstate[1][k] : G.bcstate[0][k]);
    e.ylo[k] = (R)G.bcstate[2][k];
    e.yhi[k] = (R)G.bcstate[3][k];
  }
  // wave-uniform, so strips away from such a boundary skip the x fix-up
  e.xany = __builtin_amdgcn_ballot_w64(mx.kind != 0) != 0;
  return e;
}

// A cell's state is read in two steps so that a row can be prefetched: the
// raw load of the mapped interior cell (always in bounds), then, once the
// data is needed, the boundary conditions.  The x map is applied first and
// the y map last, so a corner ghost is the y-boundary image of an x ghost.
template <typename R, int M>
__device__ __forceinline__ void load_raw(R (&v)[M], gconst<R> q, size_t plane, int nx,
                                         const AxisMap& mx, const AxisMap& my) {
  const size_t off = (size_t)my.idx * nx + mx.idx;
#pragma unroll
  for (int k = 0; k < M; ++k) v[k] = q[k * plane + off];
}
template <typename R, class P>
__device__ __forceinline__ void apply_bc(R (&v)[P::M], const AxisMap& mx, const AxisMap& my,
                                         const EdgeStates<R, P::M>& e) {
  // both branches are wave-uniform (the row's map is the same for every
  // lane); a plain map needs no fix-up
  if (e.xany) {
#pragma unroll
    for (int k = 0; k < P::M; ++k) {
      R x = mx.kind == 2 ? e.x[k] : v[k];
      if (P::odd(0, k)) x = mx.kind == 1 ? -x : x;
      v[k] = x;
    }
  }
  if (my.kind != 0) {
#pragma unroll
    for (int k = 0; k < P::M; ++k) {
      R x = v[k];
      if (P::odd(1, k)) x = my.kind == 1 ? -x : x;
      v[k] = my.kind == 2 ? (my.side ? e.yhi[k] : e.ylo[k]) : x;
    }
  }
}
template <typename R, class P>
__device__ __forceinline__ void load_state(R (&v)[P::M], gconst<R> q, size_t plane, int nx,
                                           const AxisMap& mx, const AxisMap& my,
                                           const EdgeStates<R, P::M>& e) {
  load_raw<R, P::M>(v, q, plane, nx, mx, my);
  apply_bc<R, P>(v, mx, my, e);
}

// Aux fields: ghost cells copy the mapped interior cell (no sign flips; a
// Dirichlet side copies the edge cell).  No fix-up step: prefetchable as is.
template <typename R, class P>
__device__ __forceinline__ void load_aux(R (&a)[P::NA > 0 ? P::NA : 1], gconst<R> aux,
                                         size_t plane, int nx, const AxisMap& mx,
                                         const AxisMap& my) {
  if constexpr (P::NA > 0) {
    const size_t off = (size_t)my.idx * nx + mx.idx;
#pragma unroll
    for (int k = 0; k < P::NA; ++k) a[k] = aux[k * plane + off];
  } else {
    a[0] = R(0);
  }
}

// ---------------------------------------------------------------------------
// Courant reduction and the device-side controller.
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long dbits(double x) {
  return (unsigned long long)__double_as_longlong(x);
}
__device__ __forceinline__ double bitsd(unsigned long long b) {
  return __longlong_as_double((long long)b);
}

// Controller update after an attempt whose largest speed/spacing is `speed`.
// Same arithmetic as the host controller.  Returns whether it was accepted.
__device__ inline bool ctrl_decide(Ctrl* c, double speed) {
  const double dt_try = c->dt_try;
  const double C = dt_try * speed;
  c->last_speed = speed;
  if (!(C == C) || C == __builtin_inf()) {
    c->status = -5;
    c->active = 0;
    return false;
  }
  const bool ok = C <= c->cfl_max;
  c->attempts += 1;
  if (ok) {
    c->t = c->clipped ? c->t_end : c->t + dt_try;
    c->accepted += 1;
    c->max_courant = C > c->max_courant ? C : c->max_courant;
  } else {
    c->rejected += 1;
  }
  double dt = C > 0.0 ? dt_try * c->cfl_desired / C : c->dt_max;
  c->dt = dt < c->dt_max ? dt : c->dt_max;
  // the next attempt
  if (!(c->t < c->t_end) || (c->max_attempts > 0 && c->attempts >= c->max_attempts)) {
    c->active = 0;
  } else {
    c->clipped = c->t + c->dt >= c->t_end;
    c->dt_try = c->clipped ? c->t_end - c->t : c->dt;
  }
  return ok;
}

// End-of-workgroup bookkeeping: fold this wave's max speed into the launch's
// reduction; the last workgroup of the launch (over this grid) hands the
// total to `decide` (the device controller, or just recording it for the
// host controller) and clears the reduction for the next launch.
//
// Two levels, so that no single address takes one atomic per workgroup
// (device-scope atomics on one address are performed one after another, about
// 11 ns each on this GPU, and the workgroups of a launch end nearly together):
// workgroup b folds into slot b mod S (S = min(64, nblocks) slots, 256 bytes
// apart) and counts itself there; the workgroup completing a slot counts the
// slot in the controller's counter; the one completing the counter reduces
// the S slot maxima with its whole wave and decides.
//
// Ordering without fences: every step is a device-scope read-modify-write
// whose result is returned, and each next step's operand depends on the
// previous result (the asm ties), so a completed slot count implies every
// maximum of that slot was performed, and a completed controller count
// implies every slot was.  The final loads are device-scope atomic loads
// issued after that.  No release/acquire fence is used: on this GPU a
// device-scope fence writes back and invalidates the whole L2 of the XCD,
// which every workgroup would do at once at the end of each launch.  The
// controller fields the last workgroup writes with plain stores are read by
// the next launch (kernel boundaries order them).
template <class Decide>
__device__ inline void finish_workgroup(Ctrl* c, SpeedSlot* slots, int blk, int nblocks,
                                        double local_max, Decide decide) {
  local_max = wave_max(local_max);   // NaN-preserving: NaN bits compare above every finite speed
  const int ns = nblocks < kSpeedSlots ? nblocks : kSpeedSlots;
  CLAW_GLOBAL SpeedSlot* sl = (CLAW_GLOBAL SpeedSlot*)slots;
  CLAW_GLOBAL Ctrl* g = (CLAW_GLOBAL Ctrl*)c;
  int last = 0;
  if (threadIdx.x == 0) {
    const int k = blk % ns;
    const unsigned int nk = (unsigned int)(nblocks / ns + (k < nblocks % ns ? 1 : 0));
    const unsigned long long prev = __hip_atomic_fetch_max(
        &sl[k].max_bits, dbits(local_max), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned int one = 1u;
    asm volatile("" : "+v"(one) : "v"(prev));
    const unsigned int done =
        __hip_atomic_fetch_add(&sl[k].count, one, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == nk - 1) {
      __hip_atomic_store(&sl[k].count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      unsigned int one2 = 1u;
      asm volatile("" : "+v"(one2) : "v"(done));
      const unsigned int full =
          __hip_atomic_fetch_add(&g->counter, one2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      last = full == (unsigned int)(ns - 1) ? 1 : 0;
    }
  }
  last = __builtin_amdgcn_readfirstlane(last);
  if (last) {
    const int j = threadIdx.x;
    double v = 0.0;
    if (j < ns) {
      v = bitsd(__hip_atomic_load(&sl[j].max_bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      __hip_atomic_store(&sl[j].max_bits, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const double speed = wave_max(v);
    if (threadIdx.x == 0) {
      decide(c, speed);
      __hip_atomic_store(&g->counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Locate this workgroup's grid in a batch: block_start[g] <= b < block_start[g+1].
__device__ __forceinline__ int find_grid(const int* __restrict__ bstart, int ngrids, int b) {
  if (ngrids <= 1) return 0;
  int lo = 0, hi = ngrids - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

}  // namespace claw
