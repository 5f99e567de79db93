// claw_internal.h -- structures shared by the host library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace claw {

constexpr int kLanes = 64;        // one wavefront per workgroup in the marching kernels
constexpr int kMaxEqn = 5;
constexpr int kMaxAux = 3;

// Device-resident step controller of one grid (Section 4: after each step
// the Courant number is checked and the next step size chosen).
struct Ctrl {
  unsigned int counter;           // speed slots of the current launch that are complete
  int src;                        // buffer index holding Q^n (classic ping-pong)
  int active;                     // 1 while t < t_end and attempts remain
  int ok;                         // SharpClaw: the current attempt passed the stage-1 check
  int status;                     // 0, or CLAW_E_NONPHYSICAL
  int clipped;                    // dt_try was clipped to t_end - t
  double t, t_end;
  double dt;                      // the controller's running dt
  double dt_try;                  // dt of the attempt about to run (min(dt, t_end - t))
  double dt_stage;                // SharpClaw: dt used by stages 2 and 3 of the current attempt
  double cfl_desired, cfl_max, dt_max;
  long long accepted, rejected, attempts, max_attempts;
  double max_courant;
  double last_speed;              // speed of the most recent attempt (diagnostics / host mode)
  unsigned long long sweep_bits[2];   // split steps: speed maxima of the sweeps before the last
};

// One slot of the two-level Courant reduction at the end of a launch (see
// finish_workgroup): a maximum and a count of the workgroups folded into it.
constexpr int kSpeedSlots = 64;
struct SpeedSlot {
  unsigned long long max_bits;    // max|s|/spacing (bit pattern of a non-negative double)
  unsigned int count;
  unsigned int pad[61];           // one slot per 256 bytes
};

// First row of segment `seg` when n rows are split into `segs` segments as
// evenly as possible (sizes differ by at most one row).
__host__ __device__ __forceinline__ int seg_begin(int seg, int n, int segs) {
  return (int)(((long long)seg * n) / segs);
}

// Tile (strip, segment) of workgroup lb of a grid with `strips` x `segs`
// tiles.  order 0: strips fastest; 1: segments fastest; 2 and 3: the same
// over XCD-grouped indices.  Consecutive workgroups of a launch go round-robin
// to the GPU's 8 XCDs (each with its own L2); grouping gives XCD x the
// contiguous band of tiles [start_x, start_x + count_x), so tiles that share
// halo rows or columns mostly share an L2.  A bijection for any tile count;
// results do not depend on the order.
constexpr int kXcds = 8;
__host__ __device__ __forceinline__ void tile_of(int lb, int strips, int segs, int order,
                                                 int& strip, int& seg) {
  int t = lb;
  if (order >= 2) {
    const int n = strips * segs, q = n / kXcds, r = n % kXcds;
    const int x = lb % kXcds, k = lb / kXcds;
    t = x * q + (x < r ? x : r) + k;
  }
  if (order & 1) {
    seg = t % segs;
    strip = t / segs;
  } else {
    strip = t % strips;
    seg = t / strips;
  }
}

// Everything a kernel needs about one grid.  Lives in device memory.
struct GridDesc {
  int nx, ny;
  int strips, segs;               // column strips x row segments = workgroups
  int seg_rows;                   // rows of the longest segment
  int nblocks;                    // workgroups of one launch over this grid
  int order;                      // tile order of the workgroups (see tile_of)
  int bc[4];                      // x-lower, x-upper, y-lower, y-upper
  int limiter, transverse, efix, scheme;
  int source;                     // 1: axisymmetric Euler source (r = y), fractional step
  double dx, dy;
  double ylo;                     // lower y of the domain (radius of the source term)
  double weno_eps;
  double cfl_max;                 // split steps: a sweep above it ends the Courant reading
  double bcstate[4][8];
  double pd[8];
  void* q[2];                     // state ping-pong (Real)
  void* c[2];                     // compensation ping-pong (Real, FP32 mode)
  void* s1;                       // SharpClaw stage buffers (Real)
  void* s2;
  void* s3;                       // SharpClaw SSPRK(10,4): the second register
  int weno_r;                     // SharpClaw: WENO order 2r-1 (r = 3 or 4)
  const void* aux;                // aux fields (Real)
  Ctrl* ctrl;
  SpeedSlot* slots;               // kSpeedSlots slots of the launch-end reduction
};

// One SharpClaw Runge-Kutta stage (see k_sharp.hip): y = S + gamma dt L(S),
// then PLAIN out1 = y; COMBINE out1 = a1 P1 + b1 y (and out2 = a2 P1 + b2 y
// if out2 is set); FINAL Q = a1 P1 + b1 y in place.  FINAL_Q is FINAL with
// P1 = Q^n known at compile time (SSPRK(3,3)): the compensated FP32 kernels
// then keep one copy of Q^n instead of two (launch-side choice).
enum StageKind { kStagePlain = 0, kStageCombine = 1, kStageFinal = 2, kStageFinalQ = 3 };
struct StageArgs {
  const void* in;    // S
  void* out1;
  void* out2;        // or null
  const void* p1;    // pointwise input of COMBINE / FINAL
  double gamma, a1, b1, a2, b2;
  double w;          // FINAL, FP32 increment form: a1 (P1 - w Q) + b1 ((S - Q) + gamma dt L)
  int first;         // first stage of an attempt: Courant number + controller
  int p1_is_q;       // FINAL: P1 is Q itself
};

// One 1D sweep of a dimensionally split classic step (see k_split.hip).  A
// null state pointer stands for the step's own buffers: `in` / `cin` for
// q / c[src] (Q^n), `out` / `cout` for q / c[src ^ 1] (Q^{n+1}), so that a
// captured sweep follows the controller's ping-pong.
struct SweepArgs {
  const void* in;
  const void* cin;   // compensation of `in` (FP32 mode)
  void* out;
  void* cout;
  double frac;       // the sweep advances frac * dt
  int index;         // position of the sweep in the step (0, 1, 2)
  int final_sweep;   // last sweep of the step: applies the source, closes the Courant reduction
  int nblocks;       // workgroups of this launch
  int strips;        // column strips (workgroups per row segment)
  int segs;          // row segments (rows split as evenly as possible)
};

// How a kernel obtains dt and the source buffer.
enum StepMode { kHostDt = 0, kDeviceCtrl = 1 };

}  // namespace claw
