// k_sharp.hip -- SharpClaw stage launches: the kernels of WENO5 and WENO7
// (k_sharp.h) and the dispatch over the WENO order.
#include "k_sharp.h"

namespace claw {

// prec: 0 FP64, 1 FP32 with Kahan-compensated final stage, 2 plain FP32
// (2D Euler with WENO5 only)
hipError_t launch_sharp_stage(int ndim, int riemann, int prec, int weno_r, int kind, int nblocks,
                              hipStream_t st, const GridDesc* d_grids, int mode, double dt,
                              const StageArgs& sa) {
  const dim3 grid(nblocks);
  if (prec == 2) {
    if (ndim != 2 || riemann != 3 || weno_r != 3) return hipErrorInvalidValue;
    return sharp_kind<float, false, 2, 3>(riemann, kind, grid, st, d_grids, mode, dt, sa);
  }
  const int fp32 = prec;
  switch (weno_r) {
    case 3: return launch_sharp_order<3>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
    case 4: return launch_sharp_order<4>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
    case 5: return launch_sharp_order<5>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
    case 6: return launch_sharp_order<6>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
    case 7: return launch_sharp_order<7>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
    case 8: return launch_sharp_order<8>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
    case 9: return launch_sharp_order<9>(ndim, riemann, fp32, kind, grid, st, d_grids, mode, dt, sa);
  }
  return hipErrorInvalidValue;
}

}  // namespace claw
