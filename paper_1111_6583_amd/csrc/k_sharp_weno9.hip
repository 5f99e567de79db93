// k_sharp_weno9.hip -- SharpClaw stage kernels with ninth-order WENO (r = 5).
#include "k_sharp.h"

namespace claw {
template hipError_t launch_sharp_order<5>(int, int, int, int, dim3, hipStream_t, const GridDesc*,
                                           int, double, const StageArgs&);
}  // namespace claw
