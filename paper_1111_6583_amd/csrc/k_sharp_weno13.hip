// k_sharp_weno13.hip -- SharpClaw stage kernels with thirteenth-order WENO (r = 7).
#include "k_sharp.h"

namespace claw {
template hipError_t launch_sharp_order<7>(int, int, int, int, dim3, hipStream_t, const GridDesc*,
                                           int, double, const StageArgs&);
}  // namespace claw
