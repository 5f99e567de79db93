// k_sharp_weno15.hip -- SharpClaw stage kernels with fifteenth-order WENO (r = 8).
#include "k_sharp.h"

namespace claw {
template hipError_t launch_sharp_order<8>(int, int, int, int, dim3, hipStream_t, const GridDesc*,
                                           int, double, const StageArgs&);
}  // namespace claw
