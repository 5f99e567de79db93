// k_sharp_weno17.hip -- SharpClaw stage kernels with seventeenth-order WENO (r = 9).
#include "k_sharp.h"

namespace claw {
template hipError_t launch_sharp_order<9>(int, int, int, int, dim3, hipStream_t, const GridDesc*,
                                           int, double, const StageArgs&);
}  // namespace claw
