// k_sharp_weno11.hip -- SharpClaw stage kernels with eleventh-order WENO (r = 6).
#include "k_sharp.h"

namespace claw {
template hipError_t launch_sharp_order<6>(int, int, int, int, dim3, hipStream_t, const GridDesc*,
                                           int, double, const StageArgs&);
}  // namespace claw
