// Sweep, frame and gradient kernels of precision F32, order 4.
#include "sbpe_launch_impl.h"

namespace sbpe {
template struct Launch<float, 4>;
}  // namespace sbpe
