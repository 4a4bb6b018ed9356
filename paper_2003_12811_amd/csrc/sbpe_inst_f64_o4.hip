// Sweep, frame and gradient kernels of precision F64, order 4.
#include "sbpe_launch_impl.h"

namespace sbpe {
template struct Launch<double, 4>;
}  // namespace sbpe
