// Frame and gradient kernels of precision F64, order 6.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<double, 6>::frame(const PassArgs&, int, hipStream_t);
template void Launch<double, 6>::frame_sp(const PassArgs&, dim3, dim3, hipStream_t);
template void Launch<double, 6>::grad(GradArgs, hipStream_t);
}  // namespace sbpe
