// Frame and gradient kernels of precision F64, order 4.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<double, 4>::frame(const PassArgs&, int, hipStream_t);
template void Launch<double, 4>::frame_sp(const PassArgs&, dim3, dim3, hipStream_t);
template void Launch<double, 4>::grad(GradArgs, hipStream_t);
}  // namespace sbpe
