// Frame and gradient kernels of precision F32, order 2.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<float, 2>::frame(const PassArgs&, int, hipStream_t);
template void Launch<float, 2>::frame_sp(const PassArgs&, dim3, dim3, hipStream_t);
template void Launch<float, 2>::grad(GradArgs, hipStream_t);
}  // namespace sbpe
