// Interior and one-launch sweep kernels of precision F32, order 4.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<float, 4>::interior(const PassArgs&, int, hipStream_t);
template void Launch<float, 4>::pass(const PassArgs&, int, int, hipStream_t);
}  // namespace sbpe
