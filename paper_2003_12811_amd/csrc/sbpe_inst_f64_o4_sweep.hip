// Interior and one-launch sweep kernels of precision F64, order 4.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<double, 4>::interior(const PassArgs&, int, hipStream_t);
template void Launch<double, 4>::pass(const PassArgs&, int, int, hipStream_t);
}  // namespace sbpe
