// Interior and one-launch sweep kernels of precision F64, order 6.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<double, 6>::interior(const PassArgs&, int, hipStream_t);
template void Launch<double, 6>::pass(const PassArgs&, int, int, hipStream_t);
}  // namespace sbpe
