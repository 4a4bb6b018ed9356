// Interior and one-launch sweep kernels of precision F32, order 2.
#include "sbpe_launch_impl.h"

namespace sbpe {
template void Launch<float, 2>::interior(const PassArgs&, int, hipStream_t);
template void Launch<float, 2>::pass(const PassArgs&, int, int, hipStream_t);
}  // namespace sbpe
