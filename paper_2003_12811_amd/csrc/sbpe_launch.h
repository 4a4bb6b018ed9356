// Typed launchers of the large kernels.  Each (precision, order) pair is
// instantiated in two translation units of its own, the sweeps
// (sbpe_inst_<type>_o<order>_sweep.hip) and the frame and gradient kernels
// (..._frame.hip), so the library builds in parallel; sbpe_kernels.hip
// dispatches to them.
#pragma once
#include <hip/hip_runtime.h>

#include "sbpe_internal.h"

namespace sbpe {

// Two waves per tile when there are few tiles (SBPE_SPLIT=0/1 overrides).
bool split_tiles(int total_tiles);

template <typename T, int ORD>
struct Launch {
    // interior tiles only (k_march, or k_wide for the wide-stencil operator)
    static void interior(const PassArgs& a, int total_tiles, hipStream_t s);
    // one launch for frame and tiles (k_pass, or k_pass_wide)
    static void pass(const PassArgs& a, int total_tiles, int total_frame_wg, hipStream_t s);
    // the stencil form of the frame rows (k_frame)
    static void frame(const PassArgs& a, int total_frame_wg, hipStream_t s);
    // the assembled frame operator (k_frame_sp)
    static void frame_sp(const PassArgs& a, dim3 g, dim3 b, hipStream_t s);
    // coefficient gradient of one or more stages (k_grad_int, k_grad, k_grad_band_sum)
    static void grad(GradArgs g, hipStream_t s);
};

extern template struct Launch<double, 4>;
extern template struct Launch<double, 2>;
extern template struct Launch<float, 4>;
extern template struct Launch<float, 2>;
extern template struct Launch<double, 6>;
extern template struct Launch<float, 6>;

}  // namespace sbpe
