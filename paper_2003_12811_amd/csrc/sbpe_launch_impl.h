// Definitions of the typed launchers (sbpe_launch.h); included only by the
// sbpe_inst_*.hip translation units, each of which instantiates some of the
// members of one (precision, order) pair.
#pragma once
#include "sbpe_device.h"
#include "sbpe_launch.h"

namespace sbpe {

template <typename T, int ORD>
static void launch_march_t(const PassArgs& a, int total_tiles, hipStream_t s) {
    const dim3 g(((total_tiles + 7) / 8) * 8), bl(64), bl2(128);
    const bool split = split_tiles(total_tiles);
    if (a.pass == PASS_APPLY) hipLaunchKernelGGL((k_march<T, ORD, PASS_APPLY, false>), g, bl, 0, s, a);
    else if (a.pass == PASS_RK1 && split) hipLaunchKernelGGL((k_march<T, ORD, PASS_RK1, true>), g, bl2, 0, s, a);
    else if (a.pass == PASS_RK1) hipLaunchKernelGGL((k_march<T, ORD, PASS_RK1, false>), g, bl, 0, s, a);
    else if (split) hipLaunchKernelGGL((k_march<T, ORD, PASS_RK2, true>), g, bl2, 0, s, a);
    else hipLaunchKernelGGL((k_march<T, ORD, PASS_RK2, false>), g, bl, 0, s, a);
}

template <typename T, int ORD>
static void launch_pass_t(const PassArgs& a, int total_tiles, int total_frame_wg, hipStream_t s) {
    const bool split = a.pass != PASS_APPLY && split_tiles(total_tiles);
    const int nt = split ? 128 : 64;
    // frame workgroups (nt / FRAME_LANES points each), rounded to whole XCD rounds
    const long fpts = (long)total_frame_wg * FRAME_PTS;
    const int ppw = nt / FRAME_LANES;
    const int floop = a.floop > 1 ? a.floop : 1;   // frame groups per frame workgroup
    const long ngroups = (fpts + ppw - 1) / ppw;
    const int nframe = (int)(((ngroups + floop - 1) / floop + 7) / 8 * 8);
    const dim3 g(nframe + ((total_tiles + 7) / 8) * 8), bl(nt);
    if (a.pass == PASS_APPLY) hipLaunchKernelGGL((k_pass<T, ORD, PASS_APPLY, false>), g, bl, 0, s, a, nframe, floop);
    else if (a.pass == PASS_RK1 && split) hipLaunchKernelGGL((k_pass<T, ORD, PASS_RK1, true>), g, bl, 0, s, a, nframe, floop);
    else if (a.pass == PASS_RK1) hipLaunchKernelGGL((k_pass<T, ORD, PASS_RK1, false>), g, bl, 0, s, a, nframe, floop);
    else if (split) hipLaunchKernelGGL((k_pass<T, ORD, PASS_RK2, true>), g, bl, 0, s, a, nframe, floop);
    else hipLaunchKernelGGL((k_pass<T, ORD, PASS_RK2, false>), g, bl, 0, s, a, nframe, floop);
}

template <typename T, int ORD>
static void launch_pass_wide_t(const PassArgs& a, int total_tiles, int total_frame_wg, hipStream_t s) {
    const long fpts = (long)total_frame_wg * FRAME_PTS;
    const int ppw = 64 / FRAME_LANES;
    const int floop = a.floop > 1 ? a.floop : 1;
    const long ngroups = (fpts + ppw - 1) / ppw;
    const int nframe = (int)(((ngroups + floop - 1) / floop + 7) / 8 * 8);
    const dim3 g(nframe + ((total_tiles + 7) / 8) * 8), bl(64);
    if (a.pass == PASS_APPLY) hipLaunchKernelGGL((k_pass_wide<T, ORD, PASS_APPLY>), g, bl, 0, s, a, nframe, floop);
    else if (a.pass == PASS_RK1) hipLaunchKernelGGL((k_pass_wide<T, ORD, PASS_RK1>), g, bl, 0, s, a, nframe, floop);
    else hipLaunchKernelGGL((k_pass_wide<T, ORD, PASS_RK2>), g, bl, 0, s, a, nframe, floop);
}

template <typename T, int ORD>
static void launch_wide_t(const PassArgs& a, int total_tiles, hipStream_t s) {
    const dim3 g(((total_tiles + 7) / 8) * 8), bl(64);
    if (a.pass == PASS_APPLY) hipLaunchKernelGGL((k_wide<T, ORD, PASS_APPLY>), g, bl, 0, s, a);
    else if (a.pass == PASS_RK1) hipLaunchKernelGGL((k_wide<T, ORD, PASS_RK1>), g, bl, 0, s, a);
    else hipLaunchKernelGGL((k_wide<T, ORD, PASS_RK2>), g, bl, 0, s, a);
}

template <typename T, int ORD>
static void launch_grad_t(GradArgs g, hipStream_t s) {
    // interior and band point counts per block (cumulative)
    constexpr int LO = grad_lo<ORD>();
    long oi = 0, ob = 0;
    for (int b = 0; b < g.nblocks; ++b) {
        const long n1 = g.n1[b], n2 = g.n2[b];
        const long ni = (n1 > 2 * LO && n2 > 2 * LO) ? (n1 - 2 * LO) * (n2 - 2 * LO) : 0;
        g.off[b] = oi;
        g.boff[b] = ob;
        oi += ni;
        ob += n1 * n2 - ni;
    }
    g.off[g.nblocks] = oi;
    g.boff[g.nblocks] = ob;
    g.nband = ob;
    if (oi > 0) hipLaunchKernelGGL((k_grad_int<T, ORD>), dim3((unsigned)((oi + 255) / 256)), dim3(256), 0, s, g);
    if (ob > 0) {
        // one workgroup row per stage; several stages meet in k_grad_band_sum
        hipLaunchKernelGGL((k_grad<T, ORD>), dim3((unsigned)((ob + 63) / 64), (unsigned)g.nstages),
                           dim3(GRAD_PARTS * 64), 0, s, g);
        if (g.nstages > 1)
            hipLaunchKernelGGL((k_grad_band_sum<ORD>), dim3((unsigned)((ob + 255) / 256)), dim3(256), 0, s, g);
    }
}

template <typename T, int ORD>
static void launch_frame_sp_t(const PassArgs& a, dim3 g, dim3 b, hipStream_t s) {
    if (a.pass == PASS_APPLY) hipLaunchKernelGGL((k_frame_sp<T, ORD, PASS_APPLY>), g, b, 0, s, a);
    else if (a.pass == PASS_RK1) hipLaunchKernelGGL((k_frame_sp<T, ORD, PASS_RK1>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_frame_sp<T, ORD, PASS_RK2>), g, b, 0, s, a);
}

// The wide-stencil operator and the coefficient gradient are built for
// orders 2 and 4 (the host refuses them at order 6).
template <typename T, int ORD>
void Launch<T, ORD>::interior(const PassArgs& a, int total_tiles, hipStream_t s) {
    if constexpr (ORD != 6) {
        if (a.wide) {
            launch_wide_t<T, ORD>(a, total_tiles, s);
            return;
        }
    }
    launch_march_t<T, ORD>(a, total_tiles, s);
}

template <typename T, int ORD>
void Launch<T, ORD>::pass(const PassArgs& a, int total_tiles, int total_frame_wg, hipStream_t s) {
    if constexpr (ORD != 6) {
        if (a.wide) {
            launch_pass_wide_t<T, ORD>(a, total_tiles, total_frame_wg, s);
            return;
        }
    }
    launch_pass_t<T, ORD>(a, total_tiles, total_frame_wg, s);
}

template <typename T, int ORD>
void Launch<T, ORD>::frame(const PassArgs& a, int total_frame_wg, hipStream_t s) {
    hipLaunchKernelGGL((k_frame<T, ORD>), dim3(total_frame_wg), dim3(FRAME_WG), 0, s, a);
}

template <typename T, int ORD>
void Launch<T, ORD>::frame_sp(const PassArgs& a, dim3 g, dim3 b, hipStream_t s) {
    launch_frame_sp_t<T, ORD>(a, g, b, s);
}

template <typename T, int ORD>
void Launch<T, ORD>::grad(GradArgs g, hipStream_t s) {
    if constexpr (ORD != 6) launch_grad_t<T, ORD>(g, s);
}

}  // namespace sbpe
