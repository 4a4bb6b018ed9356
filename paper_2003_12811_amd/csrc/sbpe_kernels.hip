// Host-side launchers of the HIP kernels (gfx950) and the small kernels
// (time-function table, energy reduction, linear combinations, receiver
// adjoint, frame-operator probing).  The sweep, frame and gradient kernels
// are instantiated per (precision, order) in sbpe_inst_*.hip.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <mutex>

#include "sbpe_device.h"
#include "sbpe_launch.h"

namespace sbpe {

// ---------------------------------------------------------- tau table
// tau[(s * nitems + it) * 3 + k] = tau_it(t0 + s dt + c_k dt), c = (0, 1/2, 1)
__global__ void __launch_bounds__(256) k_tau(const TimeFn* items, int nitems, int nsteps, double t0, double dt,
                                             double* tau) {
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= (long)nitems * nsteps) return;
    const int s = (int)(idx / nitems), it = (int)(idx - (long)s * nitems);
    const GLB TimeFn& g = ((const GLB TimeFn*)items)[it];
    TimeFn f;
    f.kind = g.kind;
    f.pad = 0;
    f.p[0] = g.p[0];
    f.p[1] = g.p[1];
    const double t = t0 + s * dt;
    gp<double> o = gm<double>(tau) + 3 * idx;
    o[0] = tfun(f, t);
    o[1] = tfun(f, t + 0.5 * dt);
    o[2] = tfun(f, t + dt);
}

__global__ void __launch_bounds__(256) k_energy_final(const double* partial, int n, double* out) {
    __shared__ double red[256];
    double acc = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) acc += partial[k];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = 0.5 * red[0];
}

// ---------------------------------------------------------- launchers
// Two waves per tile when there are few tiles (the single-wave kernel needs
// more registers and fills fewer slots); SBPE_SPLIT=0/1 overrides.
bool split_tiles(int total_tiles) {
    static const int split_env = [] {
        const char* e = std::getenv("SBPE_SPLIT");
        return e ? std::atoi(e) : -1;
    }();
    return split_env >= 0 ? split_env != 0 : total_tiles < 4096;
}

bool sweep_fused(int total_tiles) {
    // one launch for frame and interior pays while the tiles alone do not
    // fill the machine; on larger grids the frame overlaps better from a
    // second stream.  SBPE_FUSED=0/1 overrides.
    static const int env = [] {
        const char* e = std::getenv("SBPE_FUSED");
        return e ? std::atoi(e) : -1;
    }();
    return env >= 0 ? env != 0 : split_tiles(total_tiles);
}

// calls f with a value of the typed launcher of (dtype, order)
template <typename F>
static void with_launch(int dtype, int order, F&& f) {
    if (dtype == 0) {
        if (order == 4) f(Launch<double, 4>{});
        else if (order == 6) f(Launch<double, 6>{});
        else f(Launch<double, 2>{});
    } else {
        if (order == 4) f(Launch<float, 4>{});
        else if (order == 6) f(Launch<float, 6>{});
        else f(Launch<float, 2>{});
    }
}

int launch_pass(int dtype, int order, const PassArgs& a, int total_tiles, int total_frame_wg, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    PassArgs b = a;
    b.total_tiles = total_tiles;
    b.total_frame_wg = total_frame_wg;
    with_launch(dtype, order, [&](auto L) { decltype(L)::pass(b, total_tiles, total_frame_wg, s); });
    return (int)hipGetLastError();
}

int launch_interior(int dtype, int order, const PassArgs& a, int total_tiles, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (total_tiles <= 0) return 0;
    PassArgs b = a;
    b.total_tiles = total_tiles;
    with_launch(dtype, order, [&](auto L) { decltype(L)::interior(b, total_tiles, s); });
    return static_cast<int>(hipGetLastError());
}

int launch_frame(int dtype, int order, const PassArgs& a, int total_frame_wg, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (total_frame_wg <= 0) return 0;
    with_launch(dtype, order, [&](auto L) { decltype(L)::frame(a, total_frame_wg, s); });
    return static_cast<int>(hipGetLastError());
}

int launch_tau(const TimeFn* items, int nitems, int nsteps, double t0, double dt, double* tau, void* stream) {
    const long n = (long)nitems * nsteps;
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_tau, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, static_cast<hipStream_t>(stream), items,
                       nitems, nsteps, t0, dt, tau);
    return static_cast<int>(hipGetLastError());
}

int launch_energy(int dtype, int order, const BlockDesc* blocks_dev, int nblocks, double* partial_dev,
                  int npartial, double* result_dev, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 g(npartial), bl(256);
    if (dtype == 0) {
        if (order == 4) hipLaunchKernelGGL((k_energy_partial<double, 4>), g, bl, 0, s, blocks_dev, nblocks, partial_dev);
        else if (order == 6) hipLaunchKernelGGL((k_energy_partial<double, 6>), g, bl, 0, s, blocks_dev, nblocks, partial_dev);
        else hipLaunchKernelGGL((k_energy_partial<double, 2>), g, bl, 0, s, blocks_dev, nblocks, partial_dev);
    } else {
        if (order == 4) hipLaunchKernelGGL((k_energy_partial<float, 4>), g, bl, 0, s, blocks_dev, nblocks, partial_dev);
        else if (order == 6) hipLaunchKernelGGL((k_energy_partial<float, 6>), g, bl, 0, s, blocks_dev, nblocks, partial_dev);
        else hipLaunchKernelGGL((k_energy_partial<float, 2>), g, bl, 0, s, blocks_dev, nblocks, partial_dev);
    }
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, s, partial_dev, npartial, result_dev);
    return static_cast<int>(hipGetLastError());
}

int launch_grad(int dtype, int order, const GradArgs& g, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (g.nblocks <= 0) return 0;
    with_launch(dtype, order, [&](auto L) { decltype(L)::grad(g, s); });
    return (int)hipGetLastError();
}

// band points of the gradient launches over these blocks
template <int ORD>
static long grad_band_points_t(const int* n1, const int* n2, int nblocks) {
    constexpr int LO = grad_lo<ORD>();
    long ob = 0;
    for (int b = 0; b < nblocks; ++b) {
        const long m1 = n1[b], m2 = n2[b];
        const long ni = (m1 > 2 * LO && m2 > 2 * LO) ? (m1 - 2 * LO) * (m2 - 2 * LO) : 0;
        ob += m1 * m2 - ni;
    }
    return ob;
}

long grad_band_points(int order, const int* n1, const int* n2, int nblocks) {
    return order == 2 ? grad_band_points_t<2>(n1, n2, nblocks) : grad_band_points_t<4>(n1, n2, nblocks);
}

int launch_lincomb(int dtype, int nterms, const double* c, const void* const* x, void* y, long count, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (count <= 0) return 0;
    const dim3 grid((unsigned)((count + 255) / 256)), bl(256);
    LincombArgs a;
    for (int k = 0; k < LINCOMB_MAX; ++k) {
        a.c[k] = k < nterms ? c[k] : 0.0;
        a.x[k] = k < nterms ? x[k] : x[0];
    }
    if (dtype == 0) hipLaunchKernelGGL(k_lincomb<double>, grid, bl, 0, s, nterms, a, (double*)y, count);
    else hipLaunchKernelGGL(k_lincomb<float>, grid, bl, 0, s, nterms, a, (float*)y, count);
    return (int)hipGetLastError();
}

int launch_rk4_stages(int dtype, const Rk4StageArgs& a, long count, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (count <= 0) return 0;
    const dim3 grid((unsigned)((count + 255) / 256)), bl(256);
    if (dtype == 0) hipLaunchKernelGGL(k_rk4_stages<double>, grid, bl, 0, s, a, count);
    else hipLaunchKernelGGL(k_rk4_stages<float>, grid, bl, 0, s, a, count);
    return (int)hipGetLastError();
}

int launch_rec_adjoint(int dtype, const RecAdj* ent, int nent, const double* r, const RecAdjArgs& a, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (nent <= 0) return 0;
    const dim3 grid((unsigned)((nent + 255) / 256)), bl(256);
    if (dtype == 0) hipLaunchKernelGGL(k_rec_adjoint<double>, grid, bl, 0, s, ent, nent, r, a);
    else hipLaunchKernelGGL(k_rec_adjoint<float>, grid, bl, 0, s, ent, nent, r, a);
    return (int)hipGetLastError();
}

int launch_probe_fill(int dtype, void* x, int n1, int n2, int comp, int cx, int cy, int period, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    const long n = 2L * n1 * n2;
    const dim3 grid((unsigned)((n + 255) / 256)), bl(256);
    if (dtype == 0) hipLaunchKernelGGL(k_probe_fill<double>, grid, bl, 0, s, (double*)x, n1, n2, comp, cx, cy, period);
    else hipLaunchKernelGGL(k_probe_fill<float>, grid, bl, 0, s, (float*)x, n1, n2, comp, cx, cy, period);
    return (int)hipGetLastError();
}

int launch_frame_gather(int dtype, const void* y, int n1, int n2, int R, int frame_n, void* out, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (frame_n <= 0) return 0;
    const dim3 grid((unsigned)((frame_n + 255) / 256)), bl(256);
    if (dtype == 0)
        hipLaunchKernelGGL(k_frame_gather<double>, grid, bl, 0, s, (const double*)y, n1, n2, R, frame_n, (double*)out);
    else hipLaunchKernelGGL(k_frame_gather<float>, grid, bl, 0, s, (const float*)y, n1, n2, R, frame_n, (float*)out);
    return (int)hipGetLastError();
}

int launch_frame_sp(int dtype, int order, const PassArgs& a0, int total_frame_wg, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (total_frame_wg <= 0) return 0;
    PassArgs a = a0;
    a.total_frame_wg = total_frame_wg;
    const long pts = (long)total_frame_wg * FRAME_PTS;
    const dim3 g((unsigned)((pts + FRAME_WG / FRAME_LANES - 1) / (FRAME_WG / FRAME_LANES))), b(FRAME_WG);
    with_launch(dtype, order, [&](auto L) { decltype(L)::frame_sp(a, g, b, s); });
    return (int)hipGetLastError();
}

// ------------------------------------------------- no-allocation scratch
// The time-function table of sbpe_advance_noalloc lives in this file-scope
// device array: one copy per GPU, kept until the process ends and shared by
// every context on that GPU.  In host code `scratch` is only a stand-in for
// the symbol; its device address is looked up once per device (with that
// device current) and only that address is handed to kernels.
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};
}  // namespace

int scratch_init(int device) {
    if (device < 0 || device >= MAX_DEVICES) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return 0;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return (int)e;
    g_scratch_ptr[device] = static_cast<double*>(ptr);
    return 0;
}

double* scratch_ptr(int device) {
    if (device < 0 || device >= MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

const char* hip_error_string(int code) { return hipGetErrorString(static_cast<hipError_t>(code)); }

}  // namespace sbpe
