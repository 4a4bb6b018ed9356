// Device code (gfx950, wave64) of the SBP-SAT anisotropic elastic operator:
// every kernel template, included by the translation units that instantiate
// and launch them (sbpe_kernels.hip and the sbpe_inst_*.hip files).
//
// One right-hand-side evaluation is split by grid region:
//   * k_march: points at least Frame<ORD>::R from every face, where all 1-D
//     operators use their repeating interior stencils (Sec. 4.3-4.7).  One
//     wave spans 64 consecutive columns, writes the central 64 - 2H of them
//     and marches over the rows of its tile: input rows are staged once in
//     an LDS ring (x1 neighbours and the x2 window of the own column),
//     coefficient windows stay in registers, and the mixed terms go through
//     an LDS row (D_1 G) and a register window (D_2 E);
//   * k_frame: the band of width R along the faces, where the boundary
//     closures of D1 and D2^FC and the SATs of Sec. 5 and 6 act; one thread
//     per point, closure rows unrolled from compile-time tables.
// Both are fused with the two-sweep form of classical RK4 described in
// sbpe_internal.h, so one RK4 step streams the coefficient fields twice.
//
// Reference-frame forms used here (all follow from the paper's definitions):
//   * volume: DD_ik(c_ijkl) u_l = D_11^FC(c_1j1l) u_l + D_22^FC(c_2j2l) u_l
//             + D_1 (c_1j2l D_2 u_l) + D_2 (c_2j1l D_1 u_l)   (eq. def_cd, Sec. 4.7)
//   * Jhat T_jl = nu_i c_ijkl D_k                              (eq. n-C_conversion)
//   * Jhat Z_jl = beta d / h_1 nu_i c_ijkl nu_k (displacement; / 4 and summed
//     over both sides at interfaces), from Nanson's formula (eq. nanson)
//   * J (JH)^{-1} e_f Jhat H_f = (1 / h_1) at the face points (H = H_x1 (x) H_x2)
//   * H_t^{-1} D_t^T H_t = -D_t + H_t^{-1} (e_N e_N^T - e_0 e_0^T)  (SBP property, Sec. 4)
// Second differences are formed from differences u_m - u_r first (every row of
// D2^FC and D1 sums to zero), which keeps FP32 cancellation small.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "sbpe_internal.h"
#include "sbpe_tables.h"

namespace sbpe {

// Every field lives in global memory; loads and stores go through
// address-space-1 pointers so that they compile to global (not flat) accesses,
// which the compiler can batch freely around LDS traffic.
#define GLB __attribute__((address_space(1)))
template <typename T> using gcp = const GLB T*;
template <typename T> using gp = GLB T*;
template <typename T>
__device__ __forceinline__ gcp<T> gc(const void* p) { return (gcp<T>)p; }
template <typename T>
__device__ __forceinline__ gp<T> gm(void* p) { return (gp<T>)p; }
using BlockRef = const GLB BlockDesc&;
__device__ __forceinline__ BlockRef blk(const PassArgs& A, int b) { return ((const GLB BlockDesc*)A.blocks)[b]; }
__device__ __forceinline__ const GLB Entry& entry(BlockRef B, int e) { return ((const GLB Entry*)B.entries)[e]; }
__device__ __forceinline__ Range load_range(const Range* base, int k) {
    const GLB Range& r = ((const GLB Range*)base)[k];
    Range o;
    o.beg = r.beg;
    o.mid = r.mid;
    o.end = r.end;
    o.pad = 0;
    return o;
}
// calls fn(E) for every entry in [beg, end) at point p; the point indices
// are loaded four at a time so that a long range costs few round trips
template <typename F>
__device__ __forceinline__ void entries_at(BlockRef B, int beg, int end, long p, F&& fn) {
    for (int e = beg; e < end; e += 4) {
        int pe[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) pe[u] = e + u < end ? entry(B, e + u).p : -1;
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if ((long)pe[u] == p) fn(entry(B, e + u));
    }
}

template <int ORD> struct Op;
template <> struct Op<4> {
    static constexpr int R0 = O4_R0, W = O4_W, NB = O4_NB, HALF = 2, REACH = 4, D1W = 6;
    __host__ __device__ static constexpr double d2c(int r, int m, int s) { return D2T4.t[r][m][s]; }
    __host__ __device__ static constexpr double d1b(int r, int c) { return O4_D1B[r][c]; }
    __host__ __device__ static constexpr double d1i(int k) { return O4_D1I[k]; }
    __host__ __device__ static constexpr double hb(int k) { return O4_H[k]; }
};
template <> struct Op<2> {
    static constexpr int R0 = O2_R0, W = O2_W, NB = O2_NB, HALF = 1, REACH = 2, D1W = 6;
    __host__ __device__ static constexpr double d2c(int r, int m, int s) { return D2T2.t[r][m][s]; }
    __host__ __device__ static constexpr double d1b(int r, int c) { return O2_D1B[r][c]; }
    __host__ __device__ static constexpr double d1i(int k) { return O2_D1I[k]; }
    __host__ __device__ static constexpr double hb(int k) { return O2_H[k]; }
};
template <> struct Op<6> {
    static constexpr int R0 = O6_R0, W = O6_W, NB = O6_NB, HALF = 3, REACH = 6, D1W = O6_D1W;
    __host__ __device__ static constexpr double d2c(int r, int m, int s) { return D2T6.t[r][m][s]; }
    __host__ __device__ static constexpr double d1b(int r, int c) { return O6_D1B[r][c]; }
    __host__ __device__ static constexpr double d1i(int k) { return O6_D1I[k]; }
    __host__ __device__ static constexpr double hb(int k) { return O6_H[k]; }
};

// h (D1 u)_i at an interior point from the values at offsets +-1 .. +-H:
// sum_o d1i(H + o) (u(+o) - u(-o)); at(o) returns the value at offset o
template <int ORD, typename T, typename F>
__device__ __forceinline__ T d1_sym(F&& at) {
    using O = Op<ORD>;
    T acc = static_cast<T>(O::d1i(O::HALF + 1)) * (at(1) - at(-1));
#pragma unroll
    for (int o = 2; o <= O::HALF; ++o) acc += static_cast<T>(O::d1i(O::HALF + o)) * (at(o) - at(-o));
    return acc;
}

// weight of u_{i+2} - u_{i-2} in the interior first derivative (0 at order 2)
template <int ORD>
__host__ __device__ constexpr double d1_outer() {
    if constexpr (Op<ORD>::HALF > 1) return Op<ORD>::d1i(Op<ORD>::HALF + 2);
    else return 0.0;
}

// closure table entries with runtime indices
template <int ORD>
__device__ __forceinline__ double table_d2c(int r, int m, int s) {
    if constexpr (ORD == 6) return D2T6.t[r][m][s];
    else if constexpr (ORD == 4) return D2T4.t[r][m][s];
    else return D2T2.t[r][m][s];
}
template <int ORD>
__device__ __forceinline__ double table_d1b(int r, int c) {
    if constexpr (ORD == 6) return O6_D1B[r][c];
    else if constexpr (ORD == 4) return O4_D1B[r][c];
    else return O2_D1B[r][c];
}

// dimensionless norm weight of point k on a line of n points
template <int ORD>
__device__ __forceinline__ double hnorm(int k, int n) {
    using O = Op<ORD>;
    if (k < O::NB) return O::hb(k);
    if (k > n - 1 - O::NB) return O::hb(n - 1 - k);
    return 1.0;
}

__device__ __forceinline__ double tfun(const TimeFn& f, double t) {
    switch (f.kind) {
        case TF_ONE: return 1.0;
        case TF_COS: return cos(f.p[0] * t + f.p[1]);
        case TF_RICKER: {
            const double a = (M_PI * f.p[0] * (t - f.p[1])) * (M_PI * f.p[0] * (t - f.p[1]));
            return (1.0 - 2.0 * a) * exp(-a);
        }
        default: return 0.0;
    }
}

// weights of the three tabulated values tau(t), tau(t + dt/2), tau(t + dt)
struct W3 {
    double w0, w1, w2;
    __device__ bool any() const { return w0 != 0.0 || w1 != 0.0 || w2 != 0.0; }
};
__device__ __forceinline__ W3 weights_a(const PassArgs& A) { return W3{A.wa[0], A.wa[1], A.wa[2]}; }
// second-evaluation weights; in the second RK sweep they multiply 2/dt^2 of the block
__device__ __forceinline__ W3 weights_b(const PassArgs& A, BlockRef B) {
    const double s = A.pass == PASS_RK2 ? 2.0 / (B.dt * B.dt) : 1.0;
    return W3{s * A.wb[0], s * A.wb[1], s * A.wb[2]};
}

// weighted time-function value of an item in this step
__device__ __forceinline__ double tval(BlockRef B, const PassArgs& A, int item, const W3& w) {
    const GLB double* t = (const GLB double*)B.tau + ((long)(A.step - B.step0) * B.nitems + item) * 3;
    return w.w0 * t[0] + w.w1 * t[1] + w.w2 * t[2];
}

// receiver slots of the current step, or null
__device__ __forceinline__ gp<double> rec_slots(BlockRef B, const PassArgs& A) {
    if (!B.rec) return nullptr;
    return (gp<double>)B.rec + (long)(A.rec_base + A.step - B.step0) * B.rec_stride;
}
// sbpe_apply operand of block b.  The kernel argument is read through an
// unrolled select: indexing it with a runtime block number would make the
// compiler copy the whole argument block into per-lane scratch memory.
__device__ __forceinline__ const void* apply_in(const PassArgs& A, int b) {
    const void* p = A.in[0];
#pragma unroll
    for (int k = 1; k < MAX_APPLY_BLOCKS; ++k)
        if (b == k) p = A.in[k];
    return p;
}
__device__ __forceinline__ void* apply_out(const PassArgs& A, int b) {
    void* p = A.out[0];
#pragma unroll
    for (int k = 1; k < MAX_APPLY_BLOCKS; ++k)
        if (b == k) p = A.out[k];
    return p;
}

template <typename T>
__device__ __forceinline__ gcp<T> field_ptr(const PassArgs& A, int b, int fld) {
    BlockRef B = blk(A, b);
    switch (fld) {
        case FLD_U: return gc<T>(B.u);
        case FLD_V: return gc<T>(B.v);
        case FLD_A1: return gc<T>(B.a1);
        case FLD_A2: return gc<T>(B.a2);
        default: return gc<T>(apply_in(A, b));
    }
}

// ------------------------------------------------------------ 1-D rows
// D1 row r of a line of n points: calls f(index, weight * h) for its nonzero
// entries; closure rows are unrolled from the compile-time tables.
template <int ORD, int RR, typename F>
__device__ __forceinline__ void d1_closure_foreach(bool lo, int n, F&& f) {
    using O = Op<ORD>;
#pragma unroll
    for (int c = 0; c < O::D1W; ++c)
        if (O::d1b(RR, c) != 0.0) f(lo ? c : n - 1 - c, lo ? O::d1b(RR, c) : -O::d1b(RR, c));
}

template <int ORD, int RR, typename F>
__device__ __forceinline__ void d1_dispatch(int rr, bool lo, int n, F&& f) {
    if constexpr (RR < Op<ORD>::NB) {
        if (rr == RR) d1_closure_foreach<ORD, RR>(lo, n, f);
        else d1_dispatch<ORD, RR + 1>(rr, lo, n, f);
    }
}

template <int ORD, typename F>
__device__ __forceinline__ void d1_foreach(int r, int n, F&& f) {
    using O = Op<ORD>;
    if (r >= O::NB && r <= n - 1 - O::NB) {
#pragma unroll
        for (int k = -O::HALF; k <= O::HALF; ++k)
            if (k != 0) f(r + k, O::d1i(k + O::HALF));
        return;
    }
    const bool lo = r < O::NB;
    d1_dispatch<ORD, 0>(lo ? r : n - 1 - r, lo, n, f);
}

// h (D1 u)_r on a line with element stride st (difference form)
template <typename T, int ORD>
__device__ __forceinline__ T d1_line(gcp<T> u, long st, int r, int n) {
    const T ur = u[(long)r * st];
    T acc = 0;
    d1_foreach<ORD>(r, n, [&](int k, double w) { acc += static_cast<T>(w) * (u[(long)k * st] - ur); });
    return acc;
}

template <typename T, int ORD>
__device__ __forceinline__ void d2_weights(const T* b, T* k);
template <typename T, int ORD>
__device__ __forceinline__ T d2_edges(const T* k, const T* u);

// h^2 (D2^FC(b) u)_r at an interior row; b, u point at the row.
template <typename T, int ORD, typename PB, typename PU>
__device__ __forceinline__ T d2_interior(PB b, PU u, long st) {
    const T u0 = u[0];
    if constexpr (ORD == 6) {
        T bb[7], kk[6], uu[7];
#pragma unroll
        for (int o = 0; o < 7; ++o) {
            bb[o] = b[(o - 3) * st];
            uu[o] = u[(o - 3) * st];
        }
        d2_weights<T, 6>(bb, kk);
        return d2_edges<T, 6>(kk, uu);
    } else if constexpr (ORD == 4) {
        const T bm2 = b[-2 * st], bm1 = b[-st], b0 = b[0], bp1 = b[st], bp2 = b[2 * st];
        const T s6 = T(1) / T(6), e8 = T(0.125), hf = T(0.5);
        const T km2 = s6 * bm1 - e8 * (bm2 + b0);
        const T km1 = s6 * (bm2 + bp1) + hf * (bm1 + b0);
        const T kp1 = s6 * (bm1 + bp2) + hf * (b0 + bp1);
        const T kp2 = s6 * bp1 - e8 * (b0 + bp2);
        return km2 * (u[-2 * st] - u0) + km1 * (u[-st] - u0) + kp1 * (u[st] - u0) + kp2 * (u[2 * st] - u0);
    } else {
        const T hf = T(0.5);
        return hf * (b[-st] + b[0]) * (u[-st] - u0) + hf * (b[0] + b[st]) * (u[st] - u0);
    }
}

// The interior row of h^2 D2^FC(b) in edge form: weights k of the differences
// u_m - u_0 for m = -H..-1, 1..H, from b on the 2H+1 points of the row.
template <typename T, int ORD>
__device__ __forceinline__ void d2_weights(const T* b, T* k) {
    if constexpr (ORD == 6) {
        // weights of u_{i+m} - u_i, m = -3, -2, -1, 1, 2, 3, from b_{i-3} .. b_{i+3}
        const T a = T(11) / T(360), e = T(0.025), f = T(0.05), g = T(0.3), c7 = T(0.175), c17 = T(0.425);
        k[0] = a * (b[0] + b[3]) - e * (b[1] + b[2]);
        k[1] = g * b[2] - f * (b[0] + b[4]) - c7 * (b[1] + b[3]);
        k[2] = e * (b[0] + b[5]) + g * (b[1] + b[4]) + c17 * (b[2] + b[3]);
        k[3] = e * (b[1] + b[6]) + g * (b[2] + b[5]) + c17 * (b[3] + b[4]);
        k[4] = g * b[4] - f * (b[2] + b[6]) - c7 * (b[3] + b[5]);
        k[5] = a * (b[3] + b[6]) - e * (b[4] + b[5]);
    } else if constexpr (ORD == 4) {
        const T s6 = T(1) / T(6), e8 = T(0.125), hf = T(0.5);
        k[0] = s6 * b[1] - e8 * (b[0] + b[2]);
        k[1] = s6 * (b[0] + b[3]) + hf * (b[1] + b[2]);
        k[2] = s6 * (b[1] + b[4]) + hf * (b[2] + b[3]);
        k[3] = s6 * b[3] - e8 * (b[2] + b[4]);
    } else {
        const T hf = T(0.5);
        k[0] = hf * (b[0] + b[1]);
        k[1] = hf * (b[1] + b[2]);
    }
}
template <typename T, int ORD>
__device__ __forceinline__ T d2_edges(const T* k, const T* u) {
    if constexpr (ORD == 6) {
        const T u0 = u[3];
        return k[0] * (u[0] - u0) + k[1] * (u[1] - u0) + k[2] * (u[2] - u0) + k[3] * (u[4] - u0) +
               k[4] * (u[5] - u0) + k[5] * (u[6] - u0);
    } else if constexpr (ORD == 4) {
        const T u0 = u[2];
        return k[0] * (u[0] - u0) + k[1] * (u[1] - u0) + k[2] * (u[3] - u0) + k[3] * (u[4] - u0);
    } else {
        const T u0 = u[1];
        return k[0] * (u[0] - u0) + k[1] * (u[2] - u0);
    }
}

// closure row RR (from the lower end, or mirrored at the upper end)
template <typename T, int ORD, int RR>
__device__ __forceinline__ T d2_closure(gcp<T> b, gcp<T> u, long st, bool lo, int n) {
    using O = Op<ORD>;
    const T ur = u[(long)(lo ? RR : n - 1 - RR) * st];
    T acc = 0;
    if constexpr (ORD == 6) {
        // the order-6 closure rows are 12 wide: a loop over the table keeps
        // the frame kernels small (they run at setup and on the frame band only)
        for (int m = 0; m < O::W; ++m) {
            if (m == RR) continue;
            T cf = 0;
#pragma unroll 4
            for (int s = 0; s < O::W; ++s) cf += static_cast<T>(table_d2c<ORD>(RR, m, s)) * b[(long)(lo ? s : n - 1 - s) * st];
            acc += cf * (u[(long)(lo ? m : n - 1 - m) * st] - ur);
        }
        return acc;
    }
#pragma unroll
    for (int m = 0; m < O::W; ++m) {
        if (m == RR) continue;
        T cf = 0;
        bool any = false;
#pragma unroll
        for (int s = 0; s < O::W; ++s) {
            if (O::d2c(RR, m, s) != 0.0) {
                cf += static_cast<T>(O::d2c(RR, m, s)) * b[(long)(lo ? s : n - 1 - s) * st];
                any = true;
            }
        }
        if (any) acc += cf * (u[(long)(lo ? m : n - 1 - m) * st] - ur);
    }
    return acc;
}

template <typename T, int ORD, int RR>
__device__ __forceinline__ T d2_dispatch(int rr, gcp<T> b, gcp<T> u, long st, bool lo, int n) {
    if constexpr (RR < Op<ORD>::R0) {
        if (rr == RR) return d2_closure<T, ORD, RR>(b, u, st, lo, n);
        return d2_dispatch<T, ORD, RR + 1>(rr, b, u, st, lo, n);
    } else {
        return T(0);
    }
}

// h^2 (D2^FC(b) u)_r on a line of n points; b, u point at index 0 of the line.
template <typename T, int ORD>
__device__ __forceinline__ T d2_line(gcp<T> b, gcp<T> u, long st, int r, int n) {
    using O = Op<ORD>;
    if (r >= O::R0 && r <= n - 1 - O::R0) return d2_interior<T, ORD>(b + r * st, u + r * st, st);
    const bool lo = r < O::R0;
    return d2_dispatch<T, ORD, 0>(lo ? r : n - 1 - r, b, u, st, lo, n);
}

// h^2 (D1 b D1 u)_r on a line of n points (the wide-stencil second
// derivative); b, u point at index 0 of the line.
template <typename T, int ORD>
__device__ __forceinline__ T wide_line(gcp<T> b, gcp<T> u, long st, int r, int n) {
    T acc = 0;
    d1_foreach<ORD>(r, n, [&](int k, double w) { acc += static_cast<T>(w) * b[(long)k * st] * d1_line<T, ORD>(u, st, k, n); });
    return acc;
}

template <typename T, int ORD>
__device__ __forceinline__ T second_line(bool wide, gcp<T> b, gcp<T> u, long st, int r, int n) {
    if constexpr (ORD == 6) return d2_line<T, ORD>(b, u, st, r, n);   // the wide operator is built for orders 2, 4
    else return wide ? wide_line<T, ORD>(b, u, st, r, n) : d2_line<T, ORD>(b, u, st, r, n);
}

// -------------------------------------------------- volume at one point
// One of the four term groups of DD_ik(c_ijkl) u_l at (i, j) with
// boundary-aware 1-D rows (frame points):
//   PART 0: D_11^FC(c_1j1l) u_l        PART 1: D_22^FC(c_2j2l) u_l
//   PART 2: D_1 (c_1j2l D_2 u_l)       PART 3: D_2 (c_2j1l D_1 u_l)
// With wide set, parts 0 and 1 take D_i c D_i instead of D_ii^FC(c).
template <typename T, int ORD, int PART>
__device__ __forceinline__ void volume_part(BlockRef B, gcp<T> u, int i, int j, T& r0, T& r1, bool wide) {
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    gcp<T> c = gc<T>(B.coef);
    gcp<T> u0 = u;
    gcp<T> u1 = u + np;
    const T ih1 = T(1.0 / B.h1), ih2 = T(1.0 / B.h2);
    const long rj = (long)j * n1;
    if constexpr (PART == 0) {
        const T a00 = second_line<T, ORD>(wide, c + K_C1111 * np + rj, u0 + rj, 1, i, n1);
        const T a01 = second_line<T, ORD>(wide, c + K_C1112 * np + rj, u1 + rj, 1, i, n1);
        const T a10 = second_line<T, ORD>(wide, c + K_C1112 * np + rj, u0 + rj, 1, i, n1);
        const T a11 = second_line<T, ORD>(wide, c + K_C1212 * np + rj, u1 + rj, 1, i, n1);
        r0 += (a00 + a01) * ih1 * ih1;
        r1 += (a10 + a11) * ih1 * ih1;
    } else if constexpr (PART == 1) {
        const T b00 = second_line<T, ORD>(wide, c + K_C2121 * np + i, u0 + i, n1, j, n2);
        const T b01 = second_line<T, ORD>(wide, c + K_C2122 * np + i, u1 + i, n1, j, n2);
        const T b10 = second_line<T, ORD>(wide, c + K_C2122 * np + i, u0 + i, n1, j, n2);
        const T b11 = second_line<T, ORD>(wide, c + K_C2222 * np + i, u1 + i, n1, j, n2);
        r0 += (b00 + b01) * ih2 * ih2;
        r1 += (b10 + b11) * ih2 * ih2;
    } else if constexpr (PART == 2) {
        // D_1 (M D_2 u), M_jl = c_1j2l
        T g0 = 0, g1 = 0;
        d1_foreach<ORD>(i, n1, [&](int ii, double w) {
            const T w20 = d1_line<T, ORD>(u0 + ii, n1, j, n2);
            const T w21 = d1_line<T, ORD>(u1 + ii, n1, j, n2);
            const long q = rj + ii;
            const T m00 = c[K_C1121 * np + q], m01 = c[K_C1122 * np + q];
            const T m10 = c[K_C1221 * np + q], m11 = c[K_C1222 * np + q];
            g0 += static_cast<T>(w) * (m00 * w20 + m01 * w21);
            g1 += static_cast<T>(w) * (m10 * w20 + m11 * w21);
        });
        r0 += g0 * ih1 * ih2;
        r1 += g1 * ih1 * ih2;
    } else {
        // D_2 (M^T D_1 u), c_2j1l = c_1l2j
        T e0 = 0, e1 = 0;
        d1_foreach<ORD>(j, n2, [&](int jj, double w) {
            const long rjj = (long)jj * n1;
            const T w10 = d1_line<T, ORD>(u0 + rjj, 1, i, n1);
            const T w11 = d1_line<T, ORD>(u1 + rjj, 1, i, n1);
            const long q = rjj + i;
            const T m00 = c[K_C1121 * np + q], m01 = c[K_C1122 * np + q];
            const T m10 = c[K_C1221 * np + q], m11 = c[K_C1222 * np + q];
            e0 += static_cast<T>(w) * (m00 * w10 + m10 * w11);
            e1 += static_cast<T>(w) * (m01 * w10 + m11 * w11);
        });
        r0 += e0 * ih1 * ih2;
        r1 += e1 * ih1 * ih2;
    }
}

// --------------------------------------------------------- face helpers
struct FacePt {
    int i, j;   // grid point
};

__device__ __forceinline__ FacePt face_point(BlockRef B, int f, int t) {
    const int a = f >> 1, s = f & 1;
    FacePt q;
    if (a == 0) {
        q.i = s ? B.n1 - 1 : 0;
        q.j = t;
    } else {
        q.i = t;
        q.j = s ? B.n2 - 1 : 0;
    }
    return q;
}

// normal-narrow matrix N_a (c_ajal) and mixed matrix M (c_1j2l) at flat index q
template <typename T>
__device__ __forceinline__ void coef_mats(gcp<T> c, long np, long q, int a, T N[2][2], T M[2][2]) {
    if (a == 0) {
        N[0][0] = c[K_C1111 * np + q];
        N[0][1] = N[1][0] = c[K_C1112 * np + q];
        N[1][1] = c[K_C1212 * np + q];
    } else {
        N[0][0] = c[K_C2121 * np + q];
        N[0][1] = N[1][0] = c[K_C2122 * np + q];
        N[1][1] = c[K_C2222 * np + q];
    }
    M[0][0] = c[K_C1121 * np + q];
    M[0][1] = c[K_C1122 * np + q];
    M[1][0] = c[K_C1221 * np + q];
    M[1][1] = c[K_C1222 * np + q];
}

// Jhat T_jl u_l = nu_a c_ajkl D_k u_l at point t of face f
template <typename T, int ORD>
__device__ __forceinline__ void traction_at(BlockRef B, gcp<T> u, int f, int t, T& tr0, T& tr1) {
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const int a = f >> 1;
    const T nu = (f & 1) ? T(1) : T(-1);
    const FacePt q = face_point(B, f, t);
    const long p = (long)q.j * n1 + q.i;
    gcp<T> c = gc<T>(B.coef);
    T d1[2], d2[2];
    for (int l = 0; l < 2; ++l) {
        d1[l] = d1_line<T, ORD>(u + l * np + (long)q.j * n1, 1, q.i, n1) * T(1.0 / B.h1);
        d2[l] = d1_line<T, ORD>(u + l * np + q.i, n1, q.j, n2) * T(1.0 / B.h2);
    }
    T N[2][2], M[2][2];
    coef_mats(c, np, p, a, N, M);
    if (a == 0) {   // c_1j1l D1 u_l + c_1j2l D2 u_l
        tr0 = nu * (N[0][0] * d1[0] + N[0][1] * d1[1] + M[0][0] * d2[0] + M[0][1] * d2[1]);
        tr1 = nu * (N[1][0] * d1[0] + N[1][1] * d1[1] + M[1][0] * d2[0] + M[1][1] * d2[1]);
    } else {        // c_2j1l D1 u_l + c_2j2l D2 u_l, c_2j1l = M_lj
        tr0 = nu * (M[0][0] * d1[0] + M[1][0] * d1[1] + N[0][0] * d2[0] + N[0][1] * d2[1]);
        tr1 = nu * (M[0][1] * d1[0] + M[1][1] * d1[1] + N[1][0] * d2[0] + N[1][1] * d2[1]);
    }
}

// displacement-type jump delta at point t of face f:
//   HOM:  field on this face (minus the partner's field at an interface)
//   DATA: -tau g (displacement) or -vsign tau V (interface)
template <typename T, bool DATA>
__device__ __forceinline__ void face_delta(const PassArgs& A, int b, int f, int t, int fld, const W3& tc, T& d0,
                                           T& d1) {
    BlockRef B = blk(A, b);
    const GLB FaceDesc& F = B.face[f];
    const long np = (long)B.n1 * B.n2;
    if (!DATA) {
        gcp<T> u = field_ptr<T>(A, b, fld);
        const FacePt q = face_point(B, f, t);
        const long p = (long)q.j * B.n1 + q.i;
        d0 = u[p];
        d1 = u[np + p];
        if (F.kind == BC_INTERFACE) {
            BlockRef P = blk(A, F.partner);
            gcp<T> v = field_ptr<T>(A, F.partner, fld);
            const int tp = F.reversed ? F.nf - 1 - t : t;
            const FacePt qp = face_point(P, F.pface, tp);
            const long pp = (long)qp.j * P.n1 + qp.i;
            const long npp = (long)P.n1 * P.n2;
            d0 -= v[pp];
            d1 -= v[npp + pp];
        }
    } else {
        d0 = 0;
        d1 = 0;
        if (F.kind == BC_DISPLACEMENT && F.g) {
            const T tau = static_cast<T>(tval(B, A, F.item_g, tc));
            gcp<T> g = gc<T>(F.g);
            d0 = -tau * g[t];
            d1 = -tau * g[F.nf + t];
        } else if (F.kind == BC_INTERFACE && F.V) {
            const T tau = static_cast<T>(F.vsign * tval(B, A, F.item_v, tc));
            gcp<T> V = gc<T>(F.V);
            d0 = -tau * V[t];
            d1 = -tau * V[F.nf + t];
        }
    }
}

// Contribution of face f to r at (i, j) (dn = distance from the face along its
// normal, t = index along the face).  DATA selects the data part (time
// combination tc) instead of the homogeneous part acting on field `fld`.
template <typename T, int ORD, bool DATA>
__device__ __forceinline__ void face_sat(const PassArgs& A, int b, int f, int dn, int t, int fld, const W3& tc, T& r0, T& r1) {
    using O = Op<ORD>;
    BlockRef B = blk(A, b);
    const double beta = B.beta;
    const GLB FaceDesc& F = B.face[f];
    const int a = f >> 1;
    const long np = (long)B.n1 * B.n2;
    gcp<T> c = gc<T>(B.coef);
    const T nu = (f & 1) ? T(1) : T(-1);
    const double ha = a == 0 ? B.h1 : B.h2;
    const int na = a == 0 ? B.n1 : B.n2;
    const int nt = a == 0 ? B.n2 : B.n1;
    const double ht = a == 0 ? B.h2 : B.h1;
    const T iw = T(1.0 / F.w);
    // the data part of a face without data is zero
    if (DATA && !(F.kind == BC_DISPLACEMENT ? F.g != nullptr
                  : F.kind == BC_INTERFACE  ? (F.V != nullptr || F.Th != nullptr)
                                            : F.g != nullptr))
        return;

    if (F.kind == BC_TRACTION || F.kind == BC_ROBIN) {
        if (dn != 0) return;
        if (!DATA) {
            gcp<T> u = field_ptr<T>(A, b, fld);
            T tr0, tr1;
            traction_at<T, ORD>(B, u, f, t, tr0, tr1);
            r0 -= iw * tr0;
            r1 -= iw * tr1;
            if (F.kind == BC_ROBIN && F.U) {
                gcp<T> U = gc<T>(F.U);
                const FacePt q = face_point(B, f, t);
                const long p = (long)q.j * B.n1 + q.i;
                const T x0 = u[p], x1 = u[np + p];
                r0 -= U[t] * x0 + U[F.nf + t] * x1;
                r1 -= U[2 * F.nf + t] * x0 + U[3 * F.nf + t] * x1;
            }
        } else if (F.g) {
            const T tau = static_cast<T>(tval(B, A, F.item_g, tc));
            gcp<T> g = gc<T>(F.g);
            r0 += tau * g[t];
            r1 += tau * g[F.nf + t];
        }
        return;
    }
    // displacement or interface
    const bool itf = F.kind == BC_INTERFACE;
    const T half = itf ? T(0.5) : T(1);
    const FacePt q = face_point(B, f, t);
    const long pf = (long)q.j * B.n1 + q.i;
    T d0, d1;
    face_delta<T, DATA>(A, b, f, t, fld, tc, d0, d1);
    T N[2][2], M[2][2];
    coef_mats(c, np, pf, a, N, M);
    if (dn < O::REACH) {
        // normal part: nu_a D1[face row][dn] / H_a[dn] c_alaj delta_l
        const double hn = hnorm<ORD>(dn, na);
        const T cf = half * static_cast<T>(-O::d1b(0, dn) / (ha * ha * hn));
        r0 += cf * (N[0][0] * d0 + N[0][1] * d1);
        r1 += cf * (N[1][0] * d0 + N[1][1] * d1);
    }
    if (dn != 0) return;
    // tangential part: (1/w) (H_t^{-1} D_t^T H_t qv)(t), qv = nu c_altj delta_l
    {
        auto qv = [&](int tt, T& q0, T& q1) {
            T e0, e1;
            face_delta<T, DATA>(A, b, f, tt, fld, tc, e0, e1);
            const FacePt qq = face_point(B, f, tt);
            T Nq[2][2], Mq[2][2];
            coef_mats(c, np, (long)qq.j * B.n1 + qq.i, a, Nq, Mq);
            if (a == 0) {   // c_1l2j = M_lj
                q0 = nu * (Mq[0][0] * e0 + Mq[1][0] * e1);
                q1 = nu * (Mq[0][1] * e0 + Mq[1][1] * e1);
            } else {        // c_2l1j = c_1j2l = M_jl
                q0 = nu * (Mq[0][0] * e0 + Mq[0][1] * e1);
                q1 = nu * (Mq[1][0] * e0 + Mq[1][1] * e1);
            }
        };
        T qt0, qt1;
        qv(t, qt0, qt1);
        T dq0 = 0, dq1 = 0;
        d1_foreach<ORD>(t, nt, [&](int tt, double w) {
            T q0, q1;
            qv(tt, q0, q1);
            dq0 += static_cast<T>(w) * (q0 - qt0);
            dq1 += static_cast<T>(w) * (q1 - qt1);
        });
        const T iht = T(1.0 / ht);
        T s0v = -dq0 * iht, s1v = -dq1 * iht;
        if (t == 0) {
            const T ih0 = T(1.0 / (ht * hnorm<ORD>(0, nt)));
            s0v -= qt0 * ih0;
            s1v -= qt1 * ih0;
        }
        if (t == nt - 1) {
            const T ihN = T(1.0 / (ht * hnorm<ORD>(nt - 1, nt)));
            s0v += qt0 * ihN;
            s1v += qt1 * ihN;
        }
        r0 += half * iw * s0v;
        r1 += half * iw * s1v;
    }
    // penalty
    if (!itf) {
        const T pen = static_cast<T>(beta * 2.0) * iw * iw;
        r0 -= pen * (N[0][0] * d0 + N[0][1] * d1);
        r1 -= pen * (N[1][0] * d0 + N[1][1] * d1);
    } else {
        BlockRef P = blk(A, F.partner);
        const int tp = F.reversed ? F.nf - 1 - t : t;
        const FacePt qp = face_point(P, F.pface, tp);
        const long npp = (long)P.n1 * P.n2;
        T Np[2][2], Mp[2][2];
        coef_mats(gc<T>(P.coef), npp, (long)qp.j * P.n1 + qp.i, F.pface >> 1, Np, Mp);
        const T ipw = T(1.0 / F.pw);
        const T qf = static_cast<T>(beta * 2.0 * 0.25);
        T Z[2][2];
        for (int x = 0; x < 2; ++x)
            for (int y = 0; y < 2; ++y) Z[x][y] = qf * (N[x][y] * iw + Np[x][y] * ipw);
        r0 -= iw * (Z[0][0] * d0 + Z[0][1] * d1);
        r1 -= iw * (Z[1][0] * d0 + Z[1][1] * d1);
        // traction average
        if (!DATA) {
            T tu0, tu1, tv0, tv1;
            traction_at<T, ORD>(B, field_ptr<T>(A, b, fld), f, t, tu0, tu1);
            traction_at<T, ORD>(P, field_ptr<T>(A, F.partner, fld), F.pface, tp, tv0, tv1);
            r0 -= T(0.5) * iw * (tu0 + tv0);
            r1 -= T(0.5) * iw * (tu1 + tv1);
        } else if (F.Th) {
            const T tau = static_cast<T>(tval(B, A, F.item_v, tc));
            gcp<T> Th = gc<T>(F.Th);
            r0 += tau * Th[t];
            r1 += tau * Th[F.nf + t];
        }
    }
}

// SAT contributions of the faces FB .. FE - 1 at (i, j)
template <typename T, int ORD, bool DATA, int FB = 0, int FE = 4>
__device__ __forceinline__ void sat_point(const PassArgs& A, int b, int i, int j, int fld, const W3& tc, T& r0, T& r1) {
    using O = Op<ORD>;
    BlockRef B = blk(A, b);
    const int n1 = B.n1, n2 = B.n2;
    if (FB <= 0 && 0 < FE && i < O::REACH) face_sat<T, ORD, DATA>(A, b, 0, i, j, fld, tc, r0, r1);
    if (FB <= 1 && 1 < FE && n1 - 1 - i < O::REACH) face_sat<T, ORD, DATA>(A, b, 1, n1 - 1 - i, j, fld, tc, r0, r1);
    if (FB <= 2 && 2 < FE && j < O::REACH) face_sat<T, ORD, DATA>(A, b, 2, j, i, fld, tc, r0, r1);
    if (FB <= 3 && 3 < FE && n2 - 1 - j < O::REACH) face_sat<T, ORD, DATA>(A, b, 3, n2 - 1 - j, i, fld, tc, r0, r1);
}

// sources (and, in the frame, the forcing) at flat point p
template <typename T>
__device__ __forceinline__ void point_sources(BlockRef B, const PassArgs& A, const Range& rg, long p, const W3& tc, T& r0,
                                              T& r1) {
    entries_at(B, rg.beg, rg.mid, p, [&](const GLB Entry& E) {
        const double tau = tval(B, A, E.id, tc);
        r0 += static_cast<T>(E.c0 * tau);
        r1 += static_cast<T>(E.c1 * tau);
    });
}

template <typename T>
__device__ __forceinline__ void point_data(BlockRef B, long p, const PassArgs& A, const Range& rg, const W3& tc,
                                           T& r0, T& r1) {
    if (B.force) {
        gcp<T> F = gc<T>(B.force);
        const T tau = static_cast<T>(tval(B, A, B.item_f, tc));
        r0 += tau * F[p];
        r1 += tau * F[(long)B.n1 * B.n2 + p];
    }
    point_sources<T>(B, A, rg, p, tc, r0, r1);
}

__device__ __forceinline__ int find_block(const PassArgs& A, int wg, bool frame) {
    int b = 0;
    for (int k = 1; k < A.nblocks; ++k) {
        const int beg = frame ? blk(A, k).frame_beg : blk(A, k).tile_beg;
        if (wg >= beg) b = k;
    }
    return b;
}

// ---------------------------------------------------------------- frame
// A workgroup of four waves takes FRAME_PTS frame points.  Wave w evaluates
// term group w for every point (two lanes per point), so the long chains of
// closure-row loads are split over four waves:
//   wave 0: D_11^FC term and the homogeneous SATs of the x1 faces
//   wave 1: D_22^FC term and the homogeneous SATs of the x2 faces
//   wave 2: D_1 (c_1j2l D_2 u_l)
//   wave 3: D_2 (c_2j1l D_1 u_l), the data SATs, forcing and sources.
// In the RK sweeps lane s of a pair works on field s (u / v, or A1 / A2);
// for sbpe_apply lane 0 evaluates L and lane 1 of wave 3 the data.  The
// partial sums meet in LDS; wave 0 combines them and lane s of each pair
// writes component s of the outputs.
template <typename T, int ORD>
__global__ void __launch_bounds__(FRAME_WG) k_frame(PassArgs A) {
    constexpr int R = Frame<ORD>::R;
    __shared__ T s_r[4][64][4];
    const int wg = blockIdx.x;
    const int b = find_block(A, wg, true);
    BlockRef B = blk(A, b);
    const int part = threadIdx.x >> 6;   // wave-uniform term group
    const int lane = threadIdx.x & 63;
    const int sub = lane & 1;
    const int k = (wg - B.frame_beg) * FRAME_PTS + (lane >> 1);
    const Range rg = load_range(B.frame_rng, wg - B.frame_beg);
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const bool valid = k < B.frame_n;
    const int kk0 = valid ? k : 0;
    int i, j;
    frame_ij(kk0, n1, n2, R, i, j);
    const long p = (long)j * n1 + i;
    const W3 none{0.0, 0.0, 0.0};
    const W3 ca = weights_a(A), cb = weights_b(A, B);
    T l0 = 0, l1 = 0, d0 = 0, d1 = 0;
    if (valid) {
        const bool apply = A.pass == PASS_APPLY;
        const int fld = apply ? FLD_IN : (A.pass == PASS_RK1 ? (sub ? FLD_V : FLD_U) : (sub ? FLD_A2 : FLD_A1));
        const bool hom = !apply || sub == 0;    // this lane evaluates L of its field
        gcp<T> u = field_ptr<T>(A, b, fld);
        if (part == 0) {
            if (hom) {
                volume_part<T, ORD, 0>(B, u, i, j, l0, l1, A.wide != 0);
                sat_point<T, ORD, false, 0, 2>(A, b, i, j, fld, none, l0, l1);
            }
        } else if (part == 1) {
            if (hom) {
                volume_part<T, ORD, 1>(B, u, i, j, l0, l1, A.wide != 0);
                sat_point<T, ORD, false, 2, 4>(A, b, i, j, fld, none, l0, l1);
            }
        } else if (part == 2) {
            if (hom) volume_part<T, ORD, 2>(B, u, i, j, l0, l1, A.wide != 0);
        } else {
            if (hom) volume_part<T, ORD, 3>(B, u, i, j, l0, l1, A.wide != 0);
            // member-wise select (a runtime choice between two structs goes through scratch memory)
            const bool second = !apply && sub;
            const W3 cw{second ? cb.w0 : ca.w0, second ? cb.w1 : ca.w1, second ? cb.w2 : ca.w2};
            if ((!apply || sub == 1) && cw.any()) {
                sat_point<T, ORD, true>(A, b, i, j, fld, cw, d0, d1);
                point_data<T>(B, p, A, rg, cw, d0, d1);
            }
        }
    }
    s_r[part][lane][0] = l0;
    s_r[part][lane][1] = l1;
    s_r[part][lane][2] = d0;
    s_r[part][lane][3] = d1;
    __syncthreads();
    if (part != 0) return;
#pragma unroll
    for (int w = 1; w < 4; ++w) {
        l0 += s_r[w][lane][0];
        l1 += s_r[w][lane][1];
        d0 += s_r[w][lane][2];
        d1 += s_r[w][lane][3];
    }
    // exchange with the partner lane
    const T ol0 = __shfl_xor(l0, 1), ol1 = __shfl_xor(l1, 1);
    const T od0 = __shfl_xor(d0, 1), od1 = __shfl_xor(d1, 1);
    if (!valid) return;
    const T irho = gc<T>(B.coef)[(long)K_IRHO * np + p];
    const long q = (long)sub * np + p;   // component written by this lane
    if (A.pass == PASS_APPLY) {
        // lane 0 holds L, lane 1 the data
        const T L = sub ? ol1 : l0;
        const T D = sub ? d1 : od0;
        gm<T>(apply_out(A, b))[q] = irho * (L + D);
        return;
    }
    // field 0 (lane 0) and field 1 (lane 1) results, component sub
    const T La = sub ? ol1 : l0;     // L f0, component sub
    const T Lb = sub ? l1 : ol0;     // L f1, component sub
    const T Da = sub ? od1 : d0;
    const T Db = sub ? d1 : od0;
    const T dt = static_cast<T>(B.dt);
    if (A.pass == PASS_RK1) {
        gm<T>(B.a1)[q] = irho * (La + Da);
        gm<T>(B.a2)[q] = irho * (La + T(0.5) * dt * Lb + Db);
        return;
    }
    const T A1 = gc<T>(B.a1)[q], A2 = gc<T>(B.a2)[q];
    gp<T> uu = gm<T>(B.u);
    gp<T> vv = gm<T>(B.v);
    const T dt2 = dt * dt;
    const T A3 = A2 + T(0.25) * dt2 * irho * La;
    const T A4 = T(2) * A2 - A1 + T(0.5) * dt2 * irho * (Lb + Db);
    const T uo = uu[q], vo = vv[q];
    const T un = uo + dt * vo + dt2 / T(6) * (A1 + A2 + A3);
    uu[q] = un;
    vv[q] = vo + dt / T(6) * (A1 + T(2) * A2 + T(2) * A3 + A4);
    if (gp<double> ro = rec_slots(B, A))
        entries_at(B, rg.mid, rg.end, p,
                   [&](const GLB Entry& E) { ro[2 * E.id + sub] = E.c0 * static_cast<double>(un); });
}

// ------------------------------------------------- assembled frame operator
// The frame rows of rho~^{-1} L are assembled once at setup by probing
// k_frame with coloured unit vectors (colour (i mod 9, j mod 9): no stencil of
// a frame row spans 9 points in either direction) and applied by k_frame_sp
// in difference form,
//   (rho~^{-1} L x)_{k,q} = sum_(p',q') K (x_q'(p') - x_q'(p_k)) + sum_q' S_q' x_q'(p_k),
// with the row sums S from probes with constant fields, so that FP32 sums of
// the O(1/h^2) entries cancel like the stencil kernels' differences.
template <typename T>
__global__ void __launch_bounds__(256) k_probe_fill(T* x, int n1, int n2, int comp, int cx, int cy, int period) {
    const long np = (long)n1 * n2;
    const long idx = (long)blockIdx.x * 256 + threadIdx.x;
    if (idx >= 2 * np) return;
    const int q = (int)(idx / np);
    const long p = idx - q * np;
    const int j = (int)(p / n1), i = (int)(p - (long)j * n1);
    bool one = q == comp;
    if (one && period > 0) one = (i % period) == cx && (j % period) == cy;
    ((gp<T>)x)[idx] = one ? T(1) : T(0);
}

template <typename T>
__global__ void __launch_bounds__(256) k_frame_gather(const T* y, int n1, int n2, int R, int frame_n, T* out) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= frame_n) return;
    int i, j;
    frame_ij(k, n1, n2, R, i, j);
    const long np = (long)n1 * n2;
    const long p = (long)j * n1 + i;
    ((gp<T>)out)[2 * k] = ((gcp<T>)y)[p];
    ((gp<T>)out)[2 * k + 1] = ((gcp<T>)y)[np + p];
}

// FRAME_LANES lanes per frame point.  Frame points are numbered globally in
// groups of FRAME_PTS per block (the k_frame workgroup layout, so the
// point-entry ranges carry over); a workgroup of nt threads takes points
// fwg * nt / FRAME_LANES .. (fwg + 1) * nt / FRAME_LANES - 1.  The operator
// is stored in 2x2 blocks, one per neighbouring point: every lane takes a
// share of the point's blocks for both component rows (one column index and
// one gather of each input component per block), the lanes' sums meet by
// shuffles, and lanes 0 .. FRAME_LANES/2 - 1 go on with the first component
// row, the others with the second.  Every load that does not depend on the
// point's blocks is issued first, and the blocks are gathered FRAME_UNROLL
// per lane at a time (all column and weight loads, then all gathers).
constexpr int FRAME_LANES = 8;
constexpr int FRAME_UNROLL = 4;

// ROW_BRANCH: pick the lane's component row by a branch (inside the one-launch
// sweep kernels, where a select on it is lowered to a run-time index into
// scratch memory) or by a select (the stand-alone frame kernel, where the
// branch costs registers: 172 against 160 in the FP64 RK2 kernel, two waves
// per SIMD instead of three).
template <typename T, int ORD, int PASS, bool ROW_BRANCH = true>
__device__ __forceinline__ void frame_sp_body(const PassArgs& A, int fwg, int nt) {
    constexpr int R = Frame<ORD>::R;
    constexpr int RL = FRAME_LANES / 2;        // lanes per component row
    constexpr int U = FRAME_UNROLL;
    const int g = fwg * (nt / FRAME_LANES) + (int)(threadIdx.x / FRAME_LANES);
    const int wg = g / FRAME_PTS;
    if (wg >= A.total_frame_wg) return;        // whole point groups leave together
    const int b = find_block(A, wg, true);
    BlockRef B = blk(A, b);
    const int lane = threadIdx.x & (FRAME_LANES - 1);   // lane within the point
    const int q = lane / RL;                   // component row
    const int sl = lane & (RL - 1);            // lane within the row
    const int k = (wg - B.frame_beg) * FRAME_PTS + g % FRAME_PTS;
    const Range rg = load_range(B.frame_rng, wg - B.frame_beg);
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const bool valid = k < B.frame_n;
    int i, j;
    frame_ij(valid ? k : 0, n1, n2, R, i, j);
    const long p = (long)j * n1 + i;
    constexpr bool apply = PASS == PASS_APPLY;
    constexpr int NF = apply ? 1 : 2;
    // input fields of the sweep (own block) and their values at the point
    gcp<T> xf[NF];
    if constexpr (apply) {
        xf[0] = gc<T>(apply_in(A, b));
    } else if constexpr (PASS == PASS_RK1) {
        xf[0] = gc<T>(B.u);
        xf[1] = gc<T>(B.v);
    } else {
        xf[0] = gc<T>(B.a1);
        xf[1] = gc<T>(B.a2);
    }
    T xp[NF][2];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        xp[f][0] = xf[f][p];
        xp[f][1] = xf[f][np + p];
    }
    // per-point operands of the pass arithmetic, issued before the row
    const long qp = (long)q * np + p;
    const T irho = gc<T>(B.coef)[(long)K_IRHO * np + p];
    gcp<T> rs = gc<T>(B.fr_rsum);
    const long ridx = valid ? 2 * (2 * (long)k + q) : 0;
    const T s0 = rs[ridx], s1 = rs[ridx + 1];
    T A1 = 0, A2 = 0, uo = 0, vo = 0;
    if constexpr (PASS == PASS_RK2) {
        A1 = gc<T>(B.a1)[qp];
        A2 = gc<T>(B.a2)[qp];
        uo = gc<T>(B.u)[qp];
        vo = gc<T>(B.v)[qp];
    }
    // both component rows of the point, summed over this lane's blocks
    T ab[NF][2];
#pragma unroll
    for (int f = 0; f < NF; ++f) ab[f][0] = ab[f][1] = T(0);
    if (valid) {
        const GLB int* bp = (const GLB int*)B.fr_rowptr;
        const GLB int* cl = (const GLB int*)B.fr_col;
        gcp<T> vl = gc<T>(B.fr_val);
        const int e0 = bp[k], e1 = bp[k + 1];
        bool partner = false;
        for (int e = e0 + lane; e < e1; e += FRAME_LANES * U) {
            int cc[U];
            T ww[U][4];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int ee = e + FRAME_LANES * u;
                const int ec = ee < e1 ? ee : e0;          // e0 < e1 here: a valid block
                cc[u] = cl[ec];
#pragma unroll
                for (int r = 0; r < 4; ++r) ww[u][r] = vl[4 * (long)ec + r];
            }
            T xv[U][NF][2];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const bool in = e + FRAME_LANES * u < e1;
                const int c = cc[u];
                partner |= in && c < 0;
                if (!(in && c >= 0))
#pragma unroll
                    for (int r = 0; r < 4; ++r) ww[u][r] = T(0);
                const long ix = c >= 0 ? (long)c : p;
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    xv[u][f][0] = xf[f][ix];
                    xv[u][f][1] = xf[f][np + ix];
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T d0 = xv[u][f][0] - xp[f][0], d1 = xv[u][f][1] - xp[f][1];
                    ab[f][0] += ww[u][0] * d0 + ww[u][1] * d1;
                    ab[f][1] += ww[u][2] * d0 + ww[u][3] * d1;
                }
        }
        if (partner) {
            // blocks of a partner block's point across an interface
            for (int e = e0 + lane; e < e1; e += FRAME_LANES) {
                const int c = cl[e];
                if (c >= 0) continue;
                T w[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) w[r] = vl[4 * (long)e + r];
                const int v = -1 - c;
                const int ff = v >> 29;
                const long pp = v & ((1 << 28) - 1);
                const GLB FaceDesc& F = B.face[ff];
                const int pb = F.partner;
                BlockRef P = blk(A, pb);
                const long npp = (long)P.n1 * P.n2;
                gcp<T> pf[NF];
                if constexpr (apply) {
                    pf[0] = gc<T>(apply_in(A, pb));
                } else if constexpr (PASS == PASS_RK1) {
                    pf[0] = gc<T>(P.u);
                    pf[1] = gc<T>(P.v);
                } else {
                    pf[0] = gc<T>(P.a1);
                    pf[1] = gc<T>(P.a2);
                }
#pragma unroll
                for (int f = 0; f < NF; ++f) {
                    const T d0 = pf[f][pp] - xp[f][0], d1 = pf[f][npp + pp] - xp[f][1];
                    ab[f][0] += w[0] * d0 + w[1] * d1;
                    ab[f][1] += w[2] * d0 + w[3] * d1;
                }
            }
        }
    }
    // reduce the lanes of the point; each lane keeps its component row
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 1; m < FRAME_LANES; m <<= 1) {
            ab[f][0] += __shfl_xor(ab[f][0], m);
            ab[f][1] += __shfl_xor(ab[f][1], m);
        }
    T acc[NF];
    if constexpr (ROW_BRANCH) {
        if (q) {
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] = ab[f][1];
        } else {
#pragma unroll
            for (int f = 0; f < NF; ++f) acc[f] = ab[f][0];
        }
    } else {
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] = q ? ab[f][1] : ab[f][0];
    }
    if (valid) {
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f] += s0 * xp[f][0] + s1 * xp[f][1];
    }
    // data: lane 0 of the point with the first weights, lane RL with the second
    const W3 ca = weights_a(A), cb = weights_b(A, B);
    T d0 = 0, d1 = 0;
    if (valid && (lane == 0 || (lane == RL && !apply))) {
        const W3 cw{lane ? cb.w0 : ca.w0, lane ? cb.w1 : ca.w1, lane ? cb.w2 : ca.w2};
        if (cw.any()) {
            const int fld = apply ? FLD_IN : (PASS == PASS_RK1 ? FLD_U : FLD_A1);
            sat_point<T, ORD, true>(A, b, i, j, fld, cw, d0, d1);
            point_data<T>(B, p, A, rg, cw, d0, d1);
        }
    }
    // broadcast the data of lanes 0 and RL to the point's lanes
    const int base = threadIdx.x & ~(FRAME_LANES - 1);
    const T da0 = __shfl(d0, base), da1 = __shfl(d1, base);
    const T db0 = __shfl(d0, base + RL), db1 = __shfl(d1, base + RL);
    // the other component row's rho~^-1 L of the first field
    const T acc0o = __shfl(acc[0], base + RL * (1 - q));
    if (!valid || sl != 0) return;
    const T da = q ? da1 : da0, db = q ? db1 : db0;
    if constexpr (apply) {
        gm<T>(apply_out(A, b))[qp] = acc[0] + irho * da;
        return;
    }
    // Dissipative Robin terms V u_t (the remark after eq. sat_traction): at a
    // face point a = rho~^-1 (L u - S v + d) with S = sum over its faces of
    // Jhat V / w, so the stage velocities enter pointwise:
    //   A1 -= rho~^-1 S v,  A2 -= rho~^-1 S (v + dt/2 A1),
    //   A3 -= rho~^-1 dt/2 S (A2 - A1),  A4 += rho~^-1 dt S (A1 - A3).
    T Dm[2][2] = {{T(0), T(0)}, {T(0), T(0)}};
    bool dis = false;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const GLB FaceDesc& F = B.face[f];
        const bool on = f == 0 ? i == 0 : f == 1 ? i == n1 - 1 : f == 2 ? j == 0 : j == n2 - 1;
        if (on && F.Dv) {
            gcp<T> dv = gc<T>(F.Dv);
            const int t = f < 2 ? j : i, nf = F.nf;
            Dm[0][0] += dv[t];
            Dm[0][1] += dv[nf + t];
            Dm[1][0] += dv[2 * nf + t];
            Dm[1][1] += dv[3 * nf + t];
            dis = true;
        }
    }
    auto smul = [&](int c, T x0, T x1) { return c ? Dm[1][0] * x0 + Dm[1][1] * x1 : Dm[0][0] * x0 + Dm[0][1] * x1; };
    const T dt = static_cast<T>(B.dt);
    if constexpr (PASS == PASS_RK1) {
        T a1 = acc[0] + irho * da;
        T a2 = acc[0] + T(0.5) * dt * acc[NF - 1] + irho * db;
        if (dis) {
            const T v0 = xp[1][0], v1 = xp[1][1];
            const T dao = q ? da0 : da1;
            a1 -= irho * smul(q, v0, v1);
            const T a1o = acc0o + irho * (dao - smul(1 - q, v0, v1));
            const T w0 = v0 + T(0.5) * dt * (q ? a1o : a1), w1 = v1 + T(0.5) * dt * (q ? a1 : a1o);
            a2 -= irho * smul(q, w0, w1);
        }
        gm<T>(B.a1)[qp] = a1;
        gm<T>(B.a2)[qp] = a2;
        return;
    }
    gp<T> uu = gm<T>(B.u);
    gp<T> vv = gm<T>(B.v);
    const T dt2 = dt * dt;
    T A3 = A2 + T(0.25) * dt2 * acc[0];
    T A4 = T(2) * A2 - A1 + T(0.5) * dt2 * (acc[NF - 1] + irho * db);
    if (dis) {
        const long qo = (long)(1 - q) * np + p;
        const T A1o = gc<T>(B.a1)[qo], A2o = gc<T>(B.a2)[qo];
        const T e0 = q ? A2o - A1o : A2 - A1, e1 = q ? A2 - A1 : A2o - A1o;
        const T hdt = T(0.5) * dt;
        A3 -= irho * hdt * smul(q, e0, e1);
        const T A3o = A2o + T(0.25) * dt2 * acc0o - irho * hdt * smul(1 - q, e0, e1);
        const T g0 = q ? A1o - A3o : A1 - A3, g1 = q ? A1 - A3 : A1o - A3o;
        A4 += irho * dt * smul(q, g0, g1);
    }
    const T un = uo + dt * vo + dt2 / T(6) * (A1 + A2 + A3);
    uu[qp] = un;
    vv[qp] = vo + dt / T(6) * (A1 + T(2) * A2 + T(2) * A3 + A4);
    if (gp<double> ro = rec_slots(B, A))
        entries_at(B, rg.mid, rg.end, p,
                   [&](const GLB Entry& E) { ro[2 * E.id + q] = E.c0 * static_cast<double>(un); });
}

template <typename T, int ORD, int PASS>
__global__ void __launch_bounds__(FRAME_WG) k_frame_sp(PassArgs A) {
    frame_sp_body<T, ORD, PASS, false>(A, blockIdx.x, FRAME_WG);
}

// ------------------------------------------------------------- interior
// Marching kernel: one wave covers the 64 columns i0 .. i0+63 and writes the
// OUTW = 64 - 2H central ones (H = half width of the interior stencils), so
// every x1 neighbour a lane needs is another lane's column and no halo
// column is loaded.  The wave marches over the rows jb .. je of its tile;
// for output row j it
//   * stages the input fields of the leading row j+H in an LDS ring of 2H+1
//     rows (x1 neighbours for the staged row, x2 window of the own column),
//   * forms E(j+H) = M^T D_1 w (M_jl = c_1j2l) into a register window,
//   * forms G(j) = M D_2 w at all 64 columns into an LDS row, then D_1 G,
//   * evaluates the narrow x1 term from the staged row j and the x1
//     coefficient row, the narrow x2 term from the ring and the register
//     window of the x2 coefficients, and D_2 E from the E window,
//   * applies the pass arithmetic (sbpe_internal.h) and stores row j.
// The row loop is unrolled by 2H+1, so every ring slot and register window
// position is a compile-time constant (no window shifting).  The global
// loads of the next row are issued before the arithmetic of the current one
// into a buffer that is consumed at the start of the next row.
template <typename T>
__device__ __forceinline__ T ldo(const char* base, unsigned off) {
    return *(const GLB T*)((const GLB char*)base + off);
}
template <typename T>
__device__ __forceinline__ void sto(char* base, unsigned off, T v) {
    *(GLB T*)((GLB char*)base + off) = v;
}

// Orders the LDS accesses of one wave (the other lanes' writes before the
// reads that follow) without a workgroup barrier: LDS operations of a wave
// complete in issue order, so only compiler reordering has to be prevented.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int NS, int NX>
struct Lead {
    T w[NS];   // input fields at (i, j + H)
    T b2[3];   // x2-narrow coefficients at (i, j + H)
    T m[4];    // mixed coefficients at (i, j + H)
    T b1[3];   // x1-narrow coefficients at (i, j)
    T pt[3];   // 1/rho~ and the two forcing components at (i, j)
    T xo[NX > 0 ? NX : 1];   // RK2: the state read back at (i, j)
};

// SPLIT (RK sweeps): a workgroup of two waves shares the tile; wave w applies
// L to field w only, which halves the registers of a wave, and the two meet
// in LDS for the pass arithmetic (RK1: wave w writes a_{w+1}; RK2: wave q
// writes component q of u and v).
template <typename T, int ORD, int PASS, bool SPLIT>
__device__ __forceinline__ void march_body(const PassArgs& A, int bid) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    constexpr int NW = 2 * HF + 1;
    constexpr int NF = (PASS == PASS_APPLY || SPLIT) ? 1 : 2;
    constexpr int NS = 2 * NF;
    constexpr int NX = PASS == PASS_RK2 ? (SPLIT ? 2 : 4) : 0;   // state words read back per point
    constexpr int NWAVE = SPLIT ? 2 : 1;
    constexpr int R = Frame<ORD>::R;
    __shared__ T s_xw[NWAVE][NW][NS][64];
    __shared__ T s_bw[NWAVE][3][64];
    __shared__ T s_gw[NWAVE][NS][64];
    __shared__ T s_lb[SPLIT ? 2 : 1][SPLIT ? 2 : 1][4][64];   // exchange (by row parity): L and centre values
    const int wv = SPLIT ? (int)(threadIdx.x >> 6) : 0;
    T(&s_x)[NW][NS][64] = s_xw[wv];
    T(&s_b)[3][64] = s_bw[wv];
    T(&s_g)[NS][64] = s_gw[wv];

    // workgroup order: consecutive tiles on the same XCD (ids are dealt round-robin to 8 XCDs)
    const int total = A.total_tiles;
    const int per = (total + 7) / 8;
    const int wg = (bid % 8) * per + bid / 8;
    if (wg >= total) return;
    const int b = find_block(A, wg, false);
    BlockRef B = blk(A, b);
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const int tl = wg - B.tile_beg;
    const int ty = tl / B.tiles_x, tx = tl - ty * B.tiles_x;
    const int lane = threadIdx.x & 63;
    const int i = R - HF + tx * (64 - 2 * HF) + lane;
    const bool act = lane >= HF && lane < 64 - HF && i <= n1 - 1 - R;
    const int ic = i < n1 - 1 ? i : n1 - 1;
    const int jb = R + ty * B.tile_y;
    const int je = (jb + B.tile_y < n2 - R ? jb + B.tile_y : n2 - R) - 1;
    // Every field is addressed as a uniform base plus a 32-bit per-lane byte
    // offset (one field of a block is below 4 GiB, checked on the host), so
    // the loads use scalar base registers and a single offset register.
    const unsigned fb = (unsigned)np * (unsigned)sizeof(T);    // bytes of one scalar field
    const unsigned rowb = (unsigned)n1 * (unsigned)sizeof(T);  // bytes of one grid row
    const unsigned lo = (unsigned)ic * (unsigned)sizeof(T);
    const char* cbase = (const char*)B.coef;
    auto cf = [&](int k) { return cbase + (size_t)k * fb; };
    const char* fin[NS];
    {
        const void* f0p = PASS == PASS_APPLY ? apply_in(A, b) : (PASS == PASS_RK1 ? B.u : B.a1);
        const void* f1p = PASS == PASS_RK1 ? B.v : B.a2;
        if (SPLIT && wv == 1) f0p = f1p;
#pragma unroll
        for (int s = 0; s < NS; ++s) fin[s] = (const char*)(s < 2 ? f0p : f1p) + (s & 1) * (size_t)fb;
    }
    // without forcing, the forcing loads read the 1/rho~ field (cached) and
    // are multiplied by zero, so that every load of a row is unconditional
    const bool force = B.force != nullptr;
    const char* frc = force ? (const char*)B.force : cbase + (size_t)K_IRHO * fb;
    const unsigned frc1 = force ? fb : 0u;
    const Range rg = load_range(B.tile_rng, wg - B.tile_beg);
    const W3 ca = weights_a(A), cb = weights_b(A, B);
    T tauf_a = 0, tauf_b = 0;
    if (force) {
        tauf_a = static_cast<T>(tval(B, A, B.item_f, ca));
        tauf_b = static_cast<T>(tval(B, A, B.item_f, cb));
    }
    // Point sources and receivers of the tile, staged once per workgroup (a
    // source with its amplitudes times the time functions of both weight
    // sets, a receiver with its interpolation weight), so that the per-row
    // matching reads LDS instead of a chain of dependent global loads.  A
    // tile with more entries than fit keeps the global loop.
    constexpr int MAXE = 32;
    __shared__ int s_ep[MAXE];
    __shared__ int s_eid[MAXE];        // receiver slot, or -1 for a source
    __shared__ double s_ev[MAXE][4];
    const int ne = rg.end - rg.beg;
    const int ns = rg.mid - rg.beg;      // sources first, then receivers
    const bool staged = ne <= MAXE;
    if (ne > 0 && staged) {
        for (int k = threadIdx.x; k < ne; k += NWAVE * 64) {
            const GLB Entry& E = entry(B, rg.beg + k);
            s_ep[k] = E.p;
            if (E.kind == 0) {
                const double ta = tval(B, A, E.id, ca), tb = tval(B, A, E.id, cb);
                s_eid[k] = -1;
                s_ev[k][0] = E.c0 * ta;
                s_ev[k][1] = E.c1 * ta;
                s_ev[k][2] = E.c0 * tb;
                s_ev[k][3] = E.c1 * tb;
            } else {
                s_eid[k] = E.id;
                s_ev[k][0] = E.c0;
            }
        }
        __syncthreads();
    }
    // Both staged runs are sorted by point, so the sources of row j are
    // [s_lo, s_hi) and its receivers [r_lo, r_hi), found by cursors that only
    // move forward.
    int s_lo = 0, s_hi = 0, r_lo = ns, r_hi = ns;
    auto entry_rows = [&](int j) {
        if (ne == 0 || !staged) return;
        const long rs = (long)j * n1, re = rs + n1;
        while (s_lo < ns && (long)s_ep[s_lo] < rs) ++s_lo;
        s_hi = s_lo;
        while (s_hi < ns && (long)s_ep[s_hi] < re) ++s_hi;
        while (r_lo < ne && (long)s_ep[r_lo] < rs) ++r_lo;
        r_hi = r_lo;
        while (r_hi < ne && (long)s_ep[r_hi] < re) ++r_hi;
    };
    // add the sources at point po with the first (ca) or second (cb) weights
    auto sources = [&](long po, bool second, T& r0, T& r1) {
        if (staged) {
            const int o = second ? 2 : 0;
            for (int k = s_lo; k < s_hi; ++k)
                if ((long)s_ep[k] == po) {
                    r0 += static_cast<T>(s_ev[k][o]);
                    r1 += static_cast<T>(s_ev[k][o + 1]);
                }
        } else {
            point_sources<T>(B, A, rg, po, second ? cb : ca, r0, r1);
        }
    };
    // receiver slots of point po, component q
    auto record = [&](gp<double> ro, long po, int q, double un) {
        if (staged) {
            for (int k = r_lo; k < r_hi; ++k)
                if ((long)s_ep[k] == po) ro[2 * s_eid[k] + q] = s_ev[k][0] * un;
        } else {
            entries_at(B, rg.mid, rg.end, po, [&](const GLB Entry& E) { ro[2 * E.id + q] = E.c0 * un; });
        }
    };
    const T ih1 = T(1.0 / B.h1), ih2 = T(1.0 / B.h2);
    const T i11 = ih1 * ih1, i22 = ih2 * ih2, i12 = ih1 * ih2;
    const T dt = static_cast<T>(B.dt);

    // loads for output row j: the leading row j + H of the windows and the
    // per-point operands of row j, issued one row ahead of their use
    auto load_lead = [&](int j, Lead<T, NS, NX>& L) {
        const int jj = j < je ? j : je;
        const unsigned qn = (unsigned)(jj + HF) * rowb + lo;
        const unsigned qj = (unsigned)jj * rowb + lo;
#pragma unroll
        for (int s = 0; s < NS; ++s) L.w[s] = ldo<T>(fin[s], qn);
        L.b2[0] = ldo<T>(cf(K_C2121), qn);
        L.b2[1] = ldo<T>(cf(K_C2122), qn);
        L.b2[2] = ldo<T>(cf(K_C2222), qn);
        L.m[0] = ldo<T>(cf(K_C1121), qn);
        L.m[1] = ldo<T>(cf(K_C1122), qn);
        L.m[2] = ldo<T>(cf(K_C1221), qn);
        L.m[3] = ldo<T>(cf(K_C1222), qn);
        L.b1[0] = ldo<T>(cf(K_C1111), qj);
        L.b1[1] = ldo<T>(cf(K_C1112), qj);
        L.b1[2] = ldo<T>(cf(K_C1212), qj);
        L.pt[0] = ldo<T>(cf(K_IRHO), qj);
        L.pt[1] = ldo<T>(frc, qj);
        L.pt[2] = ldo<T>(frc + frc1, qj);
        if constexpr (PASS == PASS_RK2 && SPLIT) {
            L.xo[0] = ldo<T>((const char*)B.u + wv * fb, qj);
            L.xo[1] = ldo<T>((const char*)B.v + wv * fb, qj);
        } else if constexpr (PASS == PASS_RK2) {
            L.xo[0] = ldo<T>((const char*)B.u, qj);
            L.xo[1] = ldo<T>((const char*)B.u + fb, qj);
            L.xo[2] = ldo<T>((const char*)B.v, qj);
            L.xo[3] = ldo<T>((const char*)B.v + fb, qj);
        }
    };

    // register windows indexed by ring slot: slot(r) = (r - jb + HF) mod NW
    T b2w[3][NW];     // x2-narrow coefficients
    T mw[4][NW];      // mixed coefficients
    T ew[NS][NW];     // E = M^T D_1 w

    // E at a staged row (slot s), from the x1 neighbours in the ring
    auto e_row = [&](const int s) {
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            T w1[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int x = 2 * f + q;
                w1[q] = d1_sym<ORD, T>([&](int o) {
                    const int l = lane + o;
                    return s_x[s][x][l < 0 ? 0 : (l > 63 ? 63 : l)];
                });
            }
            ew[2 * f][s] = mw[0][s] * w1[0] + mw[2][s] * w1[1];
            ew[2 * f + 1][s] = mw[1][s] * w1[0] + mw[3][s] * w1[1];
        }
    };

    // prologue: rows jb-HF .. jb+HF-1 staged, their E formed
    {
#pragma unroll
        for (int r = 0; r < 2 * HF; ++r) {
            const unsigned q = (unsigned)(jb - HF + r) * rowb + lo;
#pragma unroll
            for (int s = 0; s < NS; ++s) s_x[r][s][lane] = ldo<T>(fin[s], q);
            b2w[0][r] = ldo<T>(cf(K_C2121), q);
            b2w[1][r] = ldo<T>(cf(K_C2122), q);
            b2w[2][r] = ldo<T>(cf(K_C2222), q);
            mw[0][r] = ldo<T>(cf(K_C1121), q);
            mw[1][r] = ldo<T>(cf(K_C1122), q);
            mw[2][r] = ldo<T>(cf(K_C1221), q);
            mw[3][r] = ldo<T>(cf(K_C1222), q);
        }
        wave_sync();
#pragma unroll
        for (int r = 0; r < 2 * HF; ++r) e_row(r);
    }

    Lead<T, NS, NX> P;
    load_lead(jb, P);

    // one output row; K is the position in the unrolled group (slot of row j is K + HF)
    auto step = [&](auto KC, const int j) {
        constexpr int K = decltype(KC)::value;
        constexpr int s0 = (K + HF) % NW;        // row j
        constexpr int sn = (K + 2 * HF) % NW;    // leading row j + HF
        // (1) consume the leading-row buffer
#pragma unroll
        for (int s = 0; s < NS; ++s) s_x[sn][s][lane] = P.w[s];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s_b[k][lane] = P.b1[k];
            b2w[k][sn] = P.b2[k];
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) mw[m][sn] = P.m[m];
        const T b1c[3] = {P.b1[0], P.b1[1], P.b1[2]};
        // (2) per-point operands of row j, then the loads for row j + 1
        const bool live = j <= je;
        if (live) entry_rows(j);
        const unsigned p = (unsigned)(live ? j : je) * rowb + lo;
        const T irho = P.pt[0], f0 = P.pt[1], f1 = P.pt[2];
        T xo[4];
        if constexpr (PASS == PASS_RK2 && SPLIT) {
            xo[0] = P.xo[0];
            xo[2] = P.xo[1];
        } else if constexpr (PASS == PASS_RK2) {
#pragma unroll
            for (int k = 0; k < 4; ++k) xo[k] = P.xo[k];
        }
        load_lead(j + 1, P);
        wave_sync();
        // (3) E at the leading row
        e_row(sn);
        // (4) G at row j (all 64 columns) and the narrow x2 term, then the
        // narrow x1 term; each direction forms its edge weights once for
        // both fields, which keeps few values live at a time
        T lx[NF][2];
        T wc[NS];
        {
            T ky[3][2 * HF];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                T bb[NW];
#pragma unroll
                for (int k = 0; k < NW; ++k) bb[k] = b2w[m][(K + k) % NW];
                d2_weights<T, ORD>(bb, ky[m]);
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                T wcol[2][NW];
#pragma unroll
                for (int q = 0; q < 2; ++q)
#pragma unroll
                    for (int k = 0; k < NW; ++k) wcol[q][k] = s_x[(K + k) % NW][2 * f + q][lane];
                T w2[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    w2[q] = d1_sym<ORD, T>([&](int o) { return wcol[q][HF + o]; });
                    wc[2 * f + q] = wcol[q][HF];
                }
                s_g[2 * f][lane] = mw[0][s0] * w2[0] + mw[1][s0] * w2[1];
                s_g[2 * f + 1][lane] = mw[2][s0] * w2[0] + mw[3][s0] * w2[1];
                const T by0 = d2_edges<T, ORD>(ky[0], wcol[0]);   // c2121 u1
                const T by1 = d2_edges<T, ORD>(ky[1], wcol[1]);   // c2122 u2
                const T by2 = d2_edges<T, ORD>(ky[1], wcol[0]);   // c2122 u1
                const T by3 = d2_edges<T, ORD>(ky[2], wcol[1]);   // c2222 u2
                lx[f][0] = (by0 + by1) * i22;
                lx[f][1] = (by2 + by3) * i22;
            }
        }
        {
            T kx[3][2 * HF];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                T bb[NW];
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    const int l = lane + k - HF;
                    bb[k] = k == HF ? b1c[m] : s_b[m][l < 0 ? 0 : (l > 63 ? 63 : l)];
                }
                d2_weights<T, ORD>(bb, kx[m]);
            }
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                T ur[2][NW];
#pragma unroll
                for (int k = 0; k < NW; ++k) {
                    const int l = lane + k - HF;
                    const int lc = l < 0 ? 0 : (l > 63 ? 63 : l);
#pragma unroll
                    for (int q = 0; q < 2; ++q) ur[q][k] = k == HF ? wc[2 * f + q] : s_x[s0][2 * f + q][lc];
                }
                const T ax0 = d2_edges<T, ORD>(kx[0], ur[0]);   // c1111 u1
                const T ax1 = d2_edges<T, ORD>(kx[1], ur[1]);   // c1112 u2
                const T ax2 = d2_edges<T, ORD>(kx[1], ur[0]);   // c1112 u1
                const T ax3 = d2_edges<T, ORD>(kx[2], ur[1]);   // c1212 u2
                lx[f][0] += (ax0 + ax1) * i11;
                lx[f][1] += (ax2 + ax3) * i11;
            }
        }
        wave_sync();
        // (5) D_1 G and D_2 E
        T L[NF][2];
#pragma unroll
        for (int x = 0; x < NS; ++x) {
            const T ag = d1_sym<ORD, T>([&](int o) {
                const int l = lane + o;
                return s_g[x][l < 0 ? 0 : (l > 63 ? 63 : l)];
            });
            const T ae = d1_sym<ORD, T>([&](int o) { return ew[x][(K + HF + o) % NW]; });
            L[x >> 1][x & 1] = lx[x >> 1][x & 1] + (ag + ae) * i12;
        }
        // (6) data, pass arithmetic, stores
        if constexpr (SPLIT) {
            // exchange L and the centre values of both fields; the buffer
            // alternates with the row, so the next row's writes never meet
            // this row's reads and one barrier per row suffices
            T(&s_l)[2][4][64] = s_lb[j & 1];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                s_l[wv][q][lane] = L[0][q];
                s_l[wv][2 + q][lane] = wc[q];
            }
            __syncthreads();
            if (act && live) {
                const long po = (long)j * n1 + i;
                if constexpr (PASS == PASS_RK1) {
                    // wave 0: a1 = irho (L u + d(t)); wave 1: a2 = irho (L u + dt/2 L v + d(t + dt/2))
                    const W3 cw{wv ? cb.w0 : ca.w0, wv ? cb.w1 : ca.w1, wv ? cb.w2 : ca.w2};
                    const T tf = wv ? tauf_b : tauf_a;
                    T d0 = tf * f0, d1v = tf * f1;
                    if (ne > 0 && cw.any()) sources(po, wv != 0, d0, d1v);
                    const T hdt = wv ? T(0.5) * dt : T(0);
                    char* o = (char*)(wv ? B.a2 : B.a1);
                    sto<T>(o, p, irho * (s_l[0][0][lane] + hdt * L[0][0] + d0));
                    sto<T>(o + fb, p, irho * (s_l[0][1][lane] + hdt * L[0][1] + d1v));
                } else {
                    // component q = wv of the RK4 update
                    const int q = wv;
                    T db0 = tauf_b * f0, db1 = tauf_b * f1;
                    if (ne > 0 && cb.any()) sources(po, true, db0, db1);
                    const T dt2 = dt * dt;
                    const T q4 = T(0.25) * dt2, q2 = T(0.5) * dt2, s6 = dt2 / T(6), d6 = dt / T(6);
                    const T A1 = s_l[0][2 + q][lane];
                    const T A2 = s_l[1][2 + q][lane];
                    const T A3 = A2 + q4 * irho * s_l[0][q][lane];
                    const T A4 = T(2) * A2 - A1 + q2 * irho * (s_l[1][q][lane] + (q ? db1 : db0));
                    const T un = xo[0] + dt * xo[2] + s6 * (A1 + A2 + A3);
                    sto<T>((char*)B.u + q * fb, p, un);
                    sto<T>((char*)B.v + q * fb, p, xo[2] + d6 * (A1 + T(2) * A2 + T(2) * A3 + A4));
                    gp<double> ro = rec_slots(B, A);
                    if (ro && ne > 0) record(ro, po, q, static_cast<double>(un));
                }
            }
        } else if (act && live) {
            const long po = (long)j * n1 + i;
            T da0 = tauf_a * f0, da1 = tauf_a * f1, db0 = tauf_b * f0, db1 = tauf_b * f1;
            if (ne > 0) {
                if (ca.any()) sources(po, false, da0, da1);
                if (NF == 2 && cb.any()) sources(po, true, db0, db1);
            }
            if constexpr (PASS == PASS_APPLY) {
                char* o = (char*)apply_out(A, b);
                sto<T>(o, p, irho * (L[0][0] + da0));
                sto<T>(o + fb, p, irho * (L[0][1] + da1));
            } else if constexpr (PASS == PASS_RK1) {
                char* a1 = (char*)B.a1;
                char* a2 = (char*)B.a2;
                const T hdt = T(0.5) * dt;
                sto<T>(a1, p, irho * (L[0][0] + da0));
                sto<T>(a1 + fb, p, irho * (L[0][1] + da1));
                sto<T>(a2, p, irho * (L[0][0] + hdt * L[NF - 1][0] + db0));
                sto<T>(a2 + fb, p, irho * (L[0][1] + hdt * L[NF - 1][1] + db1));
            } else {
                char* u = (char*)B.u;
                char* v = (char*)B.v;
                const T dt2 = dt * dt;
                const T q4 = T(0.25) * dt2, q2 = T(0.5) * dt2, s6 = dt2 / T(6), d6 = dt / T(6);
                T un[2];
#pragma unroll
                for (int q = 0; q < 2; ++q) {
                    const T A1 = wc[q];
                    const T A2 = wc[2 + q];
                    const T A3 = A2 + q4 * irho * L[0][q];
                    const T A4 = T(2) * A2 - A1 + q2 * irho * (L[1][q] + (q ? db1 : db0));
                    un[q] = xo[q] + dt * xo[2 + q] + s6 * (A1 + A2 + A3);
                    sto<T>(u + q * fb, p, un[q]);
                    sto<T>(v + q * fb, p, xo[2 + q] + d6 * (A1 + T(2) * A2 + T(2) * A3 + A4));
                }
                gp<double> ro = rec_slots(B, A);
                if (ro && ne > 0) {
                    record(ro, po, 0, static_cast<double>(un[0]));
                    record(ro, po, 1, static_cast<double>(un[1]));
                }
            }
        }
        wave_sync();
    };

    // rows past je (at most NW - 1 in the last group) are evaluated on
    // clamped rows and not stored
    for (int j0 = jb; j0 <= je; j0 += NW) {
        step(std::integral_constant<int, 0>{}, j0);
        step(std::integral_constant<int, 1>{}, j0 + 1);
        step(std::integral_constant<int, 2>{}, j0 + 2);
        if constexpr (NW > 3) {
            step(std::integral_constant<int, 3 % NW>{}, j0 + 3);
            step(std::integral_constant<int, 4 % NW>{}, j0 + 4);
        }
        if constexpr (NW > 5) {
            step(std::integral_constant<int, 5 % NW>{}, j0 + 5);
            step(std::integral_constant<int, 6 % NW>{}, j0 + 6);
        }
    }
}

// One sweep in one launch: the first nframe workgroups (a multiple of 8, so
// that the interior workgroups keep their position among the 8 XCDs) apply the
// assembled frame operator, the others march over interior tiles.  The frame
// workgroups go first: their chains of dependent loads are long, and started
// last they would set the end of the launch (spreading them evenly among the
// tiles measured slower).
// A frame workgroup takes floop consecutive frame groups (nt / FRAME_LANES
// points each): fewer, longer frame workgroups in front of the tiles.
template <typename T, int ORD, int PASS, bool SPLIT>
__global__ void __launch_bounds__(SPLIT ? 128 : 64) k_pass(PassArgs A, int nframe, int floop) {
    const int bid = (int)blockIdx.x;
    if (bid < nframe) {
        for (int r = 0; r < floop; ++r) frame_sp_body<T, ORD, PASS>(A, bid * floop + r, SPLIT ? 128 : 64);
    } else {
        march_body<T, ORD, PASS, SPLIT>(A, bid - nframe);
    }
}

template <typename T, int ORD, int PASS, bool SPLIT>
__global__ void __launch_bounds__(SPLIT ? 128 : 64) k_march(PassArgs A) {
    march_body<T, ORD, PASS, SPLIT>(A, blockIdx.x);
}

// ------------------------------------------------ wide-stencil interior
// With the wide-stencil operator (D_ii^FC(c) replaced by D_i c D_i, the
// operator the narrow one is compared with in Sec. 7.1) every interior term
// is a first derivative of a first derivative, so the operator is the
// divergence of a discrete stress:
//   s1_j = c_1j1l D_1 u_l + c_1j2l D_2 u_l,   s2_j = c_2j1l D_1 u_l + c_2j2l D_2 u_l,
//   (L u)_j = D_1 s1_j + D_2 s2_j.
// At points >= R from every face all first derivatives are interior rows.
// One wave per tile of the narrow march (same geometry and point-entry
// ranges).  For output row j the input row j + 2H enters an LDS ring of
// 2H + 1 rows (with H halo columns on each side); the stress is formed at the
// middle row m = j + H from the ring, s1 into an LDS ring (D_1 s1 needs the
// neighbouring lanes), s2 into a register window (D_2 s2 needs rows j +- H).
// The row loop is unrolled by 2H + 1, so all slots are compile-time constants.
template <typename T, int ORD, int PASS>
__device__ __forceinline__ void wide_body(const PassArgs& A, int bid) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    constexpr int NW = 2 * HF + 1;
    constexpr int NF = PASS == PASS_APPLY ? 1 : 2;
    constexpr int NS = 2 * NF;
    constexpr int XW = 64 + 2 * HF;
    constexpr int R = Frame<ORD>::R;
    static_assert(R >= 2 * HF, "the wide interior reaches 2H rows beyond a tile");
    constexpr T C1 = static_cast<T>(O::d1i(HF + 1));
    constexpr T C2 = static_cast<T>(d1_outer<ORD>());
    __shared__ T s_u[NW][NS][XW];   // input rows; column of lane l at index l + H
    __shared__ T s_s[NW][NS][64];   // s1 rows

    const int total = A.total_tiles;
    const int per = (total + 7) / 8;
    const int wg = (bid % 8) * per + bid / 8;
    if (wg >= total) return;
    const int b = find_block(A, wg, false);
    BlockRef B = blk(A, b);
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const int tl = wg - B.tile_beg;
    const int ty = tl / B.tiles_x, tx = tl - ty * B.tiles_x;
    const int lane = threadIdx.x & 63;
    const int i0 = R - HF + tx * (64 - 2 * HF);     // column of lane 0
    const int i = i0 + lane;
    const bool act = lane >= HF && lane < 64 - HF && i <= n1 - 1 - R;
    const int ic = i < n1 - 1 ? i : n1 - 1;
    // lanes 0 .. 2H-1 also load a halo column: the H columns left of lane 0
    // (i0 - H >= R - 2H >= 0), then the H columns right of lane 63
    const bool halo = lane < 2 * HF;
    int ix = lane < HF ? i0 - HF + lane : i0 + 64 + (lane - HF);
    ix = ix < n1 - 1 ? ix : n1 - 1;
    const int xs = lane < HF ? lane : 64 + lane;
    const int jb = R + ty * B.tile_y;
    const int je = (jb + B.tile_y < n2 - R ? jb + B.tile_y : n2 - R) - 1;
    const unsigned fb = (unsigned)np * (unsigned)sizeof(T);
    const unsigned rowb = (unsigned)n1 * (unsigned)sizeof(T);
    const unsigned lo = (unsigned)ic * (unsigned)sizeof(T);
    const unsigned lx = (unsigned)ix * (unsigned)sizeof(T);
    const char* cbase = (const char*)B.coef;
    auto cf = [&](int k) { return cbase + (size_t)k * fb; };
    const char* fin[NS];
    {
        const void* f0p = PASS == PASS_APPLY ? apply_in(A, b) : (PASS == PASS_RK1 ? B.u : B.a1);
        const void* f1p = PASS == PASS_RK1 ? B.v : B.a2;
#pragma unroll
        for (int s = 0; s < NS; ++s) fin[s] = (const char*)(s < 2 ? f0p : f1p) + (s & 1) * (size_t)fb;
    }
    const Range rg = load_range(B.tile_rng, wg - B.tile_beg);
    const W3 ca = weights_a(A), cb = weights_b(A, B);
    T tauf_a = 0, tauf_b = 0;
    if (B.force != nullptr) {
        tauf_a = static_cast<T>(tval(B, A, B.item_f, ca));
        tauf_b = static_cast<T>(tval(B, A, B.item_f, cb));
    }
    const bool ents = rg.end > rg.beg;
    const T ih1 = T(1.0 / B.h1), ih2 = T(1.0 / B.h2);
    const T dt = static_cast<T>(B.dt);
    auto d1 = [&](T um2, T um1, T up1, T up2) -> T {
        if constexpr (HF == 2) return C1 * (up1 - um1) + C2 * (up2 - um2);
        else return C1 * (up1 - um1);
    };
    // global loads of one step, issued one step ahead of their use: the
    // entering row (and the halo column of lanes 0 .. 2H-1), the ten stiffness
    // fields at the middle row, and the per-point operands of the output row
    struct WLead {
        T w[NS], wx[NS];
        T c[10];
        T pt[3];
        T xo[PASS == PASS_RK2 ? 4 : 1];
    };
    const bool force = B.force != nullptr;
    const char* frc = force ? (const char*)B.force : cbase + (size_t)K_IRHO * fb;
    const unsigned frc1 = force ? fb : 0u;
    auto load_lead = [&](int j, WLead& P) {
        const int jj = j < je ? j : je;
        const unsigned ql = (unsigned)(jj + 2 * HF) * rowb;
        const unsigned qm = (unsigned)(jj + HF) * rowb + lo;
        const unsigned qj = (unsigned)jj * rowb + lo;
#pragma unroll
        for (int s = 0; s < NS; ++s) P.w[s] = ldo<T>(fin[s], ql + lo);
        if (halo) {
#pragma unroll
            for (int s = 0; s < NS; ++s) P.wx[s] = ldo<T>(fin[s], ql + lx);
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) P.c[k] = ldo<T>(cf(k), qm);
        P.pt[0] = ldo<T>(cf(K_IRHO), qj);
        P.pt[1] = ldo<T>(frc, qj);
        P.pt[2] = ldo<T>(frc + frc1, qj);
        if constexpr (PASS == PASS_RK2) {
            P.xo[0] = ldo<T>((const char*)B.u, qj);
            P.xo[1] = ldo<T>((const char*)B.u + fb, qj);
            P.xo[2] = ldo<T>((const char*)B.v, qj);
            P.xo[3] = ldo<T>((const char*)B.v + fb, qj);
        }
    };
    // input row r into ring slot sl (prologue)
    auto stage = [&](const int sl, const int r) {
        const unsigned q = (unsigned)r * rowb;
#pragma unroll
        for (int s = 0; s < NS; ++s) s_u[sl][s][lane + HF] = ldo<T>(fin[s], q + lo);
        if (halo) {
#pragma unroll
            for (int s = 0; s < NS; ++s) s_u[sl][s][xs] = ldo<T>(fin[s], q + lx);
        }
    };

    T s2w[NS][NW];   // s2 by ring slot

    // the stress at the middle row (ring slot sm; the ring holds rows m - H .. m + H)
    auto stress = [&](auto KC, const T (&c)[10]) {
        constexpr int K = decltype(KC)::value;
        constexpr int sm = (K + HF) % NW;
        const T n11 = c[K_C1111], n12 = c[K_C1112], n22 = c[K_C1212];
        const T p11 = c[K_C2121], p12 = c[K_C2122], p22 = c[K_C2222];
        const T m00 = c[K_C1121], m01 = c[K_C1122], m10 = c[K_C1221], m11 = c[K_C1222];
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            T a[2], g[2];   // h1 D_1 u_l and h2 D_2 u_l at (i, m)
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const int x = 2 * f + l;
                a[l] = d1(HF > 1 ? s_u[sm][x][lane] : T(0), s_u[sm][x][lane + HF - 1], s_u[sm][x][lane + HF + 1],
                          HF > 1 ? s_u[sm][x][lane + 2 * HF] : T(0));
                g[l] = d1(HF > 1 ? s_u[K % NW][x][lane + HF] : T(0), s_u[(K + HF - 1) % NW][x][lane + HF],
                          s_u[(K + HF + 1) % NW][x][lane + HF], HF > 1 ? s_u[(K + 2 * HF) % NW][x][lane + HF] : T(0));
            }
            s_s[sm][2 * f][lane] = ih1 * (n11 * a[0] + n12 * a[1]) + ih2 * (m00 * g[0] + m01 * g[1]);
            s_s[sm][2 * f + 1][lane] = ih1 * (n12 * a[0] + n22 * a[1]) + ih2 * (m10 * g[0] + m11 * g[1]);
            s2w[2 * f][sm] = ih1 * (m00 * a[0] + m10 * a[1]) + ih2 * (p11 * g[0] + p12 * g[1]);
            s2w[2 * f + 1][sm] = ih1 * (m01 * a[0] + m11 * a[1]) + ih2 * (p12 * g[0] + p22 * g[1]);
        }
    };

    // prologue: rows jb - 2H .. jb - 1 staged (slots 1 .. 2H)
#pragma unroll
    for (int r = 0; r < 2 * HF; ++r) stage(r + 1, jb - 2 * HF + r);
    WLead P;
    load_lead(jb - 2 * HF, P);

    // one row: stage row j + 2H, the stress at j + H, and (OUT) output row j
    auto step = [&](auto KC, auto OUTC, const int j) {
        constexpr int K = decltype(KC)::value;
        constexpr bool OUT = decltype(OUTC)::value;
        constexpr int sj = K % NW;
        constexpr int sl = (K + 2 * HF) % NW;
        const int jj = j < je ? j : je;     // rows past the tile end are clamped and not stored
        wave_sync();
#pragma unroll
        for (int s = 0; s < NS; ++s) s_u[sl][s][lane + HF] = P.w[s];
        if (halo) {
#pragma unroll
            for (int s = 0; s < NS; ++s) s_u[sl][s][xs] = P.wx[s];
        }
        T c[10];
#pragma unroll
        for (int k = 0; k < 10; ++k) c[k] = P.c[k];
        const T irho = P.pt[0], f0 = P.pt[1], f1 = P.pt[2];
        T xo[4] = {0, 0, 0, 0};
        if constexpr (PASS == PASS_RK2) {
#pragma unroll
            for (int k = 0; k < 4; ++k) xo[k] = P.xo[k];
        }
        load_lead(j + 1, P);
        wave_sync();
        stress(KC, c);
        if constexpr (OUT) {
            const unsigned p = (unsigned)jj * rowb + lo;
            wave_sync();
            T L[NF][2], wc[NS];
            const int lm2 = lane - 2 < 0 ? 0 : lane - 2, lm1 = lane - 1 < 0 ? 0 : lane - 1;
            const int lp1 = lane + 1 > 63 ? 63 : lane + 1, lp2 = lane + 2 > 63 ? 63 : lane + 2;
#pragma unroll
            for (int x = 0; x < NS; ++x) {
                const T a1 = d1(HF > 1 ? s_s[sj][x][lm2] : T(0), s_s[sj][x][lm1], s_s[sj][x][lp1],
                                HF > 1 ? s_s[sj][x][lp2] : T(0));
                const T a2 = d1(HF > 1 ? s2w[x][(K + NW - 2) % NW] : T(0), s2w[x][(K + NW - 1) % NW],
                                s2w[x][(K + 1) % NW], HF > 1 ? s2w[x][(K + 2) % NW] : T(0));
                L[x >> 1][x & 1] = ih1 * a1 + ih2 * a2;
                wc[x] = s_u[sj][x][lane + HF];
            }
            if (act && j <= je) {
                const long po = (long)j * n1 + i;
                T da0 = tauf_a * f0, da1 = tauf_a * f1, db0 = tauf_b * f0, db1 = tauf_b * f1;
                if (ents) {
                    if (ca.any()) point_sources<T>(B, A, rg, po, ca, da0, da1);
                    if (NF == 2 && cb.any()) point_sources<T>(B, A, rg, po, cb, db0, db1);
                }
                if constexpr (PASS == PASS_APPLY) {
                    char* o = (char*)apply_out(A, b);
                    sto<T>(o, p, irho * (L[0][0] + da0));
                    sto<T>(o + fb, p, irho * (L[0][1] + da1));
                } else if constexpr (PASS == PASS_RK1) {
                    const T hdt = T(0.5) * dt;
                    sto<T>((char*)B.a1, p, irho * (L[0][0] + da0));
                    sto<T>((char*)B.a1 + fb, p, irho * (L[0][1] + da1));
                    sto<T>((char*)B.a2, p, irho * (L[0][0] + hdt * L[NF - 1][0] + db0));
                    sto<T>((char*)B.a2 + fb, p, irho * (L[0][1] + hdt * L[NF - 1][1] + db1));
                } else {
                    const T dt2 = dt * dt;
                    const T q4 = T(0.25) * dt2, q2 = T(0.5) * dt2, s6 = dt2 / T(6), d6 = dt / T(6);
                    gp<double> ro = rec_slots(B, A);
#pragma unroll
                    for (int q = 0; q < 2; ++q) {
                        const T A1 = wc[q];
                        const T A2 = wc[2 + q];
                        const T A3 = A2 + q4 * irho * L[0][q];
                        const T A4 = T(2) * A2 - A1 + q2 * irho * (L[NF - 1][q] + (q ? db1 : db0));
                        const T un = xo[q] + dt * xo[2 + q] + s6 * (A1 + A2 + A3);
                        sto<T>((char*)B.u + q * fb, p, un);
                        sto<T>((char*)B.v + q * fb, p, xo[2 + q] + d6 * (A1 + T(2) * A2 + T(2) * A3 + A4));
                        if (ro && ents)
                            entries_at(B, rg.mid, rg.end, po, [&](const GLB Entry& E) {
                                ro[2 * E.id + q] = E.c0 * static_cast<double>(un);
                            });
                    }
                }
            }
        }
    };
    // rows jb - 2H .. jb - 1 as middle-row producers only (their slots are 1 .. 2H)
    step(std::integral_constant<int, 1>{}, std::false_type{}, jb - 2 * HF);
    step(std::integral_constant<int, 2>{}, std::false_type{}, jb - 2 * HF + 1);
    if constexpr (HF > 1) {
        step(std::integral_constant<int, 3 % NW>{}, std::false_type{}, jb - 2);
        step(std::integral_constant<int, 4 % NW>{}, std::false_type{}, jb - 1);
    }
    for (int j0 = jb; j0 <= je; j0 += NW) {
        step(std::integral_constant<int, 0>{}, std::true_type{}, j0);
        step(std::integral_constant<int, 1>{}, std::true_type{}, j0 + 1);
        step(std::integral_constant<int, 2>{}, std::true_type{}, j0 + 2);
        if constexpr (NW > 3) {
            step(std::integral_constant<int, 3 % NW>{}, std::true_type{}, j0 + 3);
            step(std::integral_constant<int, 4 % NW>{}, std::true_type{}, j0 + 4);
        }
    }
}

template <typename T, int ORD, int PASS>
__global__ void __launch_bounds__(64) k_wide(PassArgs A) {
    wide_body<T, ORD, PASS>(A, blockIdx.x);
}

// one sweep of the wide-stencil operator in one launch: frame workgroups
// first (as k_pass), then the interior tiles
template <typename T, int ORD, int PASS>
__global__ void __launch_bounds__(64) k_pass_wide(PassArgs A, int nframe, int floop) {
    const int bid = (int)blockIdx.x;
    if (bid < nframe) {
        for (int r = 0; r < floop; ++r) frame_sp_body<T, ORD, PASS>(A, bid * floop + r, 64);
    } else {
        wide_body<T, ORD, PASS>(A, bid - nframe);
    }
}

// ------------------------------------------------------------ gradients
// Coefficient gradient of the bilinear form B(c) = z^T H L(c) y of one block
// (H = h1 h2 H^1 (x) H^2, L the reference-frame operator of the kernels
// above), accumulated per point.  Each thread owns one grid point and gathers
// every term in which the coefficients of that point appear:
//   * narrow terms: h^2 (D2^FC(b) y)_r = sum_m k_rm(b) (y_m - y_r) with k_rm
//     linear in b (interior edge weights, closure tables), so
//     dB/db_p = sum_r H_r z_r sum_m dk_rm/db_p (y_m - y_r) / h^2;
//   * mixed terms D_1 (M D_2 y) and D_2 (M^T D_1 y): dB/dM_ab(p) =
//     (D_1^T H z_a)(p) (D_2 y_b)(p) + (D_2^T H z_b)(p) (D_1 y_a)(p);
//   * traction SAT -(1/w) nu c_ajkl D_k y_l at the face points, and the
//     displacement SAT (normal part on the REACH points next to the face,
//     tangential part (D_t z)^T H_t q and penalty at the face points);
//   * rho~ (1/rho~ scales every stage): dB/drho~ = -H (z . a), a the stage value.

// weight of b_{r+o} in the interior edge weight of u_{r+e} - u_r (order 4:
// e = -2, -1, 1, 2 and o = -2..2; order 2: e = -1, 1 and o = -1..1)
template <int ORD>
__device__ __forceinline__ double d2_edge_dw(int e, int o) {
    if constexpr (ORD == 4) {
        constexpr double s6 = 1.0 / 6.0, e8 = 0.125, hf = 0.5;
        switch (e) {
            case -2: return o == -1 ? s6 : (o == -2 || o == 0) ? -e8 : 0.0;
            case -1: return (o == -2 || o == 1) ? s6 : (o == -1 || o == 0) ? hf : 0.0;
            case 1: return (o == -1 || o == 2) ? s6 : (o == 0 || o == 1) ? hf : 0.0;
            case 2: return o == 1 ? s6 : (o == 0 || o == 2) ? -e8 : 0.0;
            default: return 0.0;
        }
    } else {
        return (e == -1 && (o == -1 || o == 0)) || (e == 1 && (o == 0 || o == 1)) ? 0.5 : 0.0;
    }
}

// Closure rows of d2_coef_grad for the coefficient at distance P from the end
// of a line (lo: the lower end, else the mirrored upper end): with P a
// compile-time index the table weights are constants and their zeros drop out.
template <typename T, int ORD, int P>
__device__ __forceinline__ double d2_closure_grad_at(gcp<T> z, gcp<T> y, long st, int n, bool lo) {
    using O = Op<ORD>;
    double acc = 0.0;
#pragma unroll
    for (int r = 0; r < O::R0; ++r) {
        const int ir = lo ? r : n - 1 - r;
        const double yr = (double)y[(long)ir * st];
        double sum = 0.0;
#pragma unroll
        for (int m = 0; m < O::W; ++m) {
            if (m == r) continue;
            const double w = O::d2c(r, m, P);
            if (w != 0.0) sum += w * ((double)y[(long)(lo ? m : n - 1 - m) * st] - yr);
        }
        acc += hnorm<ORD>(ir, n) * (double)z[(long)ir * st] * sum;
    }
    return acc;
}
template <typename T, int ORD, int P>
__device__ __forceinline__ double d2_closure_grad(int p, gcp<T> z, gcp<T> y, long st, int n, bool lo) {
    if (p == P) return d2_closure_grad_at<T, ORD, P>(z, y, st, n, lo);
    if constexpr (P + 1 < Op<ORD>::W) return d2_closure_grad<T, ORD, P + 1>(p, z, y, st, n, lo);
    else return 0.0;
}

// sum_r H^_r z_r sum_m dk_rm/db_p (y_m - y_r) along a line (stride st, n points)
template <typename T, int ORD>
__device__ double d2_coef_grad(gcp<T> z, gcp<T> y, long st, int p, int n) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    double acc = 0.0;
    // interior rows r = p - o
#pragma unroll
    for (int o = -HF; o <= HF; ++o) {
        const int r = p - o;
        if (r < O::R0 || r > n - 1 - O::R0) continue;
        const double yr = (double)y[(long)r * st];
        double sum = 0.0;
#pragma unroll
        for (int e = -HF; e <= HF; ++e) {
            if (e == 0) continue;
            const double w = d2_edge_dw<ORD>(e, o);
            if (w != 0.0) sum += w * ((double)y[(long)(r + e) * st] - yr);
        }
        acc += hnorm<ORD>(r, n) * (double)z[(long)r * st] * sum;
    }
    // closure rows at the lower end (coefficient index p) and the upper end (n-1-p)
    if (p < O::W) acc += d2_closure_grad<T, ORD, 0>(p, z, y, st, n, true);
    if (n - 1 - p < O::W) acc += d2_closure_grad<T, ORD, 0>(n - 1 - p, z, y, st, n, false);
    return acc;
}

// d2_coef_grad away from the closures (every row r = p - o an interior row,
// H^_r = 1), from register windows zw[k] = z_{p-H+k} and yw[k] = y_{p-2H+k};
// the same operations in the same order as d2_coef_grad
template <int ORD>
__device__ __forceinline__ double d2_coef_grad_win(const double* zw, const double* yw) {
    constexpr int HF = Op<ORD>::HALF;
    double acc = 0.0;
#pragma unroll
    for (int o = -HF; o <= HF; ++o) {
        const double yr = yw[2 * HF - o];
        double sum = 0.0;
#pragma unroll
        for (int e = -HF; e <= HF; ++e) {
            if (e == 0) continue;
            const double w = d2_edge_dw<ORD>(e, o);
            if (w != 0.0) sum += w * (yw[2 * HF - o + e] - yr);
        }
        acc += 1.0 * zw[HF - o] * sum;
    }
    return acc;
}

// the narrow coefficient gradients of one line direction at index p: the
// window path where no closure row is involved, else the general one
template <typename T, int ORD>
__device__ __forceinline__ void d2_coef_grad_pairs(gcp<T> z0, gcp<T> z1, gcp<T> y0, gcp<T> y1, long st, int p, int n,
                                                   double& g00, double& g01, double& g11) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    constexpr int LO = (O::R0 + HF > O::W) ? O::R0 + HF : O::W;
    if (p >= LO && p <= n - 1 - LO) {
        double zw[2][2 * HF + 1], yw[2][4 * HF + 1];
#pragma unroll
        for (int k = 0; k <= 2 * HF; ++k) {
            zw[0][k] = (double)z0[(long)(p - HF + k) * st];
            zw[1][k] = (double)z1[(long)(p - HF + k) * st];
        }
#pragma unroll
        for (int k = 0; k <= 4 * HF; ++k) {
            yw[0][k] = (double)y0[(long)(p - 2 * HF + k) * st];
            yw[1][k] = (double)y1[(long)(p - 2 * HF + k) * st];
        }
        g00 = d2_coef_grad_win<ORD>(zw[0], yw[0]);
        g01 = d2_coef_grad_win<ORD>(zw[0], yw[1]) + d2_coef_grad_win<ORD>(zw[1], yw[0]);
        g11 = d2_coef_grad_win<ORD>(zw[1], yw[1]);
    } else {
        g00 = d2_coef_grad<T, ORD>(z0, y0, st, p, n);
        g01 = d2_coef_grad<T, ORD>(z0, y1, st, p, n) + d2_coef_grad<T, ORD>(z1, y0, st, p, n);
        g11 = d2_coef_grad<T, ORD>(z1, y1, st, p, n);
    }
}

// distance from the faces beyond which every row of the coefficient gradient
// is an interior row (the D2^FC closure plus the stencil half width)
template <int ORD>
__host__ __device__ constexpr int grad_lo() {
    using O = Op<ORD>;
    return (O::R0 + O::HALF > O::W) ? O::R0 + O::HALF : O::W;
}

// (D1^ T (H^ z))_p = sum_r D1^[r][p] H^_r z_r along a line (D1^ = h D1)
template <typename T, int ORD>
__device__ double d1t_weighted(gcp<T> z, long st, int p, int n) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    double acc = 0.0;
#pragma unroll
    for (int k = -HF; k <= HF; ++k) {
        const int r = p + k;
        if (k == 0 || r < O::NB || r > n - 1 - O::NB) continue;
        acc += O::d1i(-k + HF) * hnorm<ORD>(r, n) * (double)z[(long)r * st];
    }
    if (p < 6) {
#pragma unroll
        for (int r = 0; r < O::NB; ++r) {
            const double w = table_d1b<ORD>(r, p);
            if (w != 0.0) acc += w * hnorm<ORD>(r, n) * (double)z[(long)r * st];
        }
    }
    if (n - 1 - p < 6) {
#pragma unroll
        for (int r = 0; r < O::NB; ++r) {
            const double w = -table_d1b<ORD>(r, n - 1 - p);
            if (w != 0.0) acc += w * hnorm<ORD>(n - 1 - r, n) * (double)z[(long)(n - 1 - r) * st];
        }
    }
    return acc;
}

// Points closer than grad_lo<ORD>() to a face (closure rows and faces): the
// general rows; k_grad_int below takes the rest.  A workgroup takes 64 band
// points; wave w evaluates term group w for all of them (0-2: the x1 i = k
// terms of the component pairs (1,1), (1,2) + (2,1), (2,2); 3-5: the same along
// x2; 6: mixed terms; 7: face terms), so the long chains of closure-row loads
// are spread over eight waves, and wave 0 adds the groups (through LDS) and
// the rho~ term.
constexpr int GRAD_PARTS = 8;

// operand of stage s (uniform) and block k, read from the kernel argument with
// static indices only (a runtime index would copy the argument to per-lane
// scratch memory)
__device__ __forceinline__ const void* grad_operand(const void* const (&f)[GRAD_STAGES_MAX][MAX_APPLY_BLOCKS], int s,
                                                    int k) {
    const void* r = f[0][k];
#pragma unroll
    for (int q = 1; q < GRAD_STAGES_MAX; ++q)
        if (q == s) r = f[q][k];
    return r;
}
__device__ __forceinline__ double grad_alpha(const GradArgs& G, int s, int& tcol) {
    double al = G.alpha[0];
    tcol = G.tcol[0];
#pragma unroll
    for (int q = 1; q < GRAD_STAGES_MAX; ++q)
        if (q == s) {
            al = G.alpha[q];
            tcol = G.tcol[q];
        }
    return al;
}

// A launch accumulates the stages 0 .. nstages-1 (blockIdx.y = stage); with
// more than one stage each stage writes its sums to G.part and
// k_grad_band_sum adds them up in stage order.
template <typename T, int ORD>
__global__ void __launch_bounds__(GRAD_PARTS * 64) k_grad(GradArgs G) {
    using O = Op<ORD>;
    __shared__ double s_g[GRAD_PARTS][10][64];
    const int part = (int)(threadIdx.x >> 6);
    const int st = (int)blockIdx.y;
    const long gid = (long)blockIdx.x * 64 + (threadIdx.x & 63);
    // block of this point and its operands
    int b = 0;
    long end = G.boff[1];
    gcp<T> z = gc<T>(grad_operand(G.z, st, 0));
    gcp<T> y = gc<T>(grad_operand(G.y, st, 0));
    gcp<T> a = gc<T>(grad_operand(G.a, st, 0));
    double* gcb = G.gc[0];
    double* grb = G.grt[0];
    long base = 0;
#pragma unroll
    for (int k = 1; k < MAX_APPLY_BLOCKS; ++k)
        if (k < G.nblocks && gid >= G.boff[k]) {
            b = k;
            base = G.boff[k];
            end = G.boff[k + 1];
            z = gc<T>(grad_operand(G.z, st, k));
            y = gc<T>(grad_operand(G.y, st, k));
            a = gc<T>(grad_operand(G.a, st, k));
            gcb = G.gc[k];
            grb = G.grt[k];
        }
    int tcol;
    const double al = grad_alpha(G, st, tcol);
    const bool valid = gid < end;
    BlockRef B = ((const GLB BlockDesc*)G.blocks)[b];
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    constexpr int LO = grad_lo<ORD>();
    int i, j;
    const int kb = valid ? (int)(gid - base) : 0;
    if (n1 > 2 * LO && n2 > 2 * LO) {
        frame_ij(kb, n1, n2, LO, i, j);     // the band of width LO
    } else {
        j = kb / n1;                        // no interior: every point
        i = kb - j * n1;
    }
    const long p = (long)j * n1 + i;
    const double h1 = B.h1, h2 = B.h2;
    const double hn1 = hnorm<ORD>(i, n1), hn2 = hnorm<ORD>(j, n2);
    const long row = (long)j * n1;
    double g[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double tzx[2] = {0, 0}, tzy[2] = {0, 0}, dyx[2] = {0, 0}, dyy[2] = {0, 0};   // (D^T H z), D y at p
    const bool nx = part == 6 || (part <= 2 && G.wide), ny = part == 6 || (part >= 3 && part <= 5 && G.wide);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (valid && nx) {
            tzx[c] = d1t_weighted<T, ORD>(z + c * np + row, 1, i, n1);
            dyx[c] = (double)d1_line<T, ORD>(y + c * np + row, 1, i, n1);
        }
        if (valid && ny) {
            tzy[c] = d1t_weighted<T, ORD>(z + c * np + i, n1, j, n2);
            dyy[c] = (double)d1_line<T, ORD>(y + c * np + i, n1, j, n2);
        }
    }
    // i = k terms (stored fields: x1 C1111, C1112, C1212; x2 C2121, C2122, C2222)
    if (valid && part <= 5) {
        const bool ax2 = part >= 3;
        const int pr = ax2 ? part - 3 : part;              // pair: (1,1), (1,2) + (2,1), (2,2)
        const double f = ax2 ? h1 * hn1 / h2 : h2 * hn2 / h1;
        // member-wise selects: indexing a local array with a runtime choice would put it in scratch memory
        const double tz0 = ax2 ? tzy[0] : tzx[0], tz1 = ax2 ? tzy[1] : tzx[1];
        const double dy0 = ax2 ? dyy[0] : dyx[0], dy1 = ax2 ? dyy[1] : dyx[1];
        double gv;
        if (G.wide) {
            // z^T H D_i b D_i y: dB/db_p = (D_i^T H z)(p) (D_i y)(p), as for the mixed terms
            gv = pr == 0 ? tz0 * dy0 : (pr == 1 ? tz0 * dy1 + tz1 * dy0 : tz1 * dy1);
        } else {
            const long st = ax2 ? n1 : 1;
            const long l0 = ax2 ? (long)i : row;            // start of the line through p
            const int pp = ax2 ? j : i, nn = ax2 ? n2 : n1;
            if (pr == 0) {
                gv = d2_coef_grad<T, ORD>(z + l0, y + l0, st, pp, nn);
            } else if (pr == 1) {
                gv = d2_coef_grad<T, ORD>(z + l0, y + np + l0, st, pp, nn) +
                     d2_coef_grad<T, ORD>(z + np + l0, y + l0, st, pp, nn);
            } else {
                gv = d2_coef_grad<T, ORD>(z + np + l0, y + np + l0, st, pp, nn);
            }
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k == pr) {
                if (ax2) g[k == 0 ? K_C2121 : (k == 1 ? K_C2122 : K_C2222)] += f * gv;
                else g[k == 0 ? K_C1111 : (k == 1 ? K_C1112 : K_C1212)] += f * gv;
            }
        }
    }
    // mixed terms: M_ab = c_1a2b (C1121, C1122, C1221, C1222)
    if (valid && part == 6) {
        const int km[2][2] = {{K_C1121, K_C1122}, {K_C1221, K_C1222}};
#pragma unroll
        for (int aa = 0; aa < 2; ++aa)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) g[km[aa][bb]] += hn2 * tzx[aa] * dyy[bb] + hn1 * tzy[bb] * dyx[aa];
    }
    // faces through this point
#pragma unroll 1
    for (int f = 0; f < 4 && valid && part == 7; ++f) {
        const int ax = f >> 1, sd = f & 1;
        const bool on = ax == 0 ? (i == (sd ? n1 - 1 : 0)) : (j == (sd ? n2 - 1 : 0));
        if (!on) continue;
        const GLB FaceDesc& F = B.face[f];
        const int t = ax == 0 ? j : i;
        const int nt = ax == 0 ? n2 : n1;
        const int na = ax == 0 ? n1 : n2;
        const double ht = ax == 0 ? h2 : h1, ha = ax == 0 ? h1 : h2;
        const double wq = ht * hnorm<ORD>(t, nt);      // face quadrature weight
        const double iw = 1.0 / F.w;
        const double nu = sd ? 1.0 : -1.0;
        // N_jl (face-normal narrow) and M_jl fields as stored indices
        const int kn[2][2] = {{ax == 0 ? K_C1111 : K_C2121, ax == 0 ? K_C1112 : K_C2122},
                              {ax == 0 ? K_C1112 : K_C2122, ax == 0 ? K_C1212 : K_C2222}};
        const int km[2][2] = {{K_C1121, K_C1122}, {K_C1221, K_C1222}};
        const long st_n = ax == 0 ? 1 : n1;      // stride along the normal
        const long st_t = ax == 0 ? n1 : 1;      // stride along the face
        const long p_line_n = ax == 0 ? row : i; // start of the normal line through p
        const long p_line_t = ax == 0 ? i : row; // start of the face line through p
        const int pn = ax == 0 ? i : j;          // index along the normal line
        if (F.kind == BC_TRACTION || F.kind == BC_ROBIN) {
            double dn_y[2], dt_y[2];
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                dn_y[l] = (double)d1_line<T, ORD>(y + l * np + p_line_n, st_n, pn, na) / ha;
                dt_y[l] = (double)d1_line<T, ORD>(y + l * np + p_line_t, st_t, t, nt) / ht;
            }
            const double zc[2] = {(double)z[p], (double)z[np + p]};
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    g[kn[jj][l]] += -wq * nu * zc[jj] * dn_y[l];
                    if (ax == 0) g[km[jj][l]] += -wq * nu * zc[jj] * dt_y[l];    // c_1j2l D_2
                    else g[km[l][jj]] += -wq * nu * zc[jj] * dt_y[l];            // c_2j1l = M_lj, D_1
                }
        } else if (F.kind == BC_DISPLACEMENT) {
            double del[2] = {(double)y[p], (double)y[np + p]};
            if (!G.homogeneous && F.g) {
                const double tau = ((const GLB double*)G.tau)[3 * F.item_g + tcol];
                gcp<T> gg = gc<T>(F.g);
                del[0] -= tau * (double)gg[t];
                del[1] -= tau * (double)gg[F.nf + t];
            }
            // normal part: sum over the REACH points along the normal
            double zn[2] = {0.0, 0.0};
#pragma unroll
            for (int dn = 0; dn < O::REACH; ++dn) {
                const int q = sd ? na - 1 - dn : dn;
                const double cfq = -O::d1b(0, dn) * wq / ha;
#pragma unroll
                for (int c = 0; c < 2; ++c) zn[c] += cfq * (double)z[c * np + p_line_n + (long)q * st_n];
            }
            // tangential part: (D_t z)(t)
            double dtz[2];
#pragma unroll
            for (int c = 0; c < 2; ++c) dtz[c] = (double)d1_line<T, ORD>(z + c * np + p_line_t, st_t, t, nt) / ht;
            const double pen = 2.0 * B.beta * iw * wq;
            const double zc[2] = {(double)z[p], (double)z[np + p]};
#pragma unroll
            for (int jj = 0; jj < 2; ++jj)
#pragma unroll
                for (int l = 0; l < 2; ++l) {
                    g[kn[jj][l]] += (zn[jj] - pen * zc[jj]) * del[l];
                    if (ax == 0) g[km[l][jj]] += wq * dtz[jj] * nu * del[l];     // q_j = nu M_lj delta_l
                    else g[km[jj][l]] += wq * dtz[jj] * nu * del[l];             // q_j = nu M_jl delta_l
                }
        }
    }
    const int lane = (int)(threadIdx.x & 63);
#pragma unroll
    for (int k = 0; k < 10; ++k) s_g[part][k][lane] = g[k];
    __syncthreads();
    if (part != 0 || !valid) return;
    const double Hp = h1 * h2 * hn1 * hn2;
    const double rt = -al * Hp * ((double)z[p] * (double)a[p] + (double)z[np + p] * (double)a[np + p]);
    if (G.nstages == 1) {
        gp<double> gq = (gp<double>)gcb;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < GRAD_PARTS; ++w) sum += s_g[w][k][lane];
            gq[(long)k * np + p] += al * sum;
        }
        ((gp<double>)grb)[p] += rt;
    } else {
        gp<double> pt = (gp<double>)G.part + (long)st * GRAD_TERMS * G.nband + gid;
#pragma unroll
        for (int k = 0; k < 10; ++k) {
            double sum = 0.0;
#pragma unroll
            for (int w = 0; w < GRAD_PARTS; ++w) sum += s_g[w][k][lane];
            pt[(long)k * G.nband] = al * sum;
        }
        pt[(long)10 * G.nband] = rt;
    }
}

// Band points of a multi-stage launch: the stages' partial sums added in
// stage order, then to the gradient fields.
template <int ORD>
__global__ void __launch_bounds__(256) k_grad_band_sum(GradArgs G) {
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    if (gid >= G.nband) return;
    int b = 0;
    double* gcb = G.gc[0];
    double* grb = G.grt[0];
    long base = 0;
#pragma unroll
    for (int k = 1; k < MAX_APPLY_BLOCKS; ++k)
        if (k < G.nblocks && gid >= G.boff[k]) {
            b = k;
            base = G.boff[k];
            gcb = G.gc[k];
            grb = G.grt[k];
        }
    BlockRef B = ((const GLB BlockDesc*)G.blocks)[b];
    const int n1 = B.n1, n2 = B.n2;
    constexpr int LO = grad_lo<ORD>();
    int i, j;
    const int kb = (int)(gid - base);
    if (n1 > 2 * LO && n2 > 2 * LO) {
        frame_ij(kb, n1, n2, LO, i, j);
    } else {
        j = kb / n1;
        i = kb - j * n1;
    }
    const long np = (long)n1 * n2;
    const long p = (long)j * n1 + i;
    gcp<double> pt = (gcp<double>)G.part + gid;
    const long sst = (long)GRAD_TERMS * G.nband;
#pragma unroll
    for (int k = 0; k <= 10; ++k) {
        double sum = pt[(long)k * G.nband];
#pragma unroll
        for (int q = 1; q < GRAD_STAGES_MAX; ++q)
            if (q < G.nstages) sum += pt[q * sst + (long)k * G.nband];
        if (k < 10) ((gp<double>)gcb)[(long)k * np + p] += sum;
        else ((gp<double>)grb)[p] += sum;
    }
}


// Interior points (>= grad_lo<ORD>() from every face): only interior rows of
// D1 and D2^FC, no faces, unit norm weights around the point.
template <typename T, int ORD>
__global__ void __launch_bounds__(256) k_grad_int(GradArgs G) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    constexpr int LO = grad_lo<ORD>();
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    int b = 0;
    long end = G.off[1];
    double* gcb = G.gc[0];
    double* grb = G.grt[0];
    long base = 0;
#pragma unroll
    for (int k = 1; k < MAX_APPLY_BLOCKS; ++k)
        if (k < G.nblocks && gid >= G.off[k]) {
            b = k;
            base = G.off[k];
            end = G.off[k + 1];
            gcb = G.gc[k];
            grb = G.grt[k];
        }
    if (gid >= end) return;
    BlockRef B = ((const GLB BlockDesc*)G.blocks)[b];
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const int ni1 = n1 - 2 * LO;
    const int q = (int)(gid - base);
    const int j = LO + q / ni1, i = LO + q % ni1;
    const long p = (long)j * n1 + i;
    const double h1 = B.h1, h2 = B.h2;
    const double fx = h2 / h1, fy = h1 / h2;
    const int km[2][2] = {{K_C1121, K_C1122}, {K_C1221, K_C1222}};
    // sums over the stages, added to the gradient fields once
    double gt[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    double rt = 0.0;
#pragma unroll 1
    for (int st = 0; st < G.nstages; ++st) {
        gcp<T> z = gc<T>(grad_operand(G.z, st, 0));
        gcp<T> y = gc<T>(grad_operand(G.y, st, 0));
        gcp<T> a = gc<T>(grad_operand(G.a, st, 0));
#pragma unroll
        for (int k = 1; k < MAX_APPLY_BLOCKS; ++k)
            if (k == b) {
                z = gc<T>(grad_operand(G.z, st, k));
                y = gc<T>(grad_operand(G.y, st, k));
                a = gc<T>(grad_operand(G.a, st, k));
            }
        // windows of z (+-H) and y (+-2H) along both lines through p
        double zx[2][2 * HF + 1], zy[2][2 * HF + 1], yx[2][4 * HF + 1], yy[2][4 * HF + 1];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
#pragma unroll
            for (int k = 0; k <= 2 * HF; ++k) {
                zx[c][k] = (double)z[c * np + p + (k - HF)];
                zy[c][k] = (double)z[c * np + p + (long)(k - HF) * n1];
            }
#pragma unroll
            for (int k = 0; k <= 4 * HF; ++k) {
                yx[c][k] = (double)y[c * np + p + (k - 2 * HF)];
                yy[c][k] = (double)y[c * np + p + (long)(k - 2 * HF) * n1];
            }
        }
        // interior rows: h D1 y at p and (h D1^T z)_p (norm weights 1 around p)
        double tzx[2], tzy[2], dyx[2], dyy[2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            tzx[c] = tzy[c] = dyx[c] = dyy[c] = 0.0;
#pragma unroll
            for (int k = 1; k <= HF; ++k) {
                const double w = O::d1i(HF + k);
                tzx[c] += w * (zx[c][HF - k] - zx[c][HF + k]);
                tzy[c] += w * (zy[c][HF - k] - zy[c][HF + k]);
                dyx[c] += w * (yx[c][2 * HF + k] - yx[c][2 * HF - k]);
                dyy[c] += w * (yy[c][2 * HF + k] - yy[c][2 * HF - k]);
            }
        }
        double g[10];
        if (G.wide) {
            g[K_C1111] = fx * tzx[0] * dyx[0];
            g[K_C1112] = fx * (tzx[0] * dyx[1] + tzx[1] * dyx[0]);
            g[K_C1212] = fx * tzx[1] * dyx[1];
            g[K_C2121] = fy * tzy[0] * dyy[0];
            g[K_C2122] = fy * (tzy[0] * dyy[1] + tzy[1] * dyy[0]);
            g[K_C2222] = fy * tzy[1] * dyy[1];
        } else {
            g[K_C1111] = fx * d2_coef_grad_win<ORD>(zx[0], yx[0]);
            g[K_C1112] = fx * (d2_coef_grad_win<ORD>(zx[0], yx[1]) + d2_coef_grad_win<ORD>(zx[1], yx[0]));
            g[K_C1212] = fx * d2_coef_grad_win<ORD>(zx[1], yx[1]);
            g[K_C2121] = fy * d2_coef_grad_win<ORD>(zy[0], yy[0]);
            g[K_C2122] = fy * (d2_coef_grad_win<ORD>(zy[0], yy[1]) + d2_coef_grad_win<ORD>(zy[1], yy[0]));
            g[K_C2222] = fy * d2_coef_grad_win<ORD>(zy[1], yy[1]);
        }
#pragma unroll
        for (int aa = 0; aa < 2; ++aa)
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) g[km[aa][bb]] = tzx[aa] * dyy[bb] + tzy[bb] * dyx[aa];
        int tcol;
        const double al = grad_alpha(G, st, tcol);
#pragma unroll
        for (int k = 0; k < 10; ++k) gt[k] += al * g[k];
        rt += -al * h1 * h2 * ((double)z[p] * (double)a[p] + (double)z[np + p] * (double)a[np + p]);
    }
    gp<double> gq = (gp<double>)gcb;
#pragma unroll
    for (int k = 0; k < 10; ++k) gq[(long)k * np + p] += gt[k];
    ((gp<double>)grb)[p] += rt;
}

// y = sum_k c_k x_k (elementwise, at most LINCOMB_MAX terms; y may be one of the x_k)
struct LincombArgs {
    double c[LINCOMB_MAX];
    const void* x[LINCOMB_MAX];
};
template <typename T>
__global__ void __launch_bounds__(256) k_lincomb(int nterms, LincombArgs a, T* y, long count) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    double acc = a.c[0] * (double)((const T*)a.x[0])[i];
#pragma unroll
    for (int k = 1; k < LINCOMB_MAX; ++k)
        if (k < nterms) acc += a.c[k] * (double)((const T*)a.x[k])[i];
    y[i] = static_cast<T>(acc);
}

// Stage values of one classical RK4 step of u'' = a(u) from its end points
// (u0, v0) -> (u1, v1) and its first two slopes a1, a2 (sbpe_rk4_stages):
// U2 = u0 + dt/2 v0, U3 = U2 + dt^2/4 a1, U4 = u0 + dt v0 + dt^2/2 a2, copies
// of a1 and a2, and the slopes a3, a4 solved from the step's update
// u1 = u0 + dt v0 + dt^2/6 (a1 + a2 + a3), v1 = v0 + dt/6 (a1 + 2 a2 + 2 a3 + a4).
template <typename T>
__global__ void __launch_bounds__(256) k_rk4_stages(Rk4StageArgs a, long count) {
    const long i = (long)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    const double dt = a.dt;
    const double u0 = (double)((const T*)a.u0)[i], v0 = (double)((const T*)a.v0)[i];
    const double a1 = (double)((const T*)a.a1)[i], a2 = (double)((const T*)a.a2)[i];
    const double U2 = u0 + 0.5 * dt * v0;
    if (a.out[0]) ((T*)a.out[0])[i] = static_cast<T>(U2);
    if (a.out[1]) ((T*)a.out[1])[i] = static_cast<T>(U2 + 0.25 * dt * dt * a1);
    if (a.out[2]) ((T*)a.out[2])[i] = static_cast<T>(u0 + dt * v0 + 0.5 * dt * dt * a2);
    if (a.out[3]) ((T*)a.out[3])[i] = static_cast<T>(a1);
    if (a.out[4]) ((T*)a.out[4])[i] = static_cast<T>(a2);
    if (a.out[5] || a.out[6]) {
        const double u1 = (double)((const T*)a.u1)[i], v1 = (double)((const T*)a.v1)[i];
        const double a3 = 6.0 * (u1 - u0 - dt * v0) / (dt * dt) - a1 - a2;
        if (a.out[5]) ((T*)a.out[5])[i] = static_cast<T>(a3);
        if (a.out[6]) ((T*)a.out[6])[i] = static_cast<T>(6.0 * (v1 - v0) / dt - a1 - 2.0 * a2 - 2.0 * a3);
    }
}

template <typename T>
__global__ void __launch_bounds__(256) k_rec_adjoint(const RecAdj* ent, int nent, const double* r, RecAdjArgs A) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= nent) return;
    const GLB RecAdj& e = ((const GLB RecAdj*)ent)[k];
    const int b = e.block;
    T* u = nullptr;
    long np = 0;
#pragma unroll
    for (int q = 0; q < MAX_APPLY_BLOCKS; ++q)
        if (q == b) {
            u = (T*)A.u[q];
            np = A.np[q];
        }
    const GLB double* rr = (const GLB double*)r + 2 * e.rec;
    atomicAdd(&u[e.p], static_cast<T>(A.scale * e.w * rr[0]));
    atomicAdd(&u[np + e.p], static_cast<T>(A.scale * e.w * rr[1]));
}

// -------------------------------------------------------------- energy
// per point H_p rho~_p (|v|^2 - u . a) with a = rho~^{-1} D^tot u already in a1;
// partial sums per workgroup in FP64, then one workgroup sums them in order.
template <typename T, int ORD>
__global__ void __launch_bounds__(256) k_energy_partial(const BlockDesc* blocks, int nblocks, double* partial) {
    __shared__ double red[256];
    double acc = 0.0;
    long gid = (long)blockIdx.x * 256 + threadIdx.x;
    const long stride = (long)gridDim.x * 256;
    for (int b = 0; b < nblocks; ++b) {
        const GLB BlockDesc& B = ((const GLB BlockDesc*)blocks)[b];
        const long np = (long)B.n1 * B.n2;
        gcp<T> u = gc<T>(B.u);
        gcp<T> v = gc<T>(B.v);
        gcp<T> a = gc<T>(B.a1);
        gcp<T> c = gc<T>(B.coef);
        for (long p = gid; p < np; p += stride) {
            const int j = (int)(p / B.n1), i = (int)(p - (long)j * B.n1);
            const double H = B.h1 * B.h2 * hnorm<ORD>(i, B.n1) * hnorm<ORD>(j, B.n2);
            const double rt = 1.0 / static_cast<double>(c[(long)K_IRHO * np + p]);
            const double v0 = v[p], v1 = v[np + p];
            const double x0 = u[p], x1 = u[np + p];
            acc += H * rt * (v0 * v0 + v1 * v1 - x0 * static_cast<double>(a[p]) - x1 * static_cast<double>(a[np + p]));
        }
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

}  // namespace sbpe
