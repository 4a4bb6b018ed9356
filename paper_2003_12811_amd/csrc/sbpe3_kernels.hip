// The scheme on a single curvilinear 3-D block (d = 3): one right-hand-side
// evaluation per grid point, fused with the two-sweep RK4 passes of the 2-D
// path (sbpe_internal.h).  Reference-frame forms, as in 2-D:
//   * volume: DD_ik(c_ijkl) u_l = sum_i D_ii^FC(c_ijil) u_l + sum_{i != k} D_i (c_ijkl D_k u_l)
//     (Sec. 4.6-4.7), every 1-D row boundary-aware (the closure tables of
//     sbpe_tables.h through the line helpers of sbpe_device.h);
//   * traction face (Sec. 5.1): r_j -= (1/w_a) (nu_a c_ajkl D_k u_l - Jhat g_j);
//   * displacement face (Sec. 5.2, d = 3): with delta = u - g on the face,
//     the normal part of sum_k H^{-1} D_k^T (e_f H_f nu_a c_alkj delta_l) on the
//     REACH points next to the face, its two tangential parts
//     (1/w_a) H_t^{-1} D_t^T H_t (nu_a c_altj delta_l) at the face, and the
//     penalty -(beta d / w_a^2) c_ajal delta_l;
//   * r = rho~ a: a = rho~^{-1} (r + J f).
// One thread per (point, field): the two fields of an RK sweep (u and v, or
// A1 and A2) sit in neighbouring lanes and exchange their results.  The mixed
// terms run in flux form: k_flux3 stores F_ij = sum_{k != i} c_ijkl D_k u_l at
// every point, and the point kernel takes sum_i D_i F_ij, the same operator
// with one coefficient read per point instead of one per stencil point.
// Every stencil value comes from global memory (the caches serve the repeats).
#include <hip/hip_runtime.h>

#include "sbpe3_internal.h"
#include "sbpe_device.h"

namespace sbpe {

namespace {

__device__ __forceinline__ int sym3(int j, int l) {
    const int a = j < l ? j : l, b = j < l ? l : j;
    return a == 0 ? b : (a == 1 ? 2 + b : 5);
}
// stored field of c_ijil (narrow, direction i) and of c_ijkl, i != k
__device__ __forceinline__ int fN(int i, int j, int l) { return 6 * i + sym3(j, l); }
__device__ __forceinline__ int fM(int i, int k, int j, int l) {
    const int a = i < k ? i : k, b = i < k ? k : i;
    const int P = a == 0 ? (b == 1 ? 0 : 1) : 2;
    return i < k ? 18 + 9 * P + 3 * j + l : 18 + 9 * P + 3 * l + j;
}

struct Geo3 {
    int n[3];
    long st[3];
    long np;
    double h[3];
};

__device__ __forceinline__ Geo3 geo3(const Args3& A) {
    Geo3 g;
    g.n[0] = A.n1;
    g.n[1] = A.n2;
    g.n[2] = A.n3;
    g.st[0] = 1;
    g.st[1] = A.n1;
    g.st[2] = (long)A.n1 * A.n2;
    g.np = g.st[2] * A.n3;
    g.h[0] = A.h1;
    g.h[1] = A.h2;
    g.h[2] = A.h3;
    return g;
}

// h (D_k x)(p) along direction k for the point with coordinate c[k] on its line
template <typename T, int ORD>
__device__ __forceinline__ T d1_at(gcp<T> x, const Geo3& g, long p, const int* c, int k) {
    return d1_line<T, ORD>(x + (p - (long)c[k] * g.st[k]), g.st[k], c[k], g.n[k]);
}

// volume terms of L x at point p (coordinates c); fl: the nine fluxes F_ij of x
template <typename T, int ORD>
__device__ __forceinline__ void volume3(const Args3& A, const Geo3& g, gcp<T> x, gcp<T> fl, long p, const int* c,
                                        T r[3]) {
    gcp<T> cf = gc<T>(A.coef);
    const long np = g.np;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const long l0 = p - (long)c[i] * g.st[i];     // start of the line along i
        const T s = T(1.0 / (g.h[i] * g.h[i]));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T acc = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l)
                acc += d2_line<T, ORD>(cf + (long)fN(i, j, l) * np + l0, x + (long)l * np + l0, g.st[i], c[i], g.n[i]);
            r[j] += acc * s;
        }
    }
    // mixed terms: sum_i D_i F_ij with the fluxes of this lane's field
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            r[j] += d1_at<T, ORD>(fl + (long)(3 * i + j) * np, g, p, c, i) * T(1.0 / g.h[i]);
}

// index along face f of the point with coordinates c (the lower tangential direction fast)
__device__ __forceinline__ int face_t(int a, const int* c, const Geo3& g) {
    const int t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
    return c[t1] + g.n[t1] * c[t2];
}

// displacement-type delta at the face point q (coordinates cq) of face f
template <typename T, bool DATA>
__device__ __forceinline__ void delta3(const Args3& A, const Geo3& g, gcp<T> x, int f, long q, const int* cq,
                                       double tau, T d[3]) {
    if (!DATA) {
#pragma unroll
        for (int l = 0; l < 3; ++l) d[l] = x[(long)l * g.np + q];
        return;
    }
    const Face3& F = A.face[f];
    const int t = face_t(f >> 1, cq, g);
    gcp<T> gg = gc<T>(F.g);
#pragma unroll
    for (int l = 0; l < 3; ++l) d[l] = gg ? static_cast<T>(-tau * (double)gg[(long)l * F.nf + t]) : T(0);
}

// SAT contribution of face f to r at point p (coordinates c, distance dn from the face)
template <typename T, int ORD, bool DATA>
__device__ __forceinline__ void face3(const Args3& A, const Geo3& g, gcp<T> x, int f, long p, const int* c, int dn, double tau, T r[3]) {
    using O = Op<ORD>;
    const Face3& F = A.face[f];
    const int a = f >> 1;
    const T nu = (f & 1) ? T(1) : T(-1);
    gcp<T> cf = gc<T>(A.coef);
    const long np = g.np;
    const T iw = T(1.0 / F.w);
    if (F.kind == BC_TRACTION) {
        if (dn != 0) return;
        if (DATA) {
            if (!F.g) return;
            gcp<T> gg = gc<T>(F.g);
            const int t = face_t(a, c, g);
#pragma unroll
            for (int j = 0; j < 3; ++j) r[j] += static_cast<T>(tau * (double)gg[(long)j * F.nf + t]);
            return;
        }
        T du[3][3];     // h-scaled D_k u_l at the face point, [k][l]
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int l = 0; l < 3; ++l) du[k][l] = d1_at<T, ORD>(x + (long)l * np, g, p, c, k) * T(1.0 / g.h[k]);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T tr = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    const int fld = k == a ? fN(a, j, l) : fM(a, k, j, l);
                    tr += cf[(long)fld * np + p] * du[k][l];
                }
            r[j] -= iw * nu * tr;
        }
        return;
    }
    // displacement face
    if (DATA && !F.g) return;
    int cq[3] = {c[0], c[1], c[2]};
    cq[a] = (f & 1) ? g.n[a] - 1 : 0;
    const long q = p + (long)(cq[a] - c[a]) * g.st[a];
    T d[3];
    delta3<T, DATA>(A, g, x, f, q, cq, tau, d);
    if (dn < O::REACH) {
        const double hn = hnorm<ORD>(dn, g.n[a]);
        const T cfn = static_cast<T>(-O::d1b(0, dn) / (g.h[a] * g.h[a] * hn));
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T s = 0;
#pragma unroll
            for (int l = 0; l < 3; ++l) s += cf[(long)fN(a, l, j) * np + q] * d[l];
            r[j] += cfn * s;
        }
    }
    if (dn != 0) return;
    // tangential parts: (1/w) (H_t^{-1} D_t^T H_t qv)(t), qv_j = nu c_altj delta_l
    for (int tt = 0; tt < 3; ++tt) {
        if (tt == a) continue;
        auto qv = [&](long qq, const int* cc, T out[3]) {
            T e[3];
            delta3<T, DATA>(A, g, x, f, qq, cc, tau, e);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T s = 0;
#pragma unroll
                for (int l = 0; l < 3; ++l) s += cf[(long)fM(a, tt, l, j) * np + qq] * e[l];
                out[j] = nu * s;
            }
        };
        T q0[3];
        qv(q, cq, q0);
        T dq[3] = {0, 0, 0};
        int cc[3] = {cq[0], cq[1], cq[2]};
        d1_foreach<ORD>(cq[tt], g.n[tt], [&](int k2, double w) {
            cc[tt] = k2;
            const long qq = q + (long)(k2 - cq[tt]) * g.st[tt];
            T qk[3];
            qv(qq, cc, qk);
#pragma unroll
            for (int j = 0; j < 3; ++j) dq[j] += static_cast<T>(w) * (qk[j] - q0[j]);
        });
        const T iht = T(1.0 / g.h[tt]);
        const int nt = g.n[tt];
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T s = -dq[j] * iht;
            if (cq[tt] == 0) s -= q0[j] * T(1.0 / (g.h[tt] * hnorm<ORD>(0, nt)));
            if (cq[tt] == nt - 1) s += q0[j] * T(1.0 / (g.h[tt] * hnorm<ORD>(nt - 1, nt)));
            r[j] += iw * s;
        }
    }
    // penalty
    const T pen = static_cast<T>(A.beta * 3.0) * iw * iw;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T s = 0;
#pragma unroll
        for (int l = 0; l < 3; ++l) s += cf[(long)fN(a, j, l) * np + q] * d[l];
        r[j] -= pen * s;
    }
}

template <typename T, int ORD, bool DATA>
__device__ __forceinline__ void sats3(const Args3& A, const Geo3& g, gcp<T> x, long p, const int* c, const double* tw,
                                      T r[3]) {
    using O = Op<ORD>;
    for (int f = 0; f < 6; ++f) {
        const int a = f >> 1;
        const int dn = (f & 1) ? g.n[a] - 1 - c[a] : c[a];
        if (dn >= O::REACH) continue;
        if (DATA && tw[f] == 0.0) continue;
        face3<T, ORD, DATA>(A, g, x, f, p, c, dn, DATA ? tw[f] : 0.0, r);
    }
}

// data at p with the weighted time values tw (6 faces, then the forcing)
template <typename T, int ORD>
__device__ __forceinline__ void data3(const Args3& A, const Geo3& g, long p, const int* c, const double* tw, T r[3]) {
    sats3<T, ORD, true>(A, g, gcp<T>(nullptr), p, c, tw, r);
    if (A.force && tw[6] != 0.0) {
        gcp<T> Fp = gc<T>(A.force);
#pragma unroll
        for (int j = 0; j < 3; ++j) r[j] += static_cast<T>(tw[6] * (double)Fp[(long)j * g.np + p]);
    }
}

}  // namespace

// input field of lane fld of a pass
__device__ __forceinline__ const void* pass_field(const Args3& A, int fld) {
    return A.pass == PASS_APPLY ? A.in : (A.pass == PASS_RK1 ? (fld ? A.v : A.u) : (fld ? A.a2 : A.a1));
}

__device__ __forceinline__ void point_coords(const Geo3& g, long p, int c[3]) {
    c[2] = (int)(p / g.st[2]);
    const long rem = p - (long)c[2] * g.st[2];
    c[1] = (int)(rem / g.n[0]);
    c[0] = (int)(rem - (long)c[1] * g.n[0]);
}

// Mixed-term fluxes of one field at one point:
// F_ij = sum_{k != i} (1/h_k) sum_l c_ijkl (h D_k x_l), boundary rows of D_k included.
template <typename T, int ORD>
__global__ void __launch_bounds__(256) k_flux3(Args3 A) {
    const Geo3 g = geo3(A);
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    const int fld = (int)(gid & 1);
    const long p = gid >> 1;
    if (p >= g.np || (A.pass == PASS_APPLY && fld)) return;
    int c[3];
    point_coords(g, p, c);
    gcp<T> x = gc<T>(pass_field(A, fld));
    gcp<T> cf = gc<T>(A.coef);
    const long np = g.np;
    T G[3][3];      // (1/h_k) h D_k x_l
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) G[k][l] = d1_at<T, ORD>(x + (long)l * np, g, p, c, k) * T(1.0 / g.h[k]);
    gp<T> fo = gm<T>(A.flux) + (long)fld * 9 * np + p;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T f = 0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                if (k == i) continue;
#pragma unroll
                for (int l = 0; l < 3; ++l) f += cf[(long)fM(i, k, j, l) * np + p] * G[k][l];
            }
            fo[(long)(3 * i + j) * np] = f;
        }
}

// Points at least interior_margin3<ORD>() from every face: only interior rows
// of D1 and D2^FC and no face terms reach them.
template <int ORD>
__host__ __device__ constexpr int interior_margin3() {
    using O = Op<ORD>;
    constexpr int m = O::R0 > O::NB ? O::R0 : O::NB;
    return m > O::REACH ? m : O::REACH;
}

// Pass epilogue of one (point, field) lane: the partner lane of the same point
// holds the other field; L = operator, D = data of this lane's field.
template <typename T>
__device__ __forceinline__ void finish3(const Args3& A, const Geo3& g, long p, int fld, bool valid, const T L[3],
                                        const T D[3]) {
    T oL[3], oD[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        oL[j] = __shfl_xor(L[j], 1);
        oD[j] = __shfl_xor(D[j], 1);
    }
    if (!valid) return;
    const T irho = gc<T>(A.coef)[(long)45 * g.np + p];
    const long np = g.np;
    if (A.pass == PASS_APPLY) {
        if (fld) return;
        gp<T> o = gm<T>(A.out);
#pragma unroll
        for (int j = 0; j < 3; ++j) o[(long)j * np + p] = irho * (L[j] + oD[j]);
        return;
    }
    const T dt = static_cast<T>(A.dt);
    // field 0 (lane 0) and field 1 (lane 1) results
    const T* L0 = fld ? oL : L;
    const T* L1 = fld ? L : oL;
    const T* D0 = fld ? oD : D;
    const T* D1 = fld ? D : oD;
    if (A.pass == PASS_RK1) {
        // lane 0 writes a1 = irho (L u + d(t)), lane 1 a2 = irho (L u + dt/2 L v + d(t + dt/2))
        gp<T> o = gm<T>(fld ? A.a2 : A.a1);
#pragma unroll
        for (int j = 0; j < 3; ++j)
            o[(long)j * np + p] = fld ? irho * (L0[j] + T(0.5) * dt * L1[j] + D1[j]) : irho * (L0[j] + D0[j]);
        return;
    }
    // RK2: lane 0 writes u, lane 1 writes v (all three components)
    gcp<T> A1 = gc<T>(A.a1);
    gcp<T> A2 = gc<T>(A.a2);
    gp<T> uu = gm<T>(A.uo);
    gp<T> vv = gm<T>(A.vo);
    const T dt2 = dt * dt;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        const long q = (long)j * np + p;
        const T a1 = A1[q], a2 = A2[q];
        const T a3 = a2 + T(0.25) * dt2 * irho * L0[j];
        const T a4 = T(2) * a2 - a1 + T(0.5) * dt2 * irho * (L1[j] + D1[j]);
        const T uo = gc<T>(A.u)[q], vo = gc<T>(A.v)[q];
        if (fld == 0) uu[q] = uo + dt * vo + dt2 / T(6) * (a1 + a2 + a3);
        else vv[q] = vo + dt / T(6) * (a1 + T(2) * a2 + T(2) * a3 + a4);
    }
}

// Interior points: D2^FC rows in edge form and interior D1 rows of the fluxes,
// body force only.
template <typename T, int ORD>
__global__ void __launch_bounds__(256) k_point3_int(Args3 A) {
    constexpr int M = interior_margin3<ORD>();
    const Geo3 g = geo3(A);
    const int m1 = g.n[0] - 2 * M, m2 = g.n[1] - 2 * M;
    const long nint = (long)m1 * m2 * (g.n[2] - 2 * M);
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    const int fld = (int)(gid & 1);
    const long q = gid >> 1;
    const bool valid = q < nint;
    const long qq = valid ? q : 0;
    const int c2 = (int)(qq / ((long)m1 * m2));
    const long rem = qq - (long)c2 * m1 * m2;
    const int c1 = (int)(rem / m1), c0 = (int)(rem - (long)c1 * m1);
    const long p = (long)(c0 + M) + (long)(c1 + M) * g.st[1] + (long)(c2 + M) * g.st[2];
    const bool apply = A.pass == PASS_APPLY;
    gcp<T> x = gc<T>(pass_field(A, fld));
    gcp<T> fl = gc<T>(A.flux) + (long)fld * 9 * g.np;
    gcp<T> cf = gc<T>(A.coef);
    const long np = g.np;
    T L[3] = {0, 0, 0}, D[3] = {0, 0, 0};
    if (valid && !(apply && fld)) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const long st = g.st[i];
            const T s2 = T(1.0 / (g.h[i] * g.h[i])), s1 = T(1.0 / g.h[i]);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T acc = 0;
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    acc += d2_interior<T, ORD>(cf + (long)fN(i, j, l) * np + p, x + (long)l * np + p, st);
                gcp<T> f = fl + (long)(3 * i + j) * np + p;
                L[j] += acc * s2 + d1_sym<ORD, T>([&](int o) { return f[(long)o * st]; }) * s1;
            }
        }
    }
    if (valid && !(apply && !fld) && A.force) {
        const double tf = (apply || !fld) ? A.tfa[6] : A.tfb[6];
        gcp<T> Fp = gc<T>(A.force);
        if (tf != 0.0) {
#pragma unroll
            for (int j = 0; j < 3; ++j) D[j] = static_cast<T>(tf * (double)Fp[(long)j * np + p]);
        }
    }
    finish3<T>(A, g, p, fld, valid, L, D);
}

// Slab of axis AX: points within M of a face x_AX = 0 or 1 and at least M
// from the faces of the other two axes.  Only the rows along AX are closure
// rows and only the faces of AX reach them.
template <typename T, int ORD, int AX>
__global__ void __launch_bounds__(256) k_point3_slab(Args3 A) {
    using O = Op<ORD>;
    constexpr int M = interior_margin3<ORD>();
    constexpr int B1 = AX == 0 ? 1 : 0, B2 = AX == 2 ? 1 : 2;   // the other two axes, B1 fastest
    const Geo3 g = geo3(A);
    const int mb1 = g.n[B1] - 2 * M, mb2 = g.n[B2] - 2 * M;
    const long per = (long)mb1 * mb2;
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    const int fld = (int)(gid & 1);
    const long q = gid >> 1;
    const bool valid = q < 2 * M * per;
    const long qq = valid ? q : 0;
    int c[3];
    if (AX == 0) {
        // x1 layers fastest, so that neighbouring lanes read neighbouring addresses
        const int layer = (int)(qq % (2 * M));
        const long rem = qq / (2 * M);
        c[0] = layer < M ? layer : g.n[0] - 2 * M + layer;
        c[2] = M + (int)(rem / mb1);
        c[1] = M + (int)(rem - (long)(c[2] - M) * mb1);
    } else {
        const int layer = (int)(qq / per);
        const long rem = qq - (long)layer * per;
        c[AX] = layer < M ? layer : g.n[AX] - 2 * M + layer;
        c[B2] = M + (int)(rem / mb1);
        c[B1] = M + (int)(rem - (long)(c[B2] - M) * mb1);
    }
    const long p = (long)c[0] + (long)c[1] * g.st[1] + (long)c[2] * g.st[2];
    const bool apply = A.pass == PASS_APPLY;
    gcp<T> x = gc<T>(pass_field(A, fld));
    gcp<T> fl = gc<T>(A.flux) + (long)fld * 9 * g.np;
    gcp<T> cf = gc<T>(A.coef);
    const long np = g.np;
    // the face of AX within reach, if any
    const int hi = c[AX] >= M ? 1 : 0;
    const int dn = hi ? g.n[AX] - 1 - c[AX] : c[AX];
    const int f = 2 * AX + hi;
    T L[3] = {0, 0, 0}, D[3] = {0, 0, 0};
    if (valid && !(apply && fld)) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const long st = g.st[i];
            const T s2 = T(1.0 / (g.h[i] * g.h[i])), s1 = T(1.0 / g.h[i]);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T acc = 0, mx;
                gcp<T> fj = fl + (long)(3 * i + j) * np;
                if (i == AX) {
                    const long l0 = p - (long)c[i] * st;
#pragma unroll
                    for (int l = 0; l < 3; ++l)
                        acc += d2_line<T, ORD>(cf + (long)fN(i, j, l) * np + l0, x + (long)l * np + l0, st, c[i], g.n[i]);
                    mx = d1_at<T, ORD>(fj, g, p, c, i);
                } else {
#pragma unroll
                    for (int l = 0; l < 3; ++l)
                        acc += d2_interior<T, ORD>(cf + (long)fN(i, j, l) * np + p, x + (long)l * np + p, st);
                    mx = d1_sym<ORD, T>([&](int o) { return fj[p + (long)o * st]; });
                }
                L[j] += acc * s2 + mx * s1;
            }
        }
        if (dn < O::REACH) face3<T, ORD, false>(A, g, x, f, p, c, dn, 0.0, L);
    }
    if (valid && !(apply && !fld)) {
        const double* tw = (apply || !fld) ? A.tfa : A.tfb;
        if (dn < O::REACH && tw[f] != 0.0) face3<T, ORD, true>(A, g, gcp<T>(nullptr), f, p, c, dn, tw[f], D);
        if (A.force && tw[6] != 0.0) {
            gcp<T> Fp = gc<T>(A.force);
#pragma unroll
            for (int j = 0; j < 3; ++j) D[j] += static_cast<T>(tw[6] * (double)Fp[(long)j * np + p]);
        }
    }
    finish3<T>(A, g, p, fld, valid, L, D);
}

// Coordinate of index l of the 2M boundary layers of an axis of n points.
__device__ __forceinline__ int layer_coord(int l, int n, int M) { return l < M ? l : n - 2 * M + l; }

// The points near the faces of two or three axes (edges and corners), or all
// points when the block has no interior box: every row boundary-aware, face
// terms and data.
template <typename T, int ORD>
__global__ void __launch_bounds__(256) k_point3(Args3 A) {
    constexpr int M = interior_margin3<ORD>();
    const Geo3 g = geo3(A);
    const bool box = g.n[0] > 2 * M && g.n[1] > 2 * M && g.n[2] > 2 * M;
    constexpr long L2 = 4L * M * M;       // (2M)^2 layer pairs
    const long nb0 = box ? L2 * (g.n[0] - 2 * M) : 0, nb1 = box ? L2 * (g.n[1] - 2 * M) : 0,
               nb2 = box ? L2 * (g.n[2] - 2 * M) : 0;
    const long nedge = box ? nb0 + nb1 + nb2 + 2L * M * L2 : g.np;
    const long gid = (long)blockIdx.x * 256 + threadIdx.x;
    const int fld = (int)(gid & 1);                 // field of this lane
    const long q = gid >> 1;
    const bool valid = q < nedge;
    long k = valid ? q : 0;
    int c[3];
    if (!box) {
        c[2] = (int)(k / g.st[2]);
        const long rem = k - (long)c[2] * g.st[2];
        c[1] = (int)(rem / g.n[0]);
        c[0] = (int)(rem - (long)c[1] * g.n[0]);
    } else {
        // bars along x1, x2, x3 (interior coordinate along the bar, boundary
        // layers on the other two axes), then the corners
        int a = 3;
        if (k < nb0) {
            a = 0;
        } else if (k < nb0 + nb1) {
            a = 1;
            k -= nb0;
        } else if (k < nb0 + nb1 + nb2) {
            a = 2;
            k -= nb0 + nb1;
        } else {
            k -= nb0 + nb1 + nb2;
        }
        // the x1 coordinate varies fastest in every part
        if (a == 0) {
            const int ma = g.n[0] - 2 * M;
            const int l = (int)(k / ma);
            c[0] = M + (int)(k - (long)l * ma);
            c[1] = layer_coord(l % (2 * M), g.n[1], M);
            c[2] = layer_coord(l / (2 * M), g.n[2], M);
        } else if (a == 1) {
            const int m1 = g.n[1] - 2 * M;
            const long r = k / (2 * M);
            c[0] = layer_coord((int)(k - r * 2 * M), g.n[0], M);
            c[1] = M + (int)(r % m1);
            c[2] = layer_coord((int)(r / m1), g.n[2], M);
        } else if (a == 2) {
            const long r = k / (2 * M);
            c[0] = layer_coord((int)(k - r * 2 * M), g.n[0], M);
            c[1] = layer_coord((int)(r % (2 * M)), g.n[1], M);
            c[2] = M + (int)(r / (2 * M));
        } else {
            // corner: boundary layers on all three axes
            const int l = (int)k;
            c[0] = layer_coord(l % (2 * M), g.n[0], M);
            c[1] = layer_coord((l / (2 * M)) % (2 * M), g.n[1], M);
            c[2] = layer_coord(l / (4 * M * M), g.n[2], M);
        }
    }
    const long p = (long)c[0] + (long)c[1] * g.st[1] + (long)c[2] * g.st[2];
    const bool apply = A.pass == PASS_APPLY;
    // input field of this lane and its fluxes
    gcp<T> x = gc<T>(pass_field(A, fld));
    gcp<T> fl = gc<T>(A.flux) + (long)fld * 9 * g.np;
    T L[3] = {0, 0, 0}, D[3] = {0, 0, 0};
    if (valid && !(apply && fld)) {
        volume3<T, ORD>(A, g, x, fl, p, c, L);
        sats3<T, ORD, false>(A, g, x, p, c, nullptr, L);
    }
    // data: lane 0 with the first weights, lane 1 with the second (sbpe_apply: lane 1 with the first)
    if (valid) {
        const double* tw = (apply || !fld) ? A.tfa : A.tfb;
        if (!(apply && !fld)) data3<T, ORD>(A, g, p, c, tw, D);
    }
    finish3<T>(A, g, p, fld, valid, L, D);
}

template <typename T, int ORD>
static int launch_point3_t(const Args3& a, hipStream_t s, hipStream_t side, hipEvent_t fork, hipEvent_t join) {
    constexpr int M = interior_margin3<ORD>();
    const long np = (long)a.n1 * a.n2 * a.n3;
    const bool box = a.n1 > 2 * M && a.n2 > 2 * M && a.n3 > 2 * M;
    const dim3 b(256);
    auto grid = [](long pts) { return dim3((unsigned)((2 * pts + 255) / 256)); };
    hipLaunchKernelGGL((k_flux3<T, ORD>), grid(np), b, 0, s, a);
    if (!box) {
        hipLaunchKernelGGL((k_point3<T, ORD>), grid(np), b, 0, s, a);
        return (int)hipGetLastError();
    }
    // the edge and corner points (few, each a long chain) beside the rest
    const long m[3] = {a.n1 - 2 * M, a.n2 - 2 * M, a.n3 - 2 * M};
    const long edges = 4L * M * M * (m[0] + m[1] + m[2]) + 8L * M * M * M;
    hipError_t e = hipEventRecord(fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, fork, 0);
    if (e != hipSuccess) return (int)e;
    hipLaunchKernelGGL((k_point3<T, ORD>), grid(edges), b, 0, side, a);
    hipLaunchKernelGGL((k_point3_int<T, ORD>), grid(m[0] * m[1] * m[2]), b, 0, s, a);
    hipLaunchKernelGGL((k_point3_slab<T, ORD, 0>), grid(2L * M * m[1] * m[2]), b, 0, s, a);
    hipLaunchKernelGGL((k_point3_slab<T, ORD, 1>), grid(2L * M * m[0] * m[2]), b, 0, s, a);
    hipLaunchKernelGGL((k_point3_slab<T, ORD, 2>), grid(2L * M * m[0] * m[1]), b, 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return (int)e;
    e = hipEventRecord(join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, join, 0);
    return (int)e;
}

int launch_point3(int dtype, int order, const Args3& a, void* stream, void* side, void* fork, void* join) {
    hipStream_t s = static_cast<hipStream_t>(stream), sd = static_cast<hipStream_t>(side);
    hipEvent_t f = static_cast<hipEvent_t>(fork), j = static_cast<hipEvent_t>(join);
    if (dtype == 0) return order == 4 ? launch_point3_t<double, 4>(a, s, sd, f, j) : launch_point3_t<double, 2>(a, s, sd, f, j);
    return order == 4 ? launch_point3_t<float, 4>(a, s, sd, f, j) : launch_point3_t<float, 2>(a, s, sd, f, j);
}

}  // namespace sbpe
