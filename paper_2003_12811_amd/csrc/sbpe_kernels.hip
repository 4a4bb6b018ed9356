// HIP kernels (gfx950, wave64) of the SBP-SAT anisotropic elastic operator.
//
// One right-hand-side evaluation is split by grid region:
//   * k_interior: points at least Frame<ORD>::R from every face, where all
//     1-D operators use their repeating interior stencils (Sec. 4.3-4.7);
//   * k_frame:    the band of width R along the faces, where the boundary
//     closures of D1 and D2^FC and the SATs of Sec. 5 and 6 act.
// Both are fused with the two-sweep form of classical RK4 described in
// sbpe_internal.h, so one RK4 step reads the coefficient fields twice.
//
// Reference-frame forms used here (all follow from the paper's definitions):
//   * volume: DD_ik(c_ijkl) u_l = D_11^FC(c_1j1l) u_l + D_22^FC(c_2j2l) u_l
//             + D_1 (c_1j2l D_2 u_l) + D_2 (c_2j1l D_1 u_l)   (eq. def_cd, Sec. 4.7)
//   * Jhat T_jl = nu_i c_ijkl D_k                              (eq. n-C_conversion)
//   * Jhat Z_jl = beta d / h_1 nu_i c_ijkl nu_k (displacement; / 4 and summed
//     over both sides at interfaces), from Nanson's formula (eq. nanson)
//   * J (JH)^{-1} e_f Jhat H_f = (1 / h_1) at the face points (H = H_x1 (x) H_x2)
//   * H_t^{-1} D_t^T H_t = -D_t + H_t^{-1} (e_N e_N^T - e_0 e_0^T)  (SBP property, Sec. 4)
#include <hip/hip_runtime.h>

#include "sbpe_internal.h"
#include "sbpe_tables.h"

namespace sbpe {

__constant__ double c_d2c4[O4_R0][O4_W][O4_W];
__constant__ double c_d2c2[O2_R0][O2_W][O2_W];

template <int ORD> struct Op;
template <> struct Op<4> {
    static constexpr int R0 = O4_R0, W = O4_W, NB = O4_NB, HALF = 2, REACH = 4;
    __device__ static double d2c(int r, int m, int s) { return c_d2c4[r][m][s]; }
    __device__ static double d1b(int r, int c) { return O4_D1B[r][c]; }
    __device__ static double d1i(int k) { return O4_D1I[k]; }
    __device__ static double hb(int k) { return O4_H[k]; }
};
template <> struct Op<2> {
    static constexpr int R0 = O2_R0, W = O2_W, NB = O2_NB, HALF = 1, REACH = 2;
    __device__ static double d2c(int r, int m, int s) { return c_d2c2[r][m][s]; }
    __device__ static double d1b(int r, int c) { return O2_D1B[r][c]; }
    __device__ static double d1i(int k) { return O2_D1I[k]; }
    __device__ static double hb(int k) { return O2_H[k]; }
};

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

__device__ __forceinline__ double tcomb(const TimeFn& f, const TimeComb& c) {
    double s = 0.0;
    for (int k = 0; k < c.n; ++k) s += c.w[k] * tfun(f, c.t[k]);
    return s;
}

template <typename T>
__device__ __forceinline__ const T* field_ptr(const PassArgs& A, int b, int fld) {
    const BlockDesc& B = A.blocks[b];
    switch (fld) {
        case FLD_U: return static_cast<const T*>(B.u);
        case FLD_V: return static_cast<const T*>(B.v);
        case FLD_A1: return static_cast<const T*>(B.a1);
        case FLD_A2: return static_cast<const T*>(B.a2);
        default: return static_cast<const T*>(A.in[b]);
    }
}

// ------------------------------------------------------------ 1-D rows
// Row r of D1 on a line of n points: start index, up to 6 weights (times h).
template <int ORD>
__device__ __forceinline__ int d1_entries(int r, int n, int& start, double w[6]) {
    using O = Op<ORD>;
    if (r < O::NB) {
        start = 0;
        for (int c = 0; c < 6; ++c) w[c] = O::d1b(r, c);
        return 6;
    }
    if (r > n - 1 - O::NB) {
        const int rr = n - 1 - r;
        start = n - 6;
        for (int k = 0; k < 6; ++k) w[k] = -O::d1b(rr, 5 - k);
        return 6;
    }
    start = r - O::HALF;
    for (int k = 0; k < 2 * O::HALF + 1; ++k) w[k] = O::d1i(k);
    return 2 * O::HALF + 1;
}

// h (D1 u)_r on a line with element stride `st`
template <typename T, int ORD>
__device__ T d1_line(const T* u, long st, int r, int n) {
    int s0;
    double w[6];
    const int len = d1_entries<ORD>(r, n, s0, w);
    T acc = 0;
    for (int k = 0; k < len; ++k)
        if (w[k] != 0.0) acc += static_cast<T>(w[k]) * u[(long)(s0 + k) * st];
    return acc;
}

// h^2 (D2^FC(b) u)_r at an interior row; b, u point at the row.
template <typename T, int ORD>
__device__ __forceinline__ T d2_interior(const T* b, const T* u, long st) {
    const T u0 = u[0];
    if constexpr (ORD == 4) {
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

// h^2 (D2^FC(b) u)_r on a line of n points; b, u point at index 0 of the line.
template <typename T, int ORD>
__device__ T d2_line(const T* b, const T* u, long st, int r, int n) {
    using O = Op<ORD>;
    if (r >= O::R0 && r <= n - 1 - O::R0) return d2_interior<T, ORD>(b + r * st, u + r * st, st);
    const bool lo = r < O::R0;
    const int rr = lo ? r : n - 1 - r;
    const T ur = u[(long)r * st];
    T acc = 0;
    for (int m = 0; m < O::W; ++m) {
        const long pm = lo ? m : n - 1 - m;
        T cf = 0;
        bool any = false;
        for (int s = 0; s < O::W; ++s) {
            const double tv = O::d2c(rr, m, s);
            if (tv != 0.0) {
                cf += static_cast<T>(tv) * b[(long)(lo ? s : n - 1 - s) * st];
                any = true;
            }
        }
        if (any) acc += cf * (u[pm * st] - ur);
    }
    return acc;
}

// -------------------------------------------------- volume at one point
// DD_ik(c_ijkl) u_l at (i, j) with boundary-aware 1-D rows (frame points).
template <typename T, int ORD>
__device__ void volume_general(const BlockDesc& B, const T* u, int i, int j, T& r0, T& r1) {
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const T* c = static_cast<const T*>(B.coef);
    const T* u0 = u;
    const T* u1 = u + np;
    const T ih1 = T(1.0 / B.h1), ih2 = T(1.0 / B.h2);
    const long rj = (long)j * n1;
    // x1 narrow, line j
    const T a00 = d2_line<T, ORD>(c + K_C1111 * np + rj, u0 + rj, 1, i, n1);
    const T a01 = d2_line<T, ORD>(c + K_C1112 * np + rj, u1 + rj, 1, i, n1);
    const T a10 = d2_line<T, ORD>(c + K_C1112 * np + rj, u0 + rj, 1, i, n1);
    const T a11 = d2_line<T, ORD>(c + K_C1212 * np + rj, u1 + rj, 1, i, n1);
    // x2 narrow, line i
    const T b00 = d2_line<T, ORD>(c + K_C2121 * np + i, u0 + i, n1, j, n2);
    const T b01 = d2_line<T, ORD>(c + K_C2122 * np + i, u1 + i, n1, j, n2);
    const T b10 = d2_line<T, ORD>(c + K_C2122 * np + i, u0 + i, n1, j, n2);
    const T b11 = d2_line<T, ORD>(c + K_C2222 * np + i, u1 + i, n1, j, n2);
    r0 = (a00 + a01) * ih1 * ih1 + (b00 + b01) * ih2 * ih2;
    r1 = (a10 + a11) * ih1 * ih1 + (b10 + b11) * ih2 * ih2;
    // D_1 (M D_2 u), M_jl = c_1j2l
    int s0;
    double w[6];
    int len = d1_entries<ORD>(i, n1, s0, w);
    T g0 = 0, g1 = 0;
    for (int k = 0; k < len; ++k) {
        if (w[k] == 0.0) continue;
        const int ii = s0 + k;
        const T w20 = d1_line<T, ORD>(u0 + ii, n1, j, n2);
        const T w21 = d1_line<T, ORD>(u1 + ii, n1, j, n2);
        const long q = rj + ii;
        const T m00 = c[K_C1121 * np + q], m01 = c[K_C1122 * np + q];
        const T m10 = c[K_C1221 * np + q], m11 = c[K_C1222 * np + q];
        g0 += static_cast<T>(w[k]) * (m00 * w20 + m01 * w21);
        g1 += static_cast<T>(w[k]) * (m10 * w20 + m11 * w21);
    }
    // D_2 (M^T D_1 u), c_2j1l = c_1l2j
    len = d1_entries<ORD>(j, n2, s0, w);
    T e0 = 0, e1 = 0;
    for (int k = 0; k < len; ++k) {
        if (w[k] == 0.0) continue;
        const int jj = s0 + k;
        const long rjj = (long)jj * n1;
        const T w10 = d1_line<T, ORD>(u0 + rjj, 1, i, n1);
        const T w11 = d1_line<T, ORD>(u1 + rjj, 1, i, n1);
        const long q = rjj + i;
        const T m00 = c[K_C1121 * np + q], m01 = c[K_C1122 * np + q];
        const T m10 = c[K_C1221 * np + q], m11 = c[K_C1222 * np + q];
        e0 += static_cast<T>(w[k]) * (m00 * w10 + m10 * w11);
        e1 += static_cast<T>(w[k]) * (m01 * w10 + m11 * w11);
    }
    const T ihh = ih1 * ih2;
    r0 += (g0 + e0) * ihh;
    r1 += (g1 + e1) * ihh;
}

// --------------------------------------------------------- face helpers
struct FacePt {
    int i, j;   // grid point
};

__device__ __forceinline__ FacePt face_point(const BlockDesc& B, int f, int t) {
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
__device__ __forceinline__ void coef_mats(const T* c, long np, long q, int a, T N[2][2], T M[2][2]) {
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
__device__ void traction_at(const BlockDesc& B, const T* u, int f, int t, T& tr0, T& tr1) {
    const int n1 = B.n1, n2 = B.n2;
    const long np = (long)n1 * n2;
    const int a = f >> 1;
    const T nu = (f & 1) ? T(1) : T(-1);
    const FacePt q = face_point(B, f, t);
    const long p = (long)q.j * n1 + q.i;
    const T* c = static_cast<const T*>(B.coef);
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
__device__ __forceinline__ void face_delta(const PassArgs& A, int b, int f, int t, int fld,
                                           const TimeComb& tc, T& d0, T& d1) {
    const BlockDesc& B = A.blocks[b];
    const FaceDesc& F = B.face[f];
    const long np = (long)B.n1 * B.n2;
    if (!DATA) {
        const T* u = field_ptr<T>(A, b, fld);
        const FacePt q = face_point(B, f, t);
        const long p = (long)q.j * B.n1 + q.i;
        d0 = u[p];
        d1 = u[np + p];
        if (F.kind == BC_INTERFACE) {
            const BlockDesc& P = A.blocks[F.partner];
            const T* v = field_ptr<T>(A, F.partner, fld);
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
            const T tau = static_cast<T>(tcomb(F.tf, tc));
            const T* g = static_cast<const T*>(F.g);
            d0 = -tau * g[t];
            d1 = -tau * g[F.nf + t];
        } else if (F.kind == BC_INTERFACE && F.V) {
            const T tau = static_cast<T>(F.vsign * tcomb(F.vtf, tc));
            const T* V = static_cast<const T*>(F.V);
            d0 = -tau * V[t];
            d1 = -tau * V[F.nf + t];
        }
    }
}

// Contribution of face f to r at (i, j) (dn = distance from the face along its
// normal, t = index along the face).  DATA selects the data part (time
// combination tc) instead of the homogeneous part acting on field `fld`.
template <typename T, int ORD, bool DATA>
__device__ void face_sat(const PassArgs& A, int b, int f, int dn, int t, int fld,
                         const TimeComb& tc, T& r0, T& r1) {
    using O = Op<ORD>;
    const BlockDesc& B = A.blocks[b];
    const double beta = A.beta;
    const FaceDesc& F = B.face[f];
    const int a = f >> 1;
    const long np = (long)B.n1 * B.n2;
    const T* c = static_cast<const T*>(B.coef);
    const T nu = (f & 1) ? T(1) : T(-1);
    const double ha = a == 0 ? B.h1 : B.h2;
    const int na = a == 0 ? B.n1 : B.n2;
    const int nt = a == 0 ? B.n2 : B.n1;
    const double ht = a == 0 ? B.h2 : B.h1;
    const T iw = T(1.0 / F.w);

    if (F.kind == BC_TRACTION || F.kind == BC_ROBIN) {
        if (dn != 0) return;
        if (!DATA) {
            const T* u = field_ptr<T>(A, b, fld);
            T tr0, tr1;
            traction_at<T, ORD>(B, u, f, t, tr0, tr1);
            r0 -= iw * tr0;
            r1 -= iw * tr1;
            if (F.kind == BC_ROBIN && F.U) {
                const T* U = static_cast<const T*>(F.U);
                const FacePt q = face_point(B, f, t);
                const long p = (long)q.j * B.n1 + q.i;
                const T x0 = u[p], x1 = u[np + p];
                r0 -= U[t] * x0 + U[F.nf + t] * x1;
                r1 -= U[2 * F.nf + t] * x0 + U[3 * F.nf + t] * x1;
            }
        } else if (F.g) {
            const T tau = static_cast<T>(tcomb(F.tf, tc));
            const T* g = static_cast<const T*>(F.g);
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
        int s0;
        double w[6];
        const int len = d1_entries<ORD>(t, nt, s0, w);
        T dq0 = 0, dq1 = 0, qe0 = 0, qe1 = 0;
        for (int k = 0; k < len; ++k) {
            const int tt = s0 + k;
            const bool endp = (t == 0 && tt == 0) || (t == nt - 1 && tt == nt - 1);
            if (w[k] == 0.0 && !endp) continue;
            T e0, e1;
            face_delta<T, DATA>(A, b, f, tt, fld, tc, e0, e1);
            const FacePt qq = face_point(B, f, tt);
            T Nq[2][2], Mq[2][2];
            coef_mats(c, np, (long)qq.j * B.n1 + qq.i, a, Nq, Mq);
            T q0, q1;
            if (a == 0) {   // c_1l2j = M_lj
                q0 = nu * (Mq[0][0] * e0 + Mq[1][0] * e1);
                q1 = nu * (Mq[0][1] * e0 + Mq[1][1] * e1);
            } else {        // c_2l1j = c_1j2l = M_jl
                q0 = nu * (Mq[0][0] * e0 + Mq[0][1] * e1);
                q1 = nu * (Mq[1][0] * e0 + Mq[1][1] * e1);
            }
            dq0 += static_cast<T>(w[k]) * q0;
            dq1 += static_cast<T>(w[k]) * q1;
            if (tt == t) {
                qe0 = q0;
                qe1 = q1;
            }
        }
        const T iht = T(1.0 / ht);
        T s0v = -dq0 * iht, s1v = -dq1 * iht;
        if (t == 0) {
            const T ih0 = T(1.0 / (ht * hnorm<ORD>(0, nt)));
            s0v -= qe0 * ih0;
            s1v -= qe1 * ih0;
        }
        if (t == nt - 1) {
            const T ihN = T(1.0 / (ht * hnorm<ORD>(nt - 1, nt)));
            s0v += qe0 * ihN;
            s1v += qe1 * ihN;
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
        const BlockDesc& P = A.blocks[F.partner];
        const int tp = F.reversed ? F.nf - 1 - t : t;
        const FacePt qp = face_point(P, F.pface, tp);
        const long npp = (long)P.n1 * P.n2;
        T Np[2][2], Mp[2][2];
        coef_mats(static_cast<const T*>(P.coef), npp, (long)qp.j * P.n1 + qp.i, F.pface >> 1, Np, Mp);
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
            const T tau = static_cast<T>(tcomb(F.vtf, tc));
            const T* Th = static_cast<const T*>(F.Th);
            r0 += tau * Th[t];
            r1 += tau * Th[F.nf + t];
        }
    }
}

// all SAT contributions of the four faces at (i, j)
template <typename T, int ORD, bool DATA>
__device__ void sat_point(const PassArgs& A, int b, int i, int j, int fld, const TimeComb& tc, T& r0, T& r1) {
    using O = Op<ORD>;
    const BlockDesc& B = A.blocks[b];
    const int dist[4] = {i, B.n1 - 1 - i, j, B.n2 - 1 - j};
    for (int f = 0; f < 4; ++f) {
        const int dn = dist[f];
        if (dn >= O::REACH) continue;
        const int t = (f < 2) ? j : i;
        face_sat<T, ORD, DATA>(A, b, f, dn, t, fld, tc, r0, r1);
    }
}

// forcing and sources at flat point p for a time combination
template <typename T>
__device__ __forceinline__ void point_data(const BlockDesc& B, long p, const PassArgs& A, const Range& rg,
                                           const TimeComb& tc, T& r0, T& r1) {
    if (B.force) {
        const T* F = static_cast<const T*>(B.force);
        const T tau = static_cast<T>(tcomb(B.ftf, tc));
        r0 += tau * F[p];
        r1 += tau * F[(long)B.n1 * B.n2 + p];
    }
    for (int e = rg.beg; e < rg.end; ++e) {
        const Entry& E = A.entries[e];
        if (E.kind == 0 && E.p == p) {
            const double tau = tcomb(A.src_tf[E.id], tc);
            r0 += static_cast<T>(E.c0 * tau);
            r1 += static_cast<T>(E.c1 * tau);
        }
    }
}

__device__ __forceinline__ TimeComb comb1(double t, double w) {
    TimeComb c;
    c.n = 1;
    c.pad = 0;
    c.t[0] = t;
    c.w[0] = w;
    c.t[1] = c.t[2] = 0.0;
    c.w[1] = c.w[2] = 0.0;
    return c;
}

// combination 2/dt^2 (tau(t) - 2 tau(t + dt/2) + tau(t + dt)) used by the second sweep
__device__ __forceinline__ TimeComb comb_rk2(double t, double dt) {
    TimeComb c;
    c.n = 3;
    c.pad = 0;
    const double s = 2.0 / (dt * dt);
    c.t[0] = t;
    c.t[1] = t + 0.5 * dt;
    c.t[2] = t + dt;
    c.w[0] = s;
    c.w[1] = -2.0 * s;
    c.w[2] = s;
    return c;
}

// Given L f0 (l0), L f1 (l1) and the data sums of the two evaluations at p,
// write the pass outputs (see the pass definitions in sbpe_internal.h).
template <typename T>
__device__ __forceinline__ void finish_point(const PassArgs& A, int b, long p, T irho,
                                             T l00, T l01, T l10, T l11, T da0, T da1, T db0, T db1,
                                             const Range& rg) {
    const BlockDesc& B = A.blocks[b];
    const long np = (long)B.n1 * B.n2;
    if (A.pass == PASS_APPLY) {
        T* o = static_cast<T*>(A.out[b]);
        o[p] = irho * (l00 + da0);
        o[np + p] = irho * (l01 + da1);
        return;
    }
    const T dt = static_cast<T>(A.dt);
    T* a1 = static_cast<T*>(B.a1);
    T* a2 = static_cast<T*>(B.a2);
    if (A.pass == PASS_RK1) {
        const T hdt = T(0.5) * dt;
        a1[p] = irho * (l00 + da0);
        a1[np + p] = irho * (l01 + da1);
        a2[p] = irho * (l00 + hdt * l10 + db0);
        a2[np + p] = irho * (l01 + hdt * l11 + db1);
        return;
    }
    // PASS_RK2
    T* u = static_cast<T*>(B.u);
    T* v = static_cast<T*>(B.v);
    const T dt2 = dt * dt;
    const T q4 = T(0.25) * dt2, q2 = T(0.5) * dt2, s6 = dt2 / T(6), d6 = dt / T(6);
    T un[2];
    for (int cmp = 0; cmp < 2; ++cmp) {
        const long q = cmp * np + p;
        const T A1 = a1[q], A2 = a2[q];
        const T L1 = cmp ? l01 : l00;
        const T L2 = cmp ? l11 : l10;
        const T D2 = cmp ? db1 : db0;
        const T A3 = A2 + q4 * irho * L1;
        const T A4 = T(2) * A2 - A1 + q2 * irho * (L2 + D2);
        const T uo = u[q], vo = v[q];
        un[cmp] = uo + dt * vo + s6 * (A1 + A2 + A3);
        u[q] = un[cmp];
        v[q] = vo + d6 * (A1 + T(2) * A2 + T(2) * A3 + A4);
    }
    if (A.rec_out) {
        for (int e = rg.beg; e < rg.end; ++e) {
            const Entry& E = A.entries[e];
            if (E.kind == 1 && E.p == p) {
                A.rec_out[2 * E.id] = E.c0 * static_cast<double>(un[0]);
                A.rec_out[2 * E.id + 1] = E.c0 * static_cast<double>(un[1]);
            }
        }
    }
}

__device__ __forceinline__ int find_block(const PassArgs& A, int wg, bool frame) {
    int b = 0;
    for (int k = 1; k < A.nblocks; ++k) {
        const int beg = frame ? A.blocks[k].frame_beg : A.blocks[k].tile_beg;
        if (wg >= beg) b = k;
    }
    return b;
}

// ---------------------------------------------------------------- frame
template <typename T, int ORD>
__global__ void __launch_bounds__(FRAME_WG) k_frame(PassArgs A) {
    constexpr int R = Frame<ORD>::R;
    const int wg = blockIdx.x;
    const int b = find_block(A, wg, true);
    const BlockDesc& B = A.blocks[b];
    const int k = (wg - B.frame_beg) * FRAME_WG + threadIdx.x;
    const Range rg = A.frame_ranges[wg];
    if (k >= B.frame_n) return;
    const int n1 = B.n1, n2 = B.n2;
    int i, j;
    if (k < R * n1) {
        j = k / n1;
        i = k - j * n1;
    } else if (k < 2 * R * n1) {
        const int kk = k - R * n1;
        j = n2 - R + kk / n1;
        i = kk % n1;
    } else {
        const int kk = k - 2 * R * n1;
        const int row = kk / (2 * R), cc = kk % (2 * R);
        j = R + row;
        i = cc < R ? cc : n1 - 2 * R + cc;
    }
    const long p = (long)j * n1 + i;
    const T irho = static_cast<const T*>(B.coef)[(long)K_IRHO * n1 * n2 + p];
    const TimeComb none = comb1(0.0, 0.0);
    int f0, f1;
    TimeComb ca, cb;
    if (A.pass == PASS_APPLY) {
        f0 = FLD_IN;
        f1 = FLD_IN;
        ca = comb1(A.t, A.homogeneous ? 0.0 : 1.0);
        cb = none;
    } else if (A.pass == PASS_RK1) {
        f0 = FLD_U;
        f1 = FLD_V;
        ca = comb1(A.t, 1.0);
        cb = comb1(A.t + 0.5 * A.dt, 1.0);
    } else {
        f0 = FLD_A1;
        f1 = FLD_A2;
        ca = none;
        cb = comb_rk2(A.t, A.dt);
    }
    T l00, l01, l10 = 0, l11 = 0;
    volume_general<T, ORD>(B, field_ptr<T>(A, b, f0), i, j, l00, l01);
    sat_point<T, ORD, false>(A, b, i, j, f0, none, l00, l01);
    if (A.pass != PASS_APPLY) {
        volume_general<T, ORD>(B, field_ptr<T>(A, b, f1), i, j, l10, l11);
        sat_point<T, ORD, false>(A, b, i, j, f1, none, l10, l11);
    }
    T da0 = 0, da1 = 0, db0 = 0, db1 = 0;
    if (ca.w[0] != 0.0) {
        sat_point<T, ORD, true>(A, b, i, j, f0, ca, da0, da1);
        point_data<T>(B, p, A, rg, ca, da0, da1);
    }
    if (A.pass != PASS_APPLY) {
        sat_point<T, ORD, true>(A, b, i, j, f1, cb, db0, db1);
        point_data<T>(B, p, A, rg, cb, db0, db1);
    }
    finish_point<T>(A, b, p, irho, l00, l01, l10, l11, da0, da1, db0, db1, rg);
}

// ------------------------------------------------------------- interior
// Repeating interior stencils only; one thread per point, operands read
// straight from global memory (L1/L2 serve the neighbour reuse).
template <typename T, int ORD>
__device__ __forceinline__ void volume_interior(const BlockDesc& B, const T* u, long p, T& r0, T& r1) {
    using O = Op<ORD>;
    constexpr int HF = O::HALF;
    const int n1 = B.n1;
    const long np = (long)n1 * B.n2;
    const T* c = static_cast<const T*>(B.coef);
    const T* u0 = u;
    const T* u1 = u + np;
    const T ih1 = T(1.0 / B.h1), ih2 = T(1.0 / B.h2);
    const T a00 = d2_interior<T, ORD>(c + K_C1111 * np + p, u0 + p, 1);
    const T a01 = d2_interior<T, ORD>(c + K_C1112 * np + p, u1 + p, 1);
    const T a10 = d2_interior<T, ORD>(c + K_C1112 * np + p, u0 + p, 1);
    const T a11 = d2_interior<T, ORD>(c + K_C1212 * np + p, u1 + p, 1);
    const T b00 = d2_interior<T, ORD>(c + K_C2121 * np + p, u0 + p, n1);
    const T b01 = d2_interior<T, ORD>(c + K_C2122 * np + p, u1 + p, n1);
    const T b10 = d2_interior<T, ORD>(c + K_C2122 * np + p, u0 + p, n1);
    const T b11 = d2_interior<T, ORD>(c + K_C2222 * np + p, u1 + p, n1);
    r0 = (a00 + a01) * ih1 * ih1 + (b00 + b01) * ih2 * ih2;
    r1 = (a10 + a11) * ih1 * ih1 + (b10 + b11) * ih2 * ih2;
    T g0 = 0, g1 = 0, e0 = 0, e1 = 0;
#pragma unroll
    for (int k = -HF; k <= HF; ++k) {
        if (k == 0) continue;
        const T wk = static_cast<T>(O::d1i(k + HF));
        // D_1 (M D_2 u): column p + k
        {
            const long q = p + k;
            T w20 = 0, w21 = 0;
#pragma unroll
            for (int m = -HF; m <= HF; ++m) {
                if (m == 0) continue;
                const T wm = static_cast<T>(O::d1i(m + HF));
                w20 += wm * (u0[q + (long)m * n1] - u0[q]);
                w21 += wm * (u1[q + (long)m * n1] - u1[q]);
            }
            g0 += wk * (c[K_C1121 * np + q] * w20 + c[K_C1122 * np + q] * w21);
            g1 += wk * (c[K_C1221 * np + q] * w20 + c[K_C1222 * np + q] * w21);
        }
        // D_2 (M^T D_1 u): row p + k n1
        {
            const long q = p + (long)k * n1;
            T w10 = 0, w11 = 0;
#pragma unroll
            for (int m = -HF; m <= HF; ++m) {
                if (m == 0) continue;
                const T wm = static_cast<T>(O::d1i(m + HF));
                w10 += wm * (u0[q + m] - u0[q]);
                w11 += wm * (u1[q + m] - u1[q]);
            }
            e0 += wk * (c[K_C1121 * np + q] * w10 + c[K_C1221 * np + q] * w11);
            e1 += wk * (c[K_C1122 * np + q] * w10 + c[K_C1222 * np + q] * w11);
        }
    }
    const T ihh = ih1 * ih2;
    r0 += (g0 + e0) * ihh;
    r1 += (g1 + e1) * ihh;
}

template <typename T, int ORD>
__global__ void __launch_bounds__(TILE_X * TILE_Y) k_interior(PassArgs A) {
    constexpr int R = Frame<ORD>::R;
    const int wg = blockIdx.x;
    const int b = find_block(A, wg, false);
    const BlockDesc& B = A.blocks[b];
    const int tl = wg - B.tile_beg;
    const int ty = tl / B.tiles_x, tx = tl - ty * B.tiles_x;
    const int i = R + tx * TILE_X + (threadIdx.x % TILE_X);
    const int j = R + ty * TILE_Y + (threadIdx.x / TILE_X);
    const Range rg = A.tile_ranges[wg];
    if (i > B.n1 - 1 - R || j > B.n2 - 1 - R) return;
    const long p = (long)j * B.n1 + i;
    const T irho = static_cast<const T*>(B.coef)[(long)K_IRHO * B.n1 * B.n2 + p];
    int f0, f1;
    TimeComb ca, cb;
    const TimeComb none = comb1(0.0, 0.0);
    if (A.pass == PASS_APPLY) {
        f0 = f1 = FLD_IN;
        ca = comb1(A.t, A.homogeneous ? 0.0 : 1.0);
        cb = none;
    } else if (A.pass == PASS_RK1) {
        f0 = FLD_U;
        f1 = FLD_V;
        ca = comb1(A.t, 1.0);
        cb = comb1(A.t + 0.5 * A.dt, 1.0);
    } else {
        f0 = FLD_A1;
        f1 = FLD_A2;
        ca = none;
        cb = comb_rk2(A.t, A.dt);
    }
    T l00, l01, l10 = 0, l11 = 0;
    volume_interior<T, ORD>(B, field_ptr<T>(A, b, f0), p, l00, l01);
    if (A.pass != PASS_APPLY) volume_interior<T, ORD>(B, field_ptr<T>(A, b, f1), p, l10, l11);
    T da0 = 0, da1 = 0, db0 = 0, db1 = 0;
    if (ca.w[0] != 0.0) point_data<T>(B, p, A, rg, ca, da0, da1);
    if (A.pass != PASS_APPLY) point_data<T>(B, p, A, rg, cb, db0, db1);
    finish_point<T>(A, b, p, irho, l00, l01, l10, l11, da0, da1, db0, db1, rg);
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
        const BlockDesc& B = blocks[b];
        const long np = (long)B.n1 * B.n2;
        const T* u = static_cast<const T*>(B.u);
        const T* v = static_cast<const T*>(B.v);
        const T* a = static_cast<const T*>(B.a1);
        const T* c = static_cast<const T*>(B.coef);
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
template <typename T, int ORD>
static int launch_pass_t(const PassArgs& a, int total_tiles, int total_frame_wg, hipStream_t s) {
    if (total_tiles > 0) hipLaunchKernelGGL((k_interior<T, ORD>), dim3(total_tiles), dim3(TILE_X * TILE_Y), 0, s, a);
    if (total_frame_wg > 0) hipLaunchKernelGGL((k_frame<T, ORD>), dim3(total_frame_wg), dim3(FRAME_WG), 0, s, a);
    return static_cast<int>(hipGetLastError());
}

int launch_pass(int dtype, int order, const PassArgs& a, int total_tiles, int total_frame_wg, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == 0) {
        return order == 4 ? launch_pass_t<double, 4>(a, total_tiles, total_frame_wg, s)
                          : launch_pass_t<double, 2>(a, total_tiles, total_frame_wg, s);
    }
    return order == 4 ? launch_pass_t<float, 4>(a, total_tiles, total_frame_wg, s)
                      : launch_pass_t<float, 2>(a, total_tiles, total_frame_wg, s);
}

int launch_energy(int dtype, int order, const BlockDesc* blocks_dev, int nblocks, double* partial_dev,
                  int npartial, double* result_dev, void* stream) {
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dtype == 0) {
        if (order == 4) hipLaunchKernelGGL((k_energy_partial<double, 4>), dim3(npartial), dim3(256), 0, s, blocks_dev, nblocks, partial_dev);
        else hipLaunchKernelGGL((k_energy_partial<double, 2>), dim3(npartial), dim3(256), 0, s, blocks_dev, nblocks, partial_dev);
    } else {
        if (order == 4) hipLaunchKernelGGL((k_energy_partial<float, 4>), dim3(npartial), dim3(256), 0, s, blocks_dev, nblocks, partial_dev);
        else hipLaunchKernelGGL((k_energy_partial<float, 2>), dim3(npartial), dim3(256), 0, s, blocks_dev, nblocks, partial_dev);
    }
    hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(256), 0, s, partial_dev, npartial, result_dev);
    return static_cast<int>(hipGetLastError());
}

int upload_tables(const double* t4, const double* t2) {
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_d2c4), t4, sizeof(double) * O4_R0 * O4_W * O4_W);
    if (e != hipSuccess) return static_cast<int>(e);
    return static_cast<int>(hipMemcpyToSymbol(HIP_SYMBOL(c_d2c2), t2, sizeof(double) * O2_R0 * O2_W * O2_W));
}

const char* hip_error_string(int code) { return hipGetErrorString(static_cast<hipError_t>(code)); }

}  // namespace sbpe
