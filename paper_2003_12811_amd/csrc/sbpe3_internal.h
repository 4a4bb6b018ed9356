// Shared declarations of the 3-D path (sbpe3_kernels.hip and the sbpe3_*
// section of sbpe_host.cpp).
#pragma once

#include "sbpe_internal.h"

namespace sbpe {

// One curvilinear 3-D block (sbpe3_*): grid functions [n3][n2][n1], x1 fastest.
// Coefficients [46][n3][n2][n1]: c_ijil for directions i = 0..2 (6 each, (j, l)
// in the order 00, 01, 02, 11, 12, 22), c_ijkl for i < k (pairs 01, 02, 12;
// 9 each, (j, l) row-major; c_kjil = c_ilkj by major symmetry), then 1/rho~.
constexpr int NCOEF3 = 46;
struct Face3 {
    int kind;           // BC_TRACTION or BC_DISPLACEMENT
    int nf;             // face points (the lower tangential direction fast)
    double w;           // first norm weight of the face-normal direction, h_a H_0
    const void* g;      // [3][nf]: traction Jhat g / w, displacement g; or null
};
struct Args3 {
    int n1, n2, n3;
    int pass;           // PASS_APPLY, PASS_RK1, PASS_RK2 (the two-sweep RK4 of the 2-D path)
    double h1, h2, h3, beta, dt;
    const void* coef;
    const void* force;  // [3][np] J f space part, or null
    Face3 face[6];      // x1 = 0, x1 = 1, x2 = 0, x2 = 1, x3 = 0, x3 = 1
    const void* u;      // RK state (read)
    const void* v;
    void* a1;           // RK workspace
    void* a2;
    void* uo;           // RK2 output state (may be u, v: each point reads only its own state)
    void* vo;
    const void* in;     // sbpe3_apply operand and result
    void* out;
    void* flux;         // [2][9][np] mixed-term fluxes of the pass's two fields (k_flux3)
    double tfa[7], tfb[7];   // weighted time values of the 6 face items and the forcing:
                             // first / second evaluation of the pass
};
// one pass: the mixed-term fluxes (k_flux3), then the interior-box, slab and
// edge point kernels; the edges run on `side` between the events fork and join
int launch_point3(int dtype, int order, const Args3& a, void* stream, void* side, void* fork, void* join);

}  // namespace sbpe
