/*
 * sbpe3.h -- C ABI of the 3-D path of the library: the same scheme on one
 * curvilinear 3-D block (d = 3).  The paper states every operator for a
 * general dimension (Sec. 3-5); its experiments are 2-D.
 *
 *   - The block is the image of the reference cube [0,1]^3 with n1 x n2 x n3
 *     points, x_a = i_a / (n_a - 1).  Grid functions are row-major
 *     [n3][n2][n1] (x1 fastest); vector fields are three such arrays back to
 *     back ([3][n3][n2][n1], Cartesian components 1, 2, 3).
 *   - Metric (Sec. 3.2-3.3): dX/dx with the SBP first derivative, J = det,
 *     F = (dX/dx)^{-1}; face scale factor Jhat = |a_t1 x a_t2| (Sec. 3.2.2,
 *     eq. surfint_J); c_ijkl = F_Ii J C_IjKl F_Kk, rho~ = J rho.
 *   - Operator DD_ik(c_ijkl) with D_ii^FC(c_ijil) for i = k and D_i c_ijkl D_k
 *     otherwise (Sec. 4.6-4.7); traction SATs (Sec. 5.1) and displacement SATs
 *     with d = 3 in the penalty (Sec. 5.2; Sec. 4.5, eq. borrowing_nd_H_global);
 *     classical RK4 in the two sweeps of the 2-D path (Sec. 7.1).
 *   - Faces 0..5: x1 = 0, x1 = 1, x2 = 0, x2 = 1, x3 = 0, x3 = 1.  A face
 *     array has the two tangential directions in increasing order, the lower
 *     one fastest ([3][nf], nf the product of the two tangential sizes).
 *   - Device operands are caller-owned [3][n3][n2][n1] arrays of the context
 *     dtype, accessed on the context stream in enqueue order.
 *   - Every call returns SBPE_OK or a negative sbpe_status (sbpe.h), validates
 *     its arguments on the host first, and leaves a message for
 *     sbpe3_last_error on failure.  Device memory of the context (46
 *     coefficient fields, face data, forcing, RK workspace of 6 fields and
 *     18 fields of mixed-term fluxes, D_i c_ijkl D_k evaluated as D_i of the
 *     flux sum_kl c_ijkl D_k u_l) is allocated at sbpe3_finalize and freed by
 *     sbpe3_destroy.
 *   - Orders 2 and 4; FP64 and FP32; one block per context; traction and
 *     displacement faces (no Robin, interface, source or receiver terms).
 */
#ifndef SBPE3_H
#define SBPE3_H

#include "sbpe.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbpe3_ctx* sbpe3_ctx_t;

/* A 3-D context on HIP device `device` and stream `stream` (NULL: the null
 * stream); dtype SBPE_F64 or SBPE_F32, order 2 or 4, penalty factor beta >= 1
 * (1 in the paper's experiments). */
sbpe_status sbpe3_create(int device, void* stream, int dtype, int order, double beta, sbpe3_ctx_t* out);
sbpe_status sbpe3_destroy(sbpe3_ctx_t ctx);
const char* sbpe3_last_error(sbpe3_ctx_t ctx);

/* The block: grid X1, X2, X3 and density rho ([n3][n2][n1] host arrays),
 * stiffness C [81][n3][n2][n1] with component (I, J, K, L) at index
 * ((I*3 + J)*3 + K)*3 + L, major symmetric and positive semidefinite as a
 * 9 x 9 matrix (checked at finalize: SBPE_ENOT_PSD).  Copied.  Each n_a is at
 * least 6 (order 2) or 13 (order 4). */
sbpe_status sbpe3_set_block(sbpe3_ctx_t ctx, int n1, int n2, int n3, const double* X1, const double* X2,
                            const double* X3, const double* rho, const double* C81);

/* Face condition: SBPE_BC_TRACTION (Sec. 5.1, data g = traction n C grad u)
 * or SBPE_BC_DISPLACEMENT (Sec. 5.2, data g = displacement), with data
 * g [3][nf] times one time function (SBPE_TIME_*, parameters as in
 * sbpe_set_bc_data), or g = NULL for homogeneous data.  Copied. */
sbpe_status sbpe3_set_bc(sbpe3_ctx_t ctx, int face, int bc, const double* g, int time_fn, const double* time_params);

/* Body force f = F(X) tau(t): F [3][n3][n2][n1] (NULL: none).  Copied. */
sbpe_status sbpe3_set_forcing(sbpe3_ctx_t ctx, const double* F, int time_fn, const double* time_params);

/* Metric, coefficients, checks (SBPE_ENONPOS_J, SBPE_ENOT_PSD), device data. */
sbpe_status sbpe3_finalize(sbpe3_ctx_t ctx);

/* Largest stable RK4 step estimate cfl * min h / v_max, v_max^2 the largest
 * eigenvalue of rho~^{-1} xi_i c_ijkl xi_k over the block and 2000 directions
 * (the time-step rule of Sec. 7).  Host only. */
sbpe_status sbpe3_dt_cfl(sbpe3_ctx_t ctx, double cfl, double* dt);

/* a = rho~^{-1} (DD u + J SAT(u) + J f(t)) for the device field u (data at
 * time t unless homogeneous != 0, then every datum and the forcing are
 * zero); a must not alias u. */
sbpe_status sbpe3_apply(sbpe3_ctx_t ctx, const void* u, void* a, double t, int homogeneous);

/* Bind caller-owned device state u, v = u_t at time t; sbpe3_advance updates
 * them in place with nsteps classical RK4 steps of size dt. */
sbpe_status sbpe3_bind_state(sbpe3_ctx_t ctx, void* u, void* v, double t);
sbpe_status sbpe3_advance(sbpe3_ctx_t ctx, int nsteps, double dt);
sbpe_status sbpe3_get_time(sbpe3_ctx_t ctx, double* t);
/* Wait for every launch of the context (host blocks). */
sbpe_status sbpe3_synchronize(sbpe3_ctx_t ctx);

#ifdef __cplusplus
}
#endif

#endif /* SBPE3_H */
