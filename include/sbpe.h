/*
 * sbpe.h -- C ABI of the MI355X (gfx950) SBP-SAT anisotropic elastic wave library.
 *
 * The library evaluates the right-hand side of the semidiscrete scheme of
 * Almquist & Dunham, "Elastic wave propagation in anisotropic solids using
 * energy-stable finite differences with weakly enforced boundary and interface
 * conditions" (arXiv 2003.12811):
 *
 *     rho u_tt = D^Omega(C) u + f + SAT                      (Sec. 5, eq. semidiscrete_general)
 *
 * on curvilinear multiblock 2-D grids, with the narrow fully compatible
 * operator DD_ik(c_ijkl) (Sec. 4.6-4.7), Robin/traction SATs (Sec. 5.1,
 * eq. sat_traction), displacement SATs (Sec. 5.2, eq. dirichlet_ansatz,
 * Theorem 2) and interface SATs (Sec. 6, eq. scheme_interface), and advances it
 * with classical fourth-order Runge-Kutta (Sec. 7.1).
 *
 * Conventions used by every call:
 *   - A block is the image of the reference square [0,1]^2 with n1 x n2 grid
 *     points, x1 = i/(n1-1), x2 = j/(n2-1).  Grid functions are row-major
 *     [n2][n1] (x1 fastest); vector fields are two such arrays back to back
 *     ([2][n2][n1], Cartesian components u_1 then u_2).
 *   - Host arrays are read during the call (or at sbpe_finalize for arrays
 *     registered with sbpe_add_block / sbpe_set_bc_data / sbpe_set_forcing,
 *     which are copied at the call itself); the caller keeps ownership.
 *   - Device pointers (for example torch tensor data_ptr() values) are owned by
 *     the caller, must hold n1*n2*2 elements of the context dtype, and are
 *     accessed on the context stream in enqueue order; the call returns before
 *     the GPU work completes unless stated otherwise.
 *   - Every call returns SBPE_OK (0) or a negative sbpe_status; arguments are
 *     validated on the host before anything is enqueued, and a failed call
 *     leaves the context unchanged.  sbpe_last_error() gives a message.
 *   - A context is used from one host thread at a time.
 */
#ifndef SBPE_H
#define SBPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sbpe_ctx* sbpe_ctx_t;
typedef int32_t sbpe_status;

enum {
    SBPE_OK = 0,
    SBPE_EINVAL = -1,      /* invalid argument */
    SBPE_ENONPOS_J = -2,   /* discrete Jacobian J <= 0 somewhere (Sec. 3.3) */
    SBPE_ENOT_PSD = -3,    /* stiffness not major-symmetric positive semidefinite (Sec. 3, eq. definite_phys) */
    SBPE_EIFACE = -4,      /* faces of an interface are not conforming (Sec. 6) */
    SBPE_ENOMEM = -5,      /* device allocation failed */
    SBPE_EHIP = -6,        /* HIP runtime error */
    SBPE_EUNSTABLE = -7,   /* energy guard tripped: discrete energy grew or became non-finite */
    SBPE_ESTATE = -8       /* call not valid in the current context state */
};

enum { SBPE_F64 = 0, SBPE_F32 = 1 };                 /* storage and arithmetic precision */
enum { SBPE_FACE_X1LO = 0, SBPE_FACE_X1HI = 1, SBPE_FACE_X2LO = 2, SBPE_FACE_X2HI = 3 };
enum { SBPE_BC_TRACTION = 0, SBPE_BC_ROBIN = 1, SBPE_BC_DISPLACEMENT = 2, SBPE_BC_INTERFACE = 3 };
/* time functions tau(t) multiplying separable data g(x) tau(t):
 *   ZERO: 0;  ONE: 1;  COS: cos(p0 t + p1);  RICKER: (1 - 2 a) exp(-a), a = (pi p0 (t - p1))^2
 *   (Ricker wavelet with peak frequency p0 centred at p1, Sec. 7.4). */
enum { SBPE_TIME_ZERO = 0, SBPE_TIME_ONE = 1, SBPE_TIME_COS = 2, SBPE_TIME_RICKER = 3 };

/* Create a context bound to HIP device `device` and stream `stream` (NULL = the
 * default stream).  dtype: SBPE_F64 or SBPE_F32.  order: 2, 4 or 6 (interior
 * order of the SBP operators, Sec. 4; the paper's three orders, Sec. 7.1).
 * Order 6 supports every call except the wide-stencil operator and the
 * coefficient gradient (SBPE_EINVAL).  beta >= 1 scales the displacement and
 * interface penalties (Theorem 2; the paper uses beta = 1).  device = -1 makes
 * a host-only context: setup and the sbpe_host_* / sbpe_get_* queries work,
 * every call that needs a GPU returns SBPE_ESTATE. */
sbpe_status sbpe_create(int device, void* stream, int dtype, int order, double beta, sbpe_ctx_t* out);

/* Free all device memory owned by the context (after synchronising its
 * stream).  A context that is a member of a batch is refused with
 * SBPE_ESTATE and left intact: remove it with sbpe_batch_remove first (the
 * batch's descriptors point at its fields and its sweeps may still run). */
sbpe_status sbpe_destroy(sbpe_ctx_t ctx);

/* Message of the last failed call on this context (never NULL; static storage
 * for ctx == NULL). */
const char* sbpe_last_error(sbpe_ctx_t ctx);

/* Add a block (Sec. 3.2): physical grid coordinates X1, X2, density rho (all
 * [n2][n1]) and stiffness C10 ([10][n2][n1]: the major-symmetric components
 * C1111, C1112, C1121, C1122, C1212, C1221, C1222, C2121, C2122, C2222; minor
 * symmetry is not assumed, Sec. 3).  Arrays are copied.  All faces start as
 * homogeneous traction.  n1, n2 >= 19 for order 6, >= 13 for order 4, >= 6
 * for order 2, and
 * n1 n2 <= 2^28 (SBPE_EINVAL otherwise, before the arrays are read). */
sbpe_status sbpe_add_block(sbpe_ctx_t ctx, int n1, int n2, const double* X1, const double* X2,
                           const double* rho, const double* C10, int* block_id);

/* Convert Voigt stiffness (c11, c12, c16, c22, c26, c66 per point, [6][npts],
 * no factor 2, index 6 <-> 12) of a normal material to the C10 layout. */
sbpe_status sbpe_voigt_to_c10(const double* voigt, size_t npts, double* C10);

/* Output rows per interior tile, a launch-shape parameter (results do not
 * depend on it): 0 (default) = 10, or order + 1 on small grids (fewer than
 * 384 default tiles and 384 frame groups), else 1..256.  Which height runs fastest
 * depends on the grid and dtype through how the tiles fill the machine; the
 * benchmark picks it by timing a few candidates.  Call before sbpe_finalize
 * (SBPE_ESTATE after it; SBPE_EINVAL outside 0..256).  The environment
 * variable SBPE_TILE_ROWS overrides it. */
sbpe_status sbpe_set_tile_rows(sbpe_ctx_t ctx, int rows);

/* Frame groups per frame workgroup of a one-launch sweep (another launch-shape
 * parameter; results do not depend on it): 1 .. 64, default 2 (FP64) or 4
 * (FP32), 1 on small grids (as for sbpe_set_tile_rows); a group is 16 frame
 * points (8 with the wide operator).  May be
 * called at any time; it applies to the context's own sweeps (batches use the
 * default of their dtype).  SBPE_EINVAL outside 1..64. */
sbpe_status sbpe_set_frame_loop(sbpe_ctx_t ctx, int groups);

/* Second-derivative operator of the i = k terms DD_ii(c) of the elastic
 * operator (Sec. 4.6): SBPE_OP_NARROW (default) the adapted fully compatible
 * narrow-stencil D2^FC(c) of Sec. 4.1; SBPE_OP_WIDE the wide-stencil D_i c D_i
 * (the first derivative applied twice), the operator the narrow one is
 * compared with in Sec. 7.1, with the same SATs.  Call before sbpe_finalize
 * (SBPE_ESTATE after it; SBPE_EINVAL for another value).  Every other entry
 * point works with either operator; the members of one batch share it. */
enum { SBPE_OP_NARROW = 0, SBPE_OP_WIDE = 1 };
sbpe_status sbpe_set_operator(sbpe_ctx_t ctx, int op);

/* Boundary condition of a face (Sec. 5): traction, Robin (U: [2][2][nf]
 * symmetric positive semidefinite U_JL at the face points, row-major JL;
 * required for Robin, ignored otherwise) or displacement.  Interfaces are made
 * with sbpe_connect. */
sbpe_status sbpe_set_bc(sbpe_ctx_t ctx, int block, int face, int bc, const double* U);

/* Dissipative Robin term (the remark after eq. sat_traction, Sec. 5.1): the
 * condition of a traction or Robin face becomes T u + U u + V u_t = g, imposed
 * by adding V u_t to the Robin SAT; the discrete energy then decays at the rate
 * sum over the face of Jhat H_f u_t.V u_t.  V: [2][2][nf] symmetric positive
 * semidefinite at the face points (row-major JL), copied; NULL removes it.
 * SBPE_ESTATE unless the face is traction or Robin; SBPE_EINVAL for a V that
 * is not PSD.  The term acts on the velocity, so it enters sbpe_advance and
 * batches (the stage velocities of RK4) but not sbpe_apply, which evaluates
 * the right-hand side at zero velocity; sbpe_grad_accumulate rejects a context
 * with dissipative faces (the scheme is no longer self-adjoint); at most 16
 * blocks (SBPE_EINVAL at finalize otherwise). */
sbpe_status sbpe_set_bc_dissipation(sbpe_ctx_t ctx, int block, int face, const double* V);

/* Separable boundary data g_J(x) tau(t) of a face: g [2][nf] (traction data for
 * traction/Robin faces, boundary displacement for displacement faces), copied. */
sbpe_status sbpe_set_bc_data(sbpe_ctx_t ctx, int block, int face, const double* g,
                             int time_fn, const double* time_params);

/* Conforming interface between face faceA of block blkA and face faceB of block
 * blkB (Sec. 6, eq. scheme_interface); reversed != 0 when the two faces run in
 * opposite directions.  Both faces need the same number of points. */
sbpe_status sbpe_connect(sbpe_ctx_t ctx, int blkA, int faceA, int blkB, int faceB, int reversed);

/* Separable jump data of an interface (Sec. 6, eq. interface_phys and
 * eq. scheme_interface): across the interface at face `face` of `block`,
 *   u(this block) - u(partner) = V_J(x) tau(t)   (displacement jump),
 *   tau(this block) + tau(partner) = Theta_J(x) tau(t)   (traction jump),
 * with V, Theta [2][nf] in this face's point order (either may be NULL for
 * zero) and one time function for both (SBPE_TIME_*).  The data are copied and
 * apply to both sides of the interface; call after sbpe_connect and before
 * sbpe_finalize.  Returns SBPE_ESTATE if the face is not an interface. */
sbpe_status sbpe_set_interface_data(sbpe_ctx_t ctx, int block, int face, const double* V, const double* Theta,
                                    int time_fn, const double* time_params);

/* Separable body force f_J(x) tau(t) of a block: F [2][n2][n1], copied. */
sbpe_status sbpe_set_forcing(sbpe_ctx_t ctx, int block, const double* F, int time_fn,
                             const double* time_params);

/* Point force f = (f1, f2) amp W(t) delta(X - X(x0)) at reference position
 * (x1, x2) in [0,1]^2 with Ricker time function W of peak frequency peak_hz
 * centred at t0 (Sec. 7.4).  The discrete delta uses four-point moment-matching
 * weights per direction (exact for cubics). */
sbpe_status sbpe_add_source(sbpe_ctx_t ctx, int block, double x1, double x2, double f1, double f2,
                            double amp, double peak_hz, double t0);

/* Receivers at reference positions (x1[k], x2[k]); they record
 * sum_p w_p u(p) with the source weights after every RK4 step. */
sbpe_status sbpe_add_receivers(sbpe_ctx_t ctx, int block, int n, const double* x1, const double* x2);

/* Compute metric terms (Sec. 3.3: F from D1 of the scheme's order, J, Jhat,
 * Nanson normals), the transformed stiffness c = F J C F and rho~ = J rho
 * (eq. transf_density_stiffness), checks (J > 0, symmetry and PSD of C), build
 * launch plans and upload everything to the device. */
sbpe_status sbpe_finalize(sbpe_ctx_t ctx);

/* Largest stable time step estimate dt = cfl * min h / v_max with v_max from
 * the Christoffel matrix of (rho~, c) maximised over directions (Sec. 7). */
sbpe_status sbpe_dt_cfl(sbpe_ctx_t ctx, double cfl, double* dt);

/* Grid size of a block. */
sbpe_status sbpe_block_size(sbpe_ctx_t ctx, int block, int* n1, int* n2);

/* One right-hand-side evaluation on the device: for every block b,
 * a[b] = rho~^{-1} (DD(c) u + J f(t) + J SAT(u, t)), i.e. the acceleration of
 * the semidiscrete scheme.  homogeneous != 0 drops all data, forcing and
 * sources (the operator D^tot of Sec. 5.3 scaled by rho^{-1}).  u[b], a[b] are
 * device pointers of 2*n1*n2 elements; a must not alias any u. */
sbpe_status sbpe_apply(sbpe_ctx_t ctx, const void* const* u, void* const* a, double t, int homogeneous);

/* Bind caller-owned device state buffers u[b], v[b] (displacement and
 * velocity, 2*n1*n2 elements each) and set the current time.  The buffers are
 * read and written in place by sbpe_advance and must stay valid while bound. */
sbpe_status sbpe_bind_state(sbpe_ctx_t ctx, void* const* u, void* const* v, double t);

/* Advance the bound state by nsteps classical RK4 steps of size dt (Sec. 7.1). */
sbpe_status sbpe_advance(sbpe_ctx_t ctx, int nsteps, double dt);

/* Size the per-call tables of sbpe_advance ahead of time: the time-function
 * table for calls of up to nsteps steps and the receiver record for nsteps
 * more steps after those already recorded.  An sbpe_advance call that fits
 * then allocates nothing and does not synchronise the stream (only what does
 * not fit is grown, with an allocation and a stream synchronisation).
 * SBPE_EINVAL for nsteps < 0, SBPE_ENOMEM if the device memory is not there. */
sbpe_status sbpe_reserve_steps(sbpe_ctx_t ctx, int nsteps);

/* sbpe_advance that allocates nothing, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  The time functions of the call are tabulated into
 * a device scratch array of the library, 1 MiB per GPU, held from the first
 * sbpe_create on that GPU until the process ends; at most
 * floor(131072 / (3 * nitems)) steps fit one call, where nitems is 9 per
 * block plus one per source (SBPE_EINVAL beyond that, with the limit in the
 * message).  The receiver record must already hold nsteps more steps
 * (sbpe_reserve_steps; SBPE_ESTATE otherwise).  Results equal those of
 * sbpe_advance bit for bit.  Every context on one GPU shares the scratch
 * array: calls that overlap in time on one GPU (contexts on different
 * streams, or host threads) race and must be serialised by the caller. */
sbpe_status sbpe_advance_noalloc(sbpe_ctx_t ctx, int nsteps, double dt);

/* Device memory from the caller.  Every device allocation of the context
 * (coefficient fields, RK workspace, face data, frame operator, tables,
 * receiver record) is then alloc(bytes, user), and is given back with
 * release(ptr, user); the context keeps no hipMalloc'ed memory of its own
 * (the no-allocation advance's scratch array aside).  alloc returns device
 * memory of the context's device aligned to 256 bytes, or NULL (the call
 * that needed it then fails with SBPE_ENOMEM).  Before release the context
 * waits for its streams, so the memory may be reused at once, on any stream.
 * Both callbacks run on the thread that makes the library call.  Set them
 * before sbpe_finalize, before the context allocates anything (SBPE_ESTATE
 * otherwise); both NULL restores hipMalloc/hipFree.  For callers whose memory
 * comes from a framework's allocator (PyTorch's caching allocator: retiring
 * a context then returns its memory without a device-wide hipFree). */
typedef void* (*sbpe_alloc_fn)(size_t bytes, void* user);
typedef void (*sbpe_release_fn)(void* ptr, void* user);
sbpe_status sbpe_set_allocator(sbpe_ctx_t ctx, sbpe_alloc_fn alloc, sbpe_release_fn release, void* user);

/* Device memory of the context: *held = bytes it holds now (coefficient
 * fields, RK workspace, face data, frame operator, tables, receiver record),
 * *peak = the most it has held at once (finalize's probing buffers
 * included).  Caller-owned state buffers are not counted.  Either pointer
 * may be NULL. */
sbpe_status sbpe_device_bytes(sbpe_ctx_t ctx, long long* held, long long* peak);

/* Current time of the bound state. */
sbpe_status sbpe_get_time(sbpe_ctx_t ctx, double* t);

/* Copy receiver traces recorded since the last sbpe_bind_state into out
 * ([nsteps][nrec][2], FP64, host), at most max_steps steps; synchronises.
 * With out == NULL only *nsteps_out (the number of steps available, capped at
 * max_steps) is returned. */
sbpe_status sbpe_read_receivers(sbpe_ctx_t ctx, double* out, int max_steps, int* nsteps_out);

/* Discrete energy eps = 1/2 (v^T P H v - u^T A u), A = diag(JH) D^tot, of the
 * bound state (Sec. 5 and 7.2), accumulated in FP64; synchronises. */
sbpe_status sbpe_energy(sbpe_ctx_t ctx, double* eps);

/* Energy guard: every `every` steps sbpe_advance computes the energy and fails
 * with SBPE_EUNSTABLE if it is not finite or exceeds (1 + rel_growth) times the
 * energy at the start of the call.  every = 0 disables it (default). */
sbpe_status sbpe_set_energy_guard(sbpe_ctx_t ctx, int every, double rel_growth);

/* Wait for all work enqueued on the context stream. */
sbpe_status sbpe_synchronize(sbpe_ctx_t ctx);

/* Kernel timing for measurement: while enabled, every kernel launch of
 * sbpe_advance and sbpe_apply is bracketed by HIP events on the context stream.
 * sbpe_get_kernel_timing synchronises and returns, for the six launch kinds
 * (interior, frame) x (first RK4 sweep, second RK4 sweep, apply), the average
 * duration in milliseconds (ms_avg[6]) and the number of launches (count[6]),
 * then clears the accumulators. */
sbpe_status sbpe_set_kernel_timing(sbpe_ctx_t ctx, int enable);
sbpe_status sbpe_get_kernel_timing(sbpe_ctx_t ctx, double* ms_avg, int* count);

/* Launch plan after sbpe_finalize (info holds 6 entries): info[0] = interior
 * points, info[1] = frame points (summed over blocks), info[2] = interior
 * workgroups, info[3] = frame workgroups, info[4] = frame width in points,
 * info[5] = 1 when each sweep is a single launch that also updates the frame
 * points (then the kernel timing reports it as the interior kind and the frame
 * kinds stay empty), 0 when frame and interior are separate launches. */
sbpe_status sbpe_plan_info(sbpe_ctx_t ctx, long long* info);

/* ---------------------------------------------------------------- gradients
 * Building blocks of the discrete adjoint of a receiver misfit with respect
 * to rho and C.  H L is symmetric (the energy analysis of Sec. 5 and 6), so
 * with the adjoint variables scaled as zhat = z / (H rho~) the adjoint state
 * is advanced with the forward operator itself (sbpe_apply, homogeneous).
 * Either operator (sbpe_set_operator) is supported; blocks with interface
 * faces and contexts with dissipative faces are not (SBPE_EINVAL). */

/* For every block b, accumulate the gradient of one RK4 stage:
 *   gc[b]  += alpha * d/dc (z^T H L(c) y)   (10 stored transformed-stiffness
 *             fields, FP64 device [10][n2][n1], order c1111, c1112, c1212,
 *             c2121, c2122, c2222, c1121, c1122, c1221, c1222; Sec. 4.7, 5),
 *   grt[b] += -alpha * H * (z . a)          (FP64 device [n2][n1], gradient
 *             with respect to rho~ = J rho).
 * z, y, a are device fields of the context dtype, [2][n2][n1]: the scaled
 * stage adjoint, the stage displacement and the stage value
 * a = rho~^{-1} (L y + data(t)).  Unless homogeneous, displacement data at
 * time t enter delta = y - g(t).  H holds the quadrature weights
 * h1 h2 H1_i H2_j.  Enqueued on the context stream. */
sbpe_status sbpe_grad_accumulate(sbpe_ctx_t ctx, const void* const* z, const void* const* y, const void* const* a,
                                 double alpha, double t, int homogeneous, void* const* gc, void* const* grt);

/* The four stages of one classical RK4 step (Sec. 7.1) in one call: stage s =
 * 0..3 at time t + c_s dt, c = (0, 1/2, 1/2, 1), accumulates as
 * sbpe_grad_accumulate with z[s*nb + b], y[s*nb + b], a[s*nb + b] and
 * alpha[s] (nb = number of blocks; alpha: 4 host values).  The stages are
 * summed before they are added to gc and grt, so results equal four single
 * calls up to rounding.  Band partial sums go to a context buffer of
 * 4 * 11 * (points within the closure width of a face) FP64 values, allocated
 * on the first call and kept (the allocation synchronises the stream).
 * Errors as sbpe_grad_accumulate. */
sbpe_status sbpe_grad_accumulate_rk4(sbpe_ctx_t ctx, const void* const* z, const void* const* y,
                                     const void* const* a, const double* alpha, double t, double dt,
                                     int homogeneous, void* const* gc, void* const* grt);

/* Device pointers to the RK4 stage slopes of block `block` in the context's
 * workspace ([2][n2][n1] each, context dtype, owned by the context): after
 * sbpe_advance, *a1 = rho~^{-1} (L u + data(t)) and *a2 = rho~^{-1}
 * (L (u + dt/2 v) + data(t + dt/2)) of its last step, evaluated at that
 * step's initial state (u, v).  Valid until the next call on the context that
 * sweeps (sbpe_advance, batches) or evaluates the energy.  The discrete adjoint
 * rebuilds the stage displacements u + dt/2 v + dt^2/4 a1 and
 * u + dt v + dt^2/2 a2 from them.  SBPE_ESTATE before sbpe_finalize. */
sbpe_status sbpe_stage_slopes(sbpe_ctx_t ctx, int block, void** a1, void** a2);

/* Chain rule of one block to the physical parameters, c = F J C F and
 * rho~ = J rho (Sec. 3.2.1): gc, grt device arrays as above; g_c10 host
 * [10][n2][n1] in the C10 order of sbpe_add_block (C treated as major
 * symmetric), g_rho host [n2][n1].  Synchronises. */
sbpe_status sbpe_grad_to_physical(sbpe_ctx_t ctx, int block, const void* gc, const void* grt, double* g_c10,
                                  double* g_rho);

/* y = sum_k coefs[k] x[k] elementwise over count values of the context dtype
 * (device pointers, 1 <= nterms <= 6, y may be one of the x[k]); the sums are
 * formed in FP64. */
sbpe_status sbpe_lincomb(sbpe_ctx_t ctx, int nterms, const double* coefs, const void* const* x, void* y,
                         long long count);

/* Stage values of one classical RK4 step (Sec. 7.1) of u'' = a(u), rebuilt
 * elementwise over count values of the context dtype (device pointers) from
 * the state (u0, v0) at t, the state (u1, v1) at t + dt and the first two
 * stage slopes a1, a2 (sbpe_stage_slopes):
 *   out[0] U2 = u0 + dt/2 v0,   out[1] U3 = U2 + dt^2/4 a1,
 *   out[2] U4 = u0 + dt v0 + dt^2/2 a2,   out[3] = a1,   out[4] = a2,
 *   out[5] a3 = 6 (u1 - u0 - dt v0) / dt^2 - a1 - a2,
 *   out[6] a4 = 6 (v1 - v0) / dt - a1 - 2 a2 - 2 a3,
 * the last two solved from the step's update u1 = u0 + dt v0 + dt^2/6 (a1 +
 * a2 + a3), v1 = v0 + dt/6 (a1 + 2 a2 + 2 a3 + a4).  Arithmetic in FP64; the
 * difference u1 - u0 - dt v0 is of size dt^2 a, so a3 carries a relative
 * rounding error of about 6 eps / (omega dt)^2 for a solution of angular
 * frequency omega (1e-13 in FP64 for the differentiation workload's step).
 * out: 7 pointers, NULL entries are not written; u1, v1 may be NULL when
 * out[5] and out[6] are.  SBPE_EINVAL for dt <= 0 or a missing input. */
sbpe_status sbpe_rk4_stages(sbpe_ctx_t ctx, const void* u0, const void* v0, const void* u1, const void* v1,
                            const void* a1, const void* a2, double dt, void* const* out, long long count);

/* u[b] += scale * (H rho~)^{-1} S^T r, the adjoint of the receiver sampling
 * (Sec. 7.4) in the scaled variables: r is FP64 device [nrec][2] in the order
 * of sbpe_add_receivers, u the device displacement fields of every block. */
sbpe_status sbpe_receiver_adjoint(sbpe_ctx_t ctx, const void* r, void* const* u, double scale);

/* ------------------------------------------------------------------ batches
 * Continuous batching of independent solves (many contexts, e.g. one shot
 * each).  A batch advances the bound states of its members with one kernel
 * launch per RK4 sweep over the union of their blocks, each member with its
 * own time step, sources and receivers.  The arithmetic per block is exactly
 * that of sbpe_advance, so a member's result does not depend on which other
 * members share the launch.  Members join and leave between calls to
 * sbpe_batch_advance; the caller decides admission (for example by an HBM
 * budget).  All members must use the batch's device, dtype, order and operator.  A
 * batch is driven from one host thread.
 *
 * Errors: SBPE_EINVAL for bad arguments, SBPE_ESTATE when a context is not
 * finalized with a bound state or already belongs to a batch, SBPE_ENOMEM,
 * SBPE_EHIP; the message is returned by sbpe_batch_last_error(batch). */
typedef struct sbpe_batch* sbpe_batch_t;

/* Create a batch whose work is enqueued on hip_stream of hip_device. */
sbpe_status sbpe_batch_create(int hip_device, void* hip_stream, int dtype, int order, sbpe_batch_t* out);
sbpe_status sbpe_batch_destroy(sbpe_batch_t batch);
const char* sbpe_batch_last_error(sbpe_batch_t batch);

/* Admit a finalized context with a bound state for nsteps RK4 steps of size
 * dt starting at its current time.  Its time functions for all nsteps steps
 * are tabulated and its receiver buffer is sized here.  While it is a member,
 * sbpe_advance, sbpe_apply and sbpe_bind_state on it fail with SBPE_ESTATE.
 * The members of a batch share device, dtype, order and operator
 * (sbpe_set_operator; the first member of an empty batch sets it): a context
 * that differs is refused with SBPE_EINVAL, and so is a context finalized
 * without the assembled frame operator (more than 16 blocks, or the
 * environment variable SBPE_FRAME=stencil at sbpe_finalize, which runs the
 * frame band of its own sweeps with the stencil kernel instead). */
sbpe_status sbpe_batch_add(sbpe_batch_t batch, sbpe_ctx_t ctx, int nsteps, double dt);

/* Remove a member (normally once its remaining step count is 0).  Work later
 * enqueued on the context's own stream (sbpe_read_receivers, copies of the
 * state) is ordered after the batch's work. */
sbpe_status sbpe_batch_remove(sbpe_batch_t batch, sbpe_ctx_t ctx);

/* Advance every member by nsteps steps; nsteps must not exceed any member's
 * remaining step count. */
sbpe_status sbpe_batch_advance(sbpe_batch_t batch, int nsteps);

/* Remaining steps of a member; number of members, smallest remaining step
 * count and total grid points of all members. */
sbpe_status sbpe_batch_remaining(sbpe_batch_t batch, sbpe_ctx_t ctx, int* remaining);
sbpe_status sbpe_batch_info(sbpe_batch_t batch, int* members, int* min_remaining, long long* points);

/* Wait for all work enqueued by the batch. */
sbpe_status sbpe_batch_synchronize(sbpe_batch_t batch);

/* ---------------------------------------------------------------- host-side
 * Queries of the library's own setup, for checking it on a machine without a
 * GPU.  They run on the host only. */

/* The adapted fully compatible D2^FC(b) (Sec. 4.1) and D1 of the library
 * applied to one grid line of n points with h = 1/(n-1): out = D2^FC(b) u and
 * out = D1 u. */
sbpe_status sbpe_host_d2fc_line(int order, int n, const double* b, const double* u, double* out);
sbpe_status sbpe_host_d1_line(int order, int n, const double* u, double* out);

/* After sbpe_finalize: transformed stiffness of a block in the C10 layout
 * ([10][n2][n1]), J ([n2][n1]) and the surface scale factor of each face
 * (Jhat, [4][max(n1,n2)], face f uses its first n2 (f < 2) or n1 entries). */
sbpe_status sbpe_get_block_fields(sbpe_ctx_t ctx, int block, double* c10, double* J, double* jhat);

#ifdef __cplusplus
}
#endif

#endif /* SBPE_H */
