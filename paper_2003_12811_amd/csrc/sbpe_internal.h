// Device-side descriptors shared by the host setup (sbpe_host.cpp) and the
// kernels (sbpe_kernels.hip).  Plain structs of pointers and sizes; every
// pointer is device memory owned by the context (coefficients, workspace) or
// by the caller (bound state, sbpe_apply operands).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sbpe {

enum { BC_TRACTION = 0, BC_ROBIN = 1, BC_DISPLACEMENT = 2, BC_INTERFACE = 3 };
enum { TF_ZERO = 0, TF_ONE = 1, TF_COS = 2, TF_RICKER = 3 };
// kernel passes
//   APPLY: out = rho~^-1 (L in + data(t))
//   RK1  : a1 = rho~^-1 (L u + data(t)),  a2 = rho~^-1 (L u + dt/2 L v + data(t + dt/2))
//   RK2  : with A1 = a1, A2 = a2 (stages 1, 2 of classical RK4 on (u, u_t)),
//          A3 = A2 + dt^2/4 rho~^-1 L A1,
//          A4 = 2 A2 - A1 + dt^2/2 rho~^-1 (L A2 + 2/dt^2 (data(t) - 2 data(t + dt/2) + data(t + dt))),
//          u += dt v + dt^2/6 (A1 + A2 + A3),  v += dt/6 (A1 + 2 A2 + 2 A3 + A4)
// L is linear and data(t) is affine in the time functions, so these are the
// four stages of classical RK4 regrouped into two sweeps over the grid.
enum { PASS_APPLY = 0, PASS_RK1 = 1, PASS_RK2 = 2 };
// which bound field a device routine reads
enum { FLD_U = 0, FLD_V = 1, FLD_A1 = 2, FLD_A2 = 3, FLD_IN = 4 };

// coefficient field order in the per-block coefficient array [NCOEF][n2][n1]
enum {
    K_C1111 = 0, K_C1112 = 1, K_C1212 = 2,   // x1 narrow second derivative
    K_C2121 = 3, K_C2122 = 4, K_C2222 = 5,   // x2 narrow second derivative
    K_C1121 = 6, K_C1122 = 7, K_C1221 = 8, K_C1222 = 9,  // mixed terms
    K_IRHO = 10,                              // 1 / (J rho)
    NCOEF = 11
};

struct TimeFn {
    int kind;
    int pad;
    double p[2];
};

struct FaceDesc {
    int kind;          // BC_*
    int partner;       // interface: index of the partner block in the descriptor table
    int pface;         // interface: partner face
    int reversed;      // interface: faces run in opposite directions
    int nf;            // number of face points
    int pad;
    double w;          // first norm weight of the face-normal direction, h_a * H^_0
    double pw;         // interface: the partner's first norm weight
    double vsign;      // interface: +1 on the side that owns the jump data order, -1 on the other
    int item_g;        // time-function item of g
    int item_v;        // time-function item of the interface jump data
    const void* g;     // [2][nf]: traction/Robin: Jhat g / w; displacement: g; or null
    const void* U;     // [4][nf]: Robin Jhat U_JL / w (row-major JL), or null
    const void* V;     // [2][nf] displacement jump in this face's order (interface), or null
    const void* Th;    // [2][nf] Jhat Theta / (2 w) in this face's order (interface), or null
    const void* Dv;    // [4][nf] Jhat V_JL / w of a dissipative Robin term V u_t (row-major JL), or null
};

struct Entry;
struct Range;

struct BlockDesc {
    int n1, n2;
    double h1, h2;
    const void* coef;   // [NCOEF][n2][n1]
    const void* force;  // [2][n2][n1] J f space part, or null
    int item_f;         // time-function item of the forcing
    int pad_f;
    void* u;            // bound displacement [2][n2][n1]
    void* v;            // bound velocity
    void* a1;           // RK workspace
    void* a2;
    FaceDesc face[4];
    int tiles_x, tiles_y, tile_beg;     // interior launch geometry
    int tile_y, pad_t;                  // output rows per interior tile
    int frame_n, frame_wg, frame_beg;   // frame launch geometry (points, workgroups, first workgroup)
    // per-context data of a sweep (a launch may cover blocks of several contexts)
    double dt;                // RK time step
    double beta;              // penalty factor
    const double* tau;        // tabulated time functions [steps][nitems][3]
    int nitems;               // items per tabulated step
    int step0;                // launch step index at which tau row 0 (and receiver row 0) applies
    const Entry* entries;     // point entries of the context
    const Range* tile_rng;    // entry ranges of this block's interior tiles (index wg - tile_beg)
    const Range* frame_rng;   // entry ranges of this block's frame workgroups (index wg - frame_beg)
    double* rec;              // receiver slots [steps][nrec*16][2], or null
    long rec_stride;          // doubles per step in rec
    // assembled frame operator rho~^{-1} L restricted to the frame rows (null
    // until assembled), in 2x2 blocks: frame point k holds the blocks
    // fr_rowptr[k] .. fr_rowptr[k + 1] - 1, one per neighbouring point; block
    // e's column is p (point p of this block) or -1 - ((f << 29) | p) (point p
    // of the interface partner across face f), its values K[q][q'] (output
    // component q, input component q') are fr_val[4 e + 2 q + q']
    const int* fr_rowptr;
    const int* fr_col;
    const void* fr_val;       // [4 blocks] in the context dtype
    const void* fr_rsum;      // [2 frame_n][2] row sums per input component
};

// frame point k of a block -> grid point (i, j): the R rows along x2 = 0, the
// R rows along x2 = 1 (row by row), then the side bands column by column
// (R columns at each x1 face, rows R .. n2-1-R)
inline __host__ __device__ void frame_ij(int k, int n1, int n2, int R, int& i, int& j) {
    if (k < R * n1) {
        j = k / n1;
        i = k - j * n1;
    } else if (k < 2 * R * n1) {
        const int kk = k - R * n1;
        j = n2 - R + kk / n1;
        i = kk % n1;
    } else {
        const int kk = k - 2 * R * n1;
        const int cc = kk / (n2 - 2 * R), row = kk - cc * (n2 - 2 * R);
        j = R + row;
        i = cc < R ? cc : n1 - 2 * R + cc;
    }
}

// point entries: sources add to the right-hand side, receivers record u
struct Entry {
    int p;        // flat grid index in its block
    int kind;     // 0 source, 1 receiver
    int id;       // source: its time-function item; receiver: rec * 16 + slot
    int pad;
    double c0, c1;  // source: amp dir_J w / H (J f contribution); receiver: weight, unused
};

// Point entries of one workgroup: sources in [beg, mid), receivers in
// [mid, end), each run sorted by point.
struct Range {
    int beg, mid, end, pad;
};

// Time functions are tabulated per RK4 step by k_tau: tau[(step * nitems + item) * 3 + k]
// = tau_item(t_step + c_k dt), c = (0, 1/2, 1).  Items: per block 9 (face g x4,
// face jump data x4, forcing), then one per source.
constexpr int ITEMS_PER_BLOCK = 9;

constexpr int MAX_APPLY_BLOCKS = 16;

struct PassArgs {
    const BlockDesc* blocks;
    int nblocks;
    int pass;
    int homogeneous;
    int total_tiles;                    // interior workgroups over all blocks
    int total_frame_wg;                 // frame point groups (FRAME_PTS points each) over all blocks
    int step;                           // launch step index (time-function row step - step0)
    int rec_base;                       // receiver row of launch step index 0
    int wide;                           // 1: wide-stencil operator D_i c D_i for the i = k terms
    int floop;                          // one-launch sweeps: frame groups per frame workgroup (>= 1)
    double wa[3], wb[3];                // weights of the tabulated values: first / second evaluation
                                        // (second sweep: wb multiplies 2/dt^2 of each block)
    const void* in[MAX_APPLY_BLOCKS];   // sbpe_apply operands per block
    void* out[MAX_APPLY_BLOCKS];
};

// interior tile: one wave spanning 64 columns writes the central
// 64 - 2 * half-width of them and marches over tile_y rows
constexpr int TILE_LANES = 64;
constexpr int TILE_Y_DEFAULT = 10;
constexpr int FRAME_WG = 256;
constexpr int FRAME_PTS = 32;   // frame points per group (the unit of the point-entry ranges)

// Coefficient gradient of RK4 stages (sbpe_grad_accumulate: one stage;
// sbpe_grad_accumulate_rk4: the four stages of a step): for every block and
// stage s, gc[b][k] += alpha[s] d/dc_k (z_s^T H L(c) y_s) and
// grt[b] += -alpha[s] H (z_s . a_s).
constexpr int GRAD_STAGES_MAX = 4;
constexpr int GRAD_TERMS = 11;        // 10 coefficient fields and rho~
struct GradArgs {
    const BlockDesc* blocks;
    int nblocks;
    int nstages;          // 1 .. GRAD_STAGES_MAX
    int homogeneous;      // displacement data left out of delta = y - g(t)
    int wide;             // wide-stencil operator: the i = k terms are D_i c D_i
    int n1[MAX_APPLY_BLOCKS], n2[MAX_APPLY_BLOCKS];   // block sizes
    long off[MAX_APPLY_BLOCKS + 1];   // first interior point of each block (interior launch; set by the launcher)
    long boff[MAX_APPLY_BLOCKS + 1];  // first band point of each block (band launch; set by the launcher)
    long nband;                       // band points of all blocks (set by the launcher)
    double alpha[GRAD_STAGES_MAX];
    int tcol[GRAD_STAGES_MAX];        // column of row 0 of the time-function table holding stage s's time
    const double* tau;    // tabulated time functions: row 0 = tau(t), tau(t + dt/2), tau(t + dt)
    const void* z[GRAD_STAGES_MAX][MAX_APPLY_BLOCKS];
    const void* y[GRAD_STAGES_MAX][MAX_APPLY_BLOCKS];
    const void* a[GRAD_STAGES_MAX][MAX_APPLY_BLOCKS];
    double* gc[MAX_APPLY_BLOCKS];     // [10][n2][n1], the stored coefficient order K_C1111 .. K_C1222
    double* grt[MAX_APPLY_BLOCKS];    // [n2][n1], gradient with respect to rho~ = J rho
    double* part;         // nstages > 1: band partial sums [nstages][GRAD_TERMS][band points]
};

// host-side launchers (sbpe_kernels.hip)
int launch_interior(int dtype, int order, const PassArgs& a, int total_tiles, void* stream);
int launch_frame(int dtype, int order, const PassArgs& a, int total_frame_wg, void* stream);
int launch_tau(const TimeFn* items, int nitems, int nsteps, double t0, double dt, double* tau, void* stream);
int launch_energy(int dtype, int order, const BlockDesc* blocks_dev, int nblocks, double* partial_dev,
                  int npartial, double* result_dev, void* stream);
int launch_grad(int dtype, int order, const GradArgs& g, void* stream);
// band points of the gradient launches (the partial sums of a multi-stage launch)
long grad_band_points(int order, const int* n1, const int* n2, int nblocks);
// frame operator assembly: probe fill, compaction of frame outputs, sparse frame kernel
int launch_probe_fill(int dtype, void* x, int n1, int n2, int comp, int cx, int cy, int period, void* stream);
int launch_frame_gather(int dtype, const void* y, int n1, int n2, int R, int frame_n, void* out, void* stream);
int launch_frame_sp(int dtype, int order, const PassArgs& a, int total_frame_wg, void* stream);
// one sweep (frame operator and interior tiles) in one launch; sweep_fused
// says whether a grid of that many tiles is swept that way
bool sweep_fused(int total_tiles);
int launch_pass(int dtype, int order, const PassArgs& a, int total_tiles, int total_frame_wg, void* stream);
constexpr int LINCOMB_MAX = 6;   // terms of sbpe_lincomb
int launch_lincomb(int dtype, int nterms, const double* coefs, const void* const* x, void* y, long count,
                   void* stream);
struct Rk4StageArgs {
    const void* u0;
    const void* v0;
    const void* u1;
    const void* v1;
    const void* a1;
    const void* a2;
    void* out[7];       // U2, U3, U4, A1, A2, A3, A4 (null: not written)
    double dt;
};
int launch_rk4_stages(int dtype, const Rk4StageArgs& a, long count, void* stream);
// one interpolation point of one receiver: u[block][c][p] += scale * w * r[rec][c]
struct RecAdj {
    int rec;
    int block;
    long p;
    double w;       // interpolation weight / (H_p rho~_p)
};
struct RecAdjArgs {
    void* u[MAX_APPLY_BLOCKS];
    long np[MAX_APPLY_BLOCKS];
    double scale;
};
int launch_rec_adjoint(int dtype, const RecAdj* ent, int nent, const double* r, const RecAdjArgs& a, void* stream);
const char* hip_error_string(int code);
// device scratch of the no-allocation advance (sbpe_advance_noalloc): doubles
// per GPU, the device address of the array on `device` (looked up once per
// device by scratch_init with that device current; null before)
constexpr size_t NOALLOC_SCRATCH_DOUBLES = size_t(1) << 17;   // 1 MiB
int scratch_init(int device);
double* scratch_ptr(int device);

}  // namespace sbpe
