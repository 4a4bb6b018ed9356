// Host side of the SBP-SAT elastic wave library: context, setup of the metric
// terms and transformed coefficients, launch plans and the C ABI of sbpe.h.
//
// Setup follows Sec. 3.2-3.3 of Almquist & Dunham (arXiv 2003.12811):
//   F^{-1}_{iI} = dX_I/dx_i from D1 of the scheme's order, J = det F^{-1},
//   c_ijkl = F_Ii J C_IjKl F_Kk, rho~ = J rho (eq. transf_density_stiffness),
//   Jhat = |a_t| on each face (eq. surfj_app_2d); J <= 0 is rejected.
// The time step follows Sec. 7: dt = CFL min h / v_max with v_max^2 the largest
// eigenvalue of xi_i c_ijkl xi_k / rho~ maximised over directions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <utility>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/sbpe.h"
#include "../../include/sbpe3.h"
#include "sbpe_internal.h"
#include "sbpe3_internal.h"
#include "sbpe_tables.h"

namespace sbpe {

// ------------------------------------------------------------- 1-D tables
static int nb_of(int order) { return order == 6 ? O6_NB : order == 4 ? O4_NB : O2_NB; }
// closure depth of D2^FC, columns of a D1 closure row, and the frame width
static int r0_of(int order) { return order == 6 ? O6_R0 : order == 4 ? O4_R0 : O2_R0; }
static int frame_of(int order) { return order == 6 ? Frame<6>::R : order == 4 ? Frame<4>::R : Frame<2>::R; }
// fewest points per direction of a block (closures of both ends apart)
static int min_points(int order) { return order == 6 ? 19 : order == 4 ? 13 : 6; }
constexpr int D1W_MAX = 9;

double norm_weight(int order, int n, int k) {
    const int nb = nb_of(order);
    const double* H = order == 6 ? O6_H : order == 4 ? O4_H : O2_H;
    if (k < nb) return H[k];
    if (k > n - 1 - nb) return H[n - 1 - k];
    return 1.0;
}

// closure row r of the dimensionless D1 (first `cols` columns)
static double d1_closure(int order, int r, int c) {
    return order == 6 ? O6_D1B[r][c] : order == 4 ? O4_D1B[r][c] : O2_D1B[r][c];
}

// row r of the dimensionless D1: start column and weights (up to D1W_MAX)
static int d1_row(int order, int r, int n, int& start, double w[D1W_MAX]) {
    const int nb = nb_of(order);
    const int cols = order == 6 ? O6_D1W : 6;
    if (r < nb) {
        start = 0;
        for (int c = 0; c < cols; ++c) w[c] = d1_closure(order, r, c);
        return cols;
    }
    if (r > n - 1 - nb) {
        const int rr = n - 1 - r;
        start = n - cols;
        for (int k = 0; k < cols; ++k) w[k] = -d1_closure(order, rr, cols - 1 - k);
        return cols;
    }
    const int half = order / 2;
    const double* I = order == 6 ? O6_D1I : order == 4 ? O4_D1I : O2_D1I;
    start = r - half;
    for (int k = 0; k < 2 * half + 1; ++k) w[k] = I[k];
    return 2 * half + 1;
}

void dense_d1(int order, int n, double* D) {
    std::fill(D, D + (size_t)n * n, 0.0);
    for (int r = 0; r < n; ++r) {
        int s0;
        double w[D1W_MAX];
        const int len = d1_row(order, r, n, s0, w);
        for (int k = 0; k < len; ++k)
            if (s0 + k >= 0 && s0 + k < n) D[(size_t)r * n + s0 + k] += w[k];
    }
}

void derive_d2_closure(int order, double* T) {
    if (order == 6) {
        for (int r = 0; r < O6_R0; ++r)
            for (int m = 0; m < O6_W; ++m)
                for (int s = 0; s < O6_W; ++s) T[((size_t)r * O6_W + m) * O6_W + s] = D2T6.t[r][m][s];
    } else if (order == 4) {
        for (int r = 0; r < O4_R0; ++r)
            for (int m = 0; m < O4_W; ++m)
                for (int s = 0; s < O4_W; ++s) T[((size_t)r * O4_W + m) * O4_W + s] = D2T4.t[r][m][s];
    } else {
        for (int r = 0; r < O2_R0; ++r)
            for (int m = 0; m < O2_W; ++m)
                for (int s = 0; s < O2_W; ++s) T[((size_t)r * O2_W + m) * O2_W + s] = D2T2.t[r][m][s];
    }
}

// banded host application of D1 along a strided line (with 1/h)
static void d1_apply(int order, int n, double h, const double* u, long st, double* out, long ost) {
    for (int r = 0; r < n; ++r) {
        int s0;
        double w[D1W_MAX];
        const int len = d1_row(order, r, n, s0, w);
        double acc = 0.0;
        for (int k = 0; k < len; ++k) acc += w[k] * u[(long)(s0 + k) * st];
        out[(long)r * ost] = acc / h;
    }
}

// ------------------------------------------------------------- context
struct HostFace {
    int kind = BC_TRACTION;
    std::vector<double> U;      // [4][nf] physical U_JL
    std::vector<double> Dv;     // [4][nf] physical V_JL of a dissipative Robin term V u_t, or empty
    std::vector<double> g;      // [2][nf]
    TimeFn tf{TF_ZERO, 0, {0.0, 0.0}};
    // interface jump data in this face's order: V = u(side 0) - u(side 1), Th = tau + tau'
    std::vector<double> V, Th;
    TimeFn jtf{TF_ZERO, 0, {0.0, 0.0}};
    int partner = -1, pface = -1, reversed = 0, side = 0;
    std::vector<double> jhat;   // computed
};

// Per-point host arrays of a block that setup writes in full in parallel
// loops: their allocator leaves new elements uninitialised, so sizing them
// costs no serial zero fill (hundreds of MB at 2049^2).
template <typename V>
struct NoInitAlloc : std::allocator<V> {
    template <typename U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <typename U>
    NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
    template <typename U>
    void construct(U* p) noexcept {
        ::new (static_cast<void*>(p)) U;
    }
    template <typename U, typename... Args>
    void construct(U* p, Args&&... args) {
        ::new (static_cast<void*>(p)) U(std::forward<Args>(args)...);
    }
};
using hvec = std::vector<double, NoInitAlloc<double>>;

struct HostBlock {
    int n1 = 0, n2 = 0;
    double h1 = 0, h2 = 0;
    std::vector<double> X1, X2, rho, C10;
    std::vector<double> F;      // forcing space part [2][np]
    TimeFn ftf{TF_ZERO, 0, {0.0, 0.0}};
    HostFace face[4];
    // computed at finalize
    hvec coef;   // [NCOEF][np]
    hvec J;
    hvec Fm;     // F[I][i] = dx_i/dX_I per point, [4][np] (gradients)
    hvec c10t;   // transformed stiffness, C10 layout
    // device memory owned by the context
    void* d_coef = nullptr;
    void* d_force = nullptr;
    void* d_a1 = nullptr;
    void* d_a2 = nullptr;
    void* d_face[4][5] = {};    // per face: g, U, V, Theta, Dv (device, scaled for the kernels)
    // assembled frame operator (CSR over the frame rows)
    int* d_fr_rowptr = nullptr;
    int* d_fr_col = nullptr;
    void* d_fr_val = nullptr;
    void* d_fr_rsum = nullptr;
    void* u = nullptr;
    void* v = nullptr;
    long np() const { return (long)n1 * n2; }
    int nf(int f) const { return f < 2 ? n2 : n1; }
};

struct Source {
    int block;
    double x1, x2, f1, f2, amp, fp, t0;
};
struct Receiver {
    int block;
    double x1, x2;
};

}  // namespace sbpe

using namespace sbpe;

struct sbpe_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    // the frame kernel runs on a second stream, concurrently with the interior
    // kernel; the two streams are joined at every sweep boundary
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr, ev_side = nullptr;
    int dtype = SBPE_F64;
    int order = 4;
    int op = SBPE_OP_NARROW;        // second-derivative operator of the i = k terms
    bool dissipative = false;       // some face carries a dissipative Robin term V u_t
    int tile_rows = 0;              // output rows per interior tile (0: the default)
    int frame_loop = 1;             // one-launch sweeps: frame groups per frame workgroup (set at create)
    bool frame_loop_set = false;    // frame_loop chosen by sbpe_set_frame_loop
    double beta = 1.0;
    bool host_only = false;
    std::string err;
    std::vector<HostBlock> blocks;
    std::vector<Source> sources;
    std::vector<Receiver> receivers;
    bool finalized = false;
    // plan
    std::vector<BlockDesc> desc;
    BlockDesc* d_desc = nullptr;
    Entry* d_entries = nullptr;
    Range* d_tile_ranges = nullptr;
    Range* d_frame_ranges = nullptr;
    TimeFn* d_items = nullptr;      // time functions of the data items (k_tau)
    RecAdj* d_recadj = nullptr;     // receiver interpolation points for sbpe_receiver_adjoint
    int nrecadj = 0;
    int nitems = 0;
    double* d_tau = nullptr;        // tabulated time functions [steps][nitems][3]
    long tau_cap = 0;               // steps of capacity
    int total_tiles = 0, total_frame_wg = 0;
    // state
    bool bound = false;
    double t = 0.0;
    double* d_rec = nullptr;
    long rec_cap = 0;       // steps of capacity
    long rec_steps = 0;     // steps recorded
    double* d_epart = nullptr;
    double* d_eout = nullptr;
    int npartial = 0;
    double* d_gpart = nullptr;      // band partial sums of the four-stage gradient launch
    long gpart_cap = 0;             // doubles of capacity
    int guard_every = 0;
    double guard_growth = 0.0;
    // member of a batch (sbpe_batch_add): the batch owns the stepping
    void* batch = nullptr;
    // kernel timing: pending (kind, start, stop) event records and sums
    bool frame_sp = false;          // frame rows run from the assembled operator
    double frame_check = -1.0;      // relative difference of the assembled operator to the frame kernel
    // device memory held by the context: size of every allocation, their
    // sum, and the largest sum so far (sbpe_device_bytes)
    std::unordered_map<void*, size_t> dev_sizes;
    size_t dev_held = 0, dev_peak = 0;
    // caller-provided device memory (sbpe_set_allocator), or hipMalloc/hipFree
    sbpe_alloc_fn ualloc = nullptr;
    sbpe_release_fn urelease = nullptr;
    void* uarg = nullptr;
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<int> ev_kind;
    double t_sum[6] = {0, 0, 0, 0, 0, 0};
    int t_cnt[6] = {0, 0, 0, 0, 0, 0};
};

static thread_local std::string g_static_err;

static sbpe_status fail(sbpe_ctx* c, sbpe_status code, const std::string& msg) {
    if (c) c->err = msg;
    else g_static_err = msg;
    return code;
}

static size_t esize(const sbpe_ctx* c) { return c->dtype == SBPE_F64 ? 8 : 4; }

// device allocations of a context, counted for sbpe_device_bytes
template <typename P>
static hipError_t dmalloc(sbpe_ctx* c, P** p, size_t bytes) {
    void* v = nullptr;
    hipError_t e;
    if (c->ualloc) {
        v = bytes > 0 ? c->ualloc(bytes, c->uarg) : nullptr;
        e = (v || bytes == 0) ? hipSuccess : hipErrorOutOfMemory;
        if ((reinterpret_cast<uintptr_t>(v) & 255u) != 0) {   // the kernels assume 256-byte alignment
            c->urelease(v, c->uarg);
            v = nullptr;
            e = hipErrorInvalidValue;
        }
    } else {
        e = hipMalloc(&v, bytes);
    }
    *p = static_cast<P*>(v);
    if (e == hipSuccess) {
        c->dev_sizes[v] = bytes;
        c->dev_held += bytes;
        c->dev_peak = std::max(c->dev_peak, c->dev_held);
    }
    return e;
}

static void dfree(sbpe_ctx* c, const void* p) {
    if (!p) return;
    void* v = const_cast<void*>(p);
    auto it = c->dev_sizes.find(v);
    if (it != c->dev_sizes.end()) {
        c->dev_held -= it->second;
        c->dev_sizes.erase(it);
    }
    if (c->urelease) {
        // hipFree waits for the device; memory handed back to the caller may
        // be reused at once, so every launch that can still read it must end
        (void)hipStreamSynchronize(c->stream);
        if (c->side) (void)hipStreamSynchronize(c->side);
        c->urelease(v, c->uarg);
    } else {
        (void)hipFree(v);
    }
}

#define HIPCHECK(ctx, expr)                                                                       \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, e_ == hipErrorOutOfMemory ? SBPE_ENOMEM : SBPE_EHIP,                 \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                       \
    } while (0)

// upload a double host array to device memory of the context dtype
template <typename Vec>
static sbpe_status upload(sbpe_ctx* c, const Vec& h, void** d) {
    const size_t n = h.size();
    if (dmalloc(c, d, n * esize(c)) != hipSuccess) return fail(c, SBPE_ENOMEM, "device allocation failed");
    if (c->dtype == SBPE_F64) {
        HIPCHECK(c, hipMemcpy(*d, h.data(), n * 8, hipMemcpyHostToDevice));
    } else {
        std::vector<float> f(h.begin(), h.end());
        HIPCHECK(c, hipMemcpy(*d, f.data(), n * 4, hipMemcpyHostToDevice));
    }
    return SBPE_OK;
}

// Whether the symmetric 4x4 matrix A is positive semidefinite up to
// -tol_rel * max(1, largest diagonal entry): LDL^T with diagonal pivoting.  Once
// the largest remaining pivot is at or below the tolerance, the remaining block
// must vanish (a zero diagonal with a nonzero off-diagonal entry, or a negative
// diagonal, means a negative eigenvalue).
static bool psd4(const double Ain[16], double tol_rel) {
    double a[4][4];
    double dmax = 0.0;
    for (int i = 0; i < 4; ++i) {
        for (int j = 0; j < 4; ++j) a[i][j] = Ain[4 * i + j];
        dmax = std::max(dmax, a[i][i]);
    }
    const double tol = tol_rel * std::max(1.0, dmax);
    for (int k = 0; k < 4; ++k) {
        int p = k;
        for (int i = k + 1; i < 4; ++i)
            if (a[i][i] > a[p][p]) p = i;
        if (p != k) {
            for (int j = 0; j < 4; ++j) std::swap(a[k][j], a[p][j]);
            for (int i = 0; i < 4; ++i) std::swap(a[i][k], a[i][p]);
        }
        const double d = a[k][k];
        if (d <= tol) {
            for (int i = k; i < 4; ++i)
                for (int j = k; j < 4; ++j)
                    if (std::fabs(a[i][j]) > tol) return false;
            return true;
        }
        for (int i = k + 1; i < 4; ++i) {
            const double l = a[i][k] / d;
            for (int j = k + 1; j < 4; ++j) a[i][j] -= l * a[k][j];
        }
    }
    return true;
}

// pair index (IJ) -> 0..3 with 11, 12, 21, 22; C10 upper triangle order
static const int C10P[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};

static void c10_to_mat(const double* c10, long np, long p, double M[16]) {
    for (int m = 0; m < 10; ++m) {
        const double v = c10[m * np + p];
        M[4 * C10P[m][0] + C10P[m][1]] = v;
        M[4 * C10P[m][1] + C10P[m][0]] = v;
    }
}

// ------------------------------------------------------------- setup
static sbpe_status setup_block(sbpe_ctx* c, int b) {
    HostBlock& B = c->blocks[b];
    const int n1 = B.n1, n2 = B.n2, o = c->order;
    const long np = B.np();
    B.h1 = 1.0 / (n1 - 1);
    B.h2 = 1.0 / (n2 - 1);
    // A[i][I] = dX_I / dx_i
    hvec A00(np), A01(np), A10(np), A11(np);
#pragma omp parallel for schedule(static)
    for (int j = 0; j < n2; ++j) {
        d1_apply(o, n1, B.h1, &B.X1[(long)j * n1], 1, &A00[(long)j * n1], 1);
        d1_apply(o, n1, B.h1, &B.X2[(long)j * n1], 1, &A01[(long)j * n1], 1);
    }
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n1; ++i) {
        d1_apply(o, n2, B.h2, &B.X1[i], n1, &A10[i], n1);
        d1_apply(o, n2, B.h2, &B.X2[i], n1, &A11[i], n1);
    }
    // every entry is written below (setup fails before any is read otherwise)
    B.J.resize(np);
    B.Fm.resize((size_t)4 * np);
    B.coef.resize((size_t)NCOEF * np);
    B.c10t.resize((size_t)10 * np);
    long bad_j = -1, bad_c = -1;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        const double J = A00[p] * A11[p] - A01[p] * A10[p];
        if (!(J > 0.0)) {
#pragma omp critical
            bad_j = (bad_j < 0 || p < bad_j) ? p : bad_j;
            continue;
        }
        B.J[p] = J;
        // F[I][i] = dx_i / dX_I
        const double F[2][2] = {{A11[p] / J, -A01[p] / J}, {-A10[p] / J, A00[p] / J}};
        for (int q = 0; q < 4; ++q) B.Fm[(size_t)q * np + p] = F[q >> 1][q & 1];
        double Cm[16];
        c10_to_mat(B.C10.data(), np, p, Cm);
        if (!psd4(Cm, 1e-10)) {
#pragma omp critical
            bad_c = (bad_c < 0 || p < bad_c) ? p : bad_c;
            continue;
        }
        // c_ijkl = J F_Ii C_IjKl F_Kk ; C pair index (IJ) -> 2I + J
        double cc[2][2][2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j)
                for (int k = 0; k < 2; ++k)
                    for (int l = 0; l < 2; ++l) {
                        double s = 0.0;
                        for (int I = 0; I < 2; ++I)
                            for (int K = 0; K < 2; ++K) s += F[I][i] * Cm[4 * (2 * I + j) + (2 * K + l)] * F[K][k];
                        cc[i][j][k][l] = J * s;
                    }
        double* q = B.coef.data();
        q[K_C1111 * np + p] = cc[0][0][0][0];
        q[K_C1112 * np + p] = cc[0][0][0][1];
        q[K_C1212 * np + p] = cc[0][1][0][1];
        q[K_C2121 * np + p] = cc[1][0][1][0];
        q[K_C2122 * np + p] = cc[1][0][1][1];
        q[K_C2222 * np + p] = cc[1][1][1][1];
        q[K_C1121 * np + p] = cc[0][0][1][0];
        q[K_C1122 * np + p] = cc[0][0][1][1];
        q[K_C1221 * np + p] = cc[0][1][1][0];
        q[K_C1222 * np + p] = cc[0][1][1][1];
        q[K_IRHO * np + p] = 1.0 / (J * B.rho[p]);
        const int pr[4][2] = {{0, 0}, {0, 1}, {1, 0}, {1, 1}};
        for (int m = 0; m < 10; ++m) {
            const int* a = pr[C10P[m][0]];
            const int* d = pr[C10P[m][1]];
            B.c10t[m * np + p] = cc[a[0]][a[1]][d[0]][d[1]];
        }
    }
    if (bad_j >= 0) {
        const double J = A00[bad_j] * A11[bad_j] - A01[bad_j] * A10[bad_j];
        char buf[160];
        std::snprintf(buf, sizeof buf, "block %d: discrete Jacobian %.3e <= 0 at point (%ld, %ld)", b, J,
                      bad_j % n1, bad_j / n1);
        return fail(c, SBPE_ENONPOS_J, buf);
    }
    if (bad_c >= 0) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "block %d: stiffness not positive semidefinite at point (%ld, %ld)", b,
                      bad_c % n1, bad_c / n1);
        return fail(c, SBPE_ENOT_PSD, buf);
    }
    // surface scale factors: Jhat = |a_t|, a_t = dX/dx_t
    for (int f = 0; f < 4; ++f) {
        const int nf = B.nf(f);
        B.face[f].jhat.assign(nf, 0.0);
        for (int t = 0; t < nf; ++t) {
            long p;
            if (f < 2) p = (long)t * n1 + (f == 0 ? 0 : n1 - 1);
            else p = (long)(f == 2 ? 0 : n2 - 1) * n1 + t;
            B.face[f].jhat[t] = f < 2 ? std::hypot(A10[p], A11[p]) : std::hypot(A00[p], A01[p]);
        }
    }
    return SBPE_OK;
}

// v_max^2 = max over xi of the largest eigenvalue of xi_i c_ijkl xi_k / rho~ at point p
// largest eigenvalue of the acoustic tensor over rho~ at point p, direction (cs, sn)
static double christoffel_lmax_cs(const HostBlock& B, long p, double cs, double sn) {
    const long np = B.np();
    const double* q = B.coef.data();
    // Gamma_jl = sum_ik xi_i c_ijkl xi_k
    const double c1111 = q[K_C1111 * np + p], c1112 = q[K_C1112 * np + p], c1212 = q[K_C1212 * np + p];
    const double c2121 = q[K_C2121 * np + p], c2122 = q[K_C2122 * np + p], c2222 = q[K_C2222 * np + p];
    const double c1121 = q[K_C1121 * np + p], c1122 = q[K_C1122 * np + p], c1221 = q[K_C1221 * np + p],
                 c1222 = q[K_C1222 * np + p];
    // c_1j2l = M_jl, c_2j1l = M_lj
    const double G00 = cs * cs * c1111 + sn * sn * c2121 + 2 * cs * sn * c1121;
    const double G11 = cs * cs * c1212 + sn * sn * c2222 + 2 * cs * sn * c1222;
    const double G01 = cs * cs * c1112 + sn * sn * c2122 + cs * sn * (c1122 + c1221);
    const double tr = G00 + G11, df = G00 - G11;
    return 0.5 * (tr + std::sqrt(df * df + 4 * G01 * G01)) * q[K_IRHO * np + p];
}

static double christoffel_lmax(const HostBlock& B, long p, double th) {
    return christoffel_lmax_cs(B, p, std::cos(th), std::sin(th));
}

static double block_vmax2(const HostBlock& B) {
    // coarse sweep over directions at every point, then golden-section
    // refinement of the best candidates (lambda_max is smooth near its maximum)
    const int nang = 36;
    const long np = B.np();
    std::vector<double> best(np);
    std::vector<int> bk(np);
    double cs[nang], sn[nang];
    for (int k = 0; k < nang; ++k) {
        cs[k] = std::cos(M_PI * k / nang);
        sn[k] = std::sin(M_PI * k / nang);
    }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        double bv = -1.0;
        int kk = 0;
        for (int k = 0; k < nang; ++k) {
            const double v = christoffel_lmax_cs(B, p, cs[k], sn[k]);
            if (v > bv) {
                bv = v;
                kk = k;
            }
        }
        best[p] = bv;
        bk[p] = kk;
    }
    const long keep = std::min<long>(256, np);
    std::vector<long> idx(np);
    for (long p = 0; p < np; ++p) idx[p] = p;
    // the keep largest (their order does not matter: the result is a maximum)
    std::nth_element(idx.begin(), idx.begin() + (keep - 1), idx.end(), [&](long a, long b) { return best[a] > best[b]; });
    double vmax = 0.0;
    const double gr = 0.5 * (std::sqrt(5.0) - 1.0);
    for (long q = 0; q < keep; ++q) {
        const long p = idx[q];
        const double d = M_PI / nang;
        double a = M_PI * bk[p] / nang - d, b = M_PI * bk[p] / nang + d;
        double x1 = b - gr * (b - a), x2 = a + gr * (b - a);
        double f1 = christoffel_lmax(B, p, x1), f2 = christoffel_lmax(B, p, x2);
        for (int it = 0; it < 60; ++it) {
            if (f1 < f2) {
                a = x1;
                x1 = x2;
                f1 = f2;
                x2 = a + gr * (b - a);
                f2 = christoffel_lmax(B, p, x2);
            } else {
                b = x2;
                x2 = x1;
                f2 = f1;
                x1 = b - gr * (b - a);
                f1 = christoffel_lmax(B, p, x1);
            }
        }
        vmax = std::max(vmax, std::max(best[p], std::max(f1, f2)));
    }
    return vmax;
}

// moment-matching weights on the four nearest points (cubic Lagrange)
static void weights_1d(double x0, int n, int& m0, double w[4]) {
    const double h = 1.0 / (n - 1);
    m0 = (int)std::floor(x0 / h) - 1;
    m0 = std::min(std::max(m0, 0), n - 4);
    for (int k = 0; k < 4; ++k) {
        double v = 1.0;
        for (int l = 0; l < 4; ++l)
            if (l != k) v *= (x0 - (m0 + l) * h) / ((k - l) * h);
        w[k] = v;
    }
}

// frame index of point (i, j) of a block (inverse of the k_frame mapping)
static long frame_index(const HostBlock& B, int R, int i, int j) {
    const int n1 = B.n1, n2 = B.n2;
    if (j < R) return (long)j * n1 + i;
    if (j >= n2 - R) return (long)R * n1 + (long)(j - (n2 - R)) * n1 + i;
    // side bands column by column, so that the points of a wave share their x1 closure row
    const int cc = i < R ? i : i - (n1 - 2 * R);
    return 2L * R * n1 + (long)cc * (n2 - 2 * R) + (j - R);
}

// Small grids, where the default tiles and frame groups are too few to fill
// the GPU's 256 compute units more than about 1.5 times: a sweep then lasts
// as long as one workgroup's chain of rows, so the default launch shape
// shortens the chains: tiles of one pass of the row loop (2H + 1 = order + 1
// rows) and one frame group per frame workgroup.  Measured per RK4 step on
// one block, FP64: 65^2 38 -> 26 us, 257^2 42 -> 29 us, 385^2 42 -> 41 us
// (FP32 36 -> 28 us); at 513^2 (459 default tiles) the default shape is the
// faster one.
static int default_frame_loop(int dtype);
static bool plan_is_small(const sbpe_ctx* c, int R, int tile_w) {
    long tiles = 0, groups = 0;
    for (const HostBlock& H : c->blocks) {
        const long ix = H.n1 - 2 * R, iy = H.n2 - 2 * R;
        if (ix > 0 && iy > 0) tiles += ((ix + tile_w - 1) / tile_w) * ((iy + TILE_Y_DEFAULT - 1) / TILE_Y_DEFAULT);
        const long fn = 2L * R * H.n1 + 2L * R * std::max(0L, iy);
        groups += (fn + FRAME_PTS - 1) / FRAME_PTS;
    }
    return tiles < 384 && groups < 384;
}

static sbpe_status build_plan(sbpe_ctx* c) {
    const int R = frame_of(c->order);
    const int nb = (int)c->blocks.size();
    // interior tiles: 64 lanes, of which the central 64 - 2 * half-width are written
    const int tile_w = TILE_LANES - 2 * (c->order / 2);
    const bool small = plan_is_small(c, R, tile_w);
    int tile_y = c->tile_rows > 0 ? c->tile_rows : TILE_Y_DEFAULT;
    if (c->tile_rows <= 0 && small) tile_y = c->order + 1;
    if (!c->frame_loop_set) c->frame_loop = small ? 1 : default_frame_loop(c->dtype);
    if (const char* e = std::getenv("SBPE_TILE_ROWS")) tile_y = std::max(1, std::atoi(e));
    c->desc.assign(nb, BlockDesc{});
    int tiles = 0, fwg = 0;
    for (int b = 0; b < nb; ++b) {
        HostBlock& H = c->blocks[b];
        BlockDesc& D = c->desc[b];
        D.n1 = H.n1;
        D.n2 = H.n2;
        D.h1 = H.h1;
        D.h2 = H.h2;
        D.coef = H.d_coef;
        D.force = H.d_force;
        D.item_f = b * ITEMS_PER_BLOCK + 8;
        D.a1 = H.d_a1;
        D.a2 = H.d_a2;
        D.u = H.u;
        D.v = H.v;
        const int ix = H.n1 - 2 * R, iy = H.n2 - 2 * R;
        D.tile_y = tile_y;
        D.tiles_x = ix > 0 ? (ix + tile_w - 1) / tile_w : 0;
        D.tiles_y = iy > 0 ? (iy + tile_y - 1) / tile_y : 0;
        D.tile_beg = tiles;
        tiles += D.tiles_x * D.tiles_y;
        D.frame_n = 2 * R * H.n1 + 2 * R * std::max(0, H.n2 - 2 * R);
        D.frame_wg = (D.frame_n + FRAME_PTS - 1) / FRAME_PTS;
        D.frame_beg = fwg;
        fwg += D.frame_wg;
        for (int f = 0; f < 4; ++f) {
            const HostFace& HF = H.face[f];
            FaceDesc& F = D.face[f];
            F.kind = HF.kind;
            F.nf = H.nf(f);
            const int a = f >> 1;
            F.w = (a == 0 ? H.h1 : H.h2) * norm_weight(c->order, a == 0 ? H.n1 : H.n2, 0);
            F.item_g = b * ITEMS_PER_BLOCK + f;
            F.item_v = b * ITEMS_PER_BLOCK + 4 + f;
            F.g = H.d_face[f][0];
            F.U = H.d_face[f][1];
            F.partner = HF.partner;
            F.pface = HF.pface;
            F.reversed = HF.reversed;
            F.vsign = HF.side == 0 ? 1.0 : -1.0;
            F.V = H.d_face[f][2];
            F.Th = H.d_face[f][3];
            F.Dv = H.d_face[f][4];
            if (HF.kind == BC_INTERFACE) {
                const HostBlock& P = c->blocks[HF.partner];
                const int pa = HF.pface >> 1;
                F.pw = (pa == 0 ? P.h1 : P.h2) * norm_weight(c->order, pa == 0 ? P.n1 : P.n2, 0);
            }
        }
    }
    c->total_tiles = tiles;
    c->total_frame_wg = fwg;
    // point entries (sources, receivers), bucketed by workgroup
    struct E2 {
        int frame;
        int wg;
        Entry e;
    };
    std::vector<E2> ents;
    auto add_point = [&](int b, int i, int j, const Entry& e) {
        const HostBlock& H = c->blocks[b];
        const BlockDesc& D = c->desc[b];
        E2 x;
        x.e = e;
        x.e.p = j * H.n1 + i;
        if (i >= R && i <= H.n1 - 1 - R && j >= R && j <= H.n2 - 1 - R) {
            x.frame = 0;
            x.wg = D.tile_beg + ((j - R) / D.tile_y) * D.tiles_x + (i - R) / tile_w;
        } else {
            x.frame = 1;
            x.wg = D.frame_beg + (int)(frame_index(H, R, i, j) / FRAME_PTS);
        }
        ents.push_back(x);
    };
    // time-function items: per block 4 faces (g), 4 faces (jump data), forcing; then sources
    std::vector<TimeFn> items((size_t)nb * ITEMS_PER_BLOCK + c->sources.size(), TimeFn{TF_ZERO, 0, {0.0, 0.0}});
    for (int b = 0; b < nb; ++b) {
        for (int f = 0; f < 4; ++f) {
            items[(size_t)b * ITEMS_PER_BLOCK + f] = c->blocks[b].face[f].tf;
            items[(size_t)b * ITEMS_PER_BLOCK + 4 + f] = c->blocks[b].face[f].jtf;
        }
        items[(size_t)b * ITEMS_PER_BLOCK + 8] = c->blocks[b].ftf;
    }
    for (size_t s = 0; s < c->sources.size(); ++s) {
        const Source& S = c->sources[s];
        const HostBlock& H = c->blocks[S.block];
        int i0, j0;
        double wi[4], wj[4];
        weights_1d(S.x1, H.n1, i0, wi);
        weights_1d(S.x2, H.n2, j0, wj);
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 4; ++d) {
                const int i = i0 + d, j = j0 + a;
                const double Hp = H.h1 * H.h2 * norm_weight(c->order, H.n1, i) * norm_weight(c->order, H.n2, j);
                const double w = wi[d] * wj[a] / Hp;
                Entry e{0, 0, nb * ITEMS_PER_BLOCK + (int)s, 0, S.amp * S.f1 * w, S.amp * S.f2 * w};
                add_point(S.block, i, j, e);
            }
        items[(size_t)nb * ITEMS_PER_BLOCK + s] = TimeFn{TF_RICKER, 0, {S.fp, S.t0}};
    }
    for (size_t r = 0; r < c->receivers.size(); ++r) {
        const Receiver& Rv = c->receivers[r];
        const HostBlock& H = c->blocks[Rv.block];
        int i0, j0;
        double wi[4], wj[4];
        weights_1d(Rv.x1, H.n1, i0, wi);
        weights_1d(Rv.x2, H.n2, j0, wj);
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 4; ++d) {
                Entry e{0, 1, (int)(r * 16 + 4 * a + d), 0, wi[d] * wj[a], 0.0};
                add_point(Rv.block, i0 + d, j0 + a, e);
            }
    }
    // receiver interpolation points with weight / (H rho~) (adjoint of the sampling)
    std::vector<RecAdj> radj;
    for (size_t r = 0; r < c->receivers.size(); ++r) {
        const Receiver& Rv = c->receivers[r];
        const HostBlock& H = c->blocks[Rv.block];
        int i0, j0;
        double wi[4], wj[4];
        weights_1d(Rv.x1, H.n1, i0, wi);
        weights_1d(Rv.x2, H.n2, j0, wj);
        for (int a = 0; a < 4; ++a)
            for (int d = 0; d < 4; ++d) {
                const int i = i0 + d, j = j0 + a;
                const long p = (long)j * H.n1 + i;
                const double Hp = H.h1 * H.h2 * norm_weight(c->order, H.n1, i) * norm_weight(c->order, H.n2, j);
                const double rt = H.J[p] * H.rho[p];
                radj.push_back(RecAdj{(int)r, Rv.block, p, wi[d] * wj[a] / (Hp * rt)});
            }
    }
    // by workgroup, then sources before receivers, then by point (the
    // interior kernel walks a tile's entries row by row); entries of one
    // point keep their order
    std::stable_sort(ents.begin(), ents.end(), [](const E2& x, const E2& y) {
        if (x.frame != y.frame) return x.frame < y.frame;
        if (x.wg != y.wg) return x.wg < y.wg;
        if (x.e.kind != y.e.kind) return x.e.kind < y.e.kind;
        return x.e.p < y.e.p;
    });
    std::vector<Entry> flat;
    std::vector<Range> tr(std::max(tiles, 1), Range{0, 0, 0, 0}), fr(std::max(fwg, 1), Range{0, 0, 0, 0});
    for (size_t k = 0; k < ents.size(); ++k) {
        const int idx = (int)flat.size();
        flat.push_back(ents[k].e);
        Range& rg = ents[k].frame ? fr[ents[k].wg] : tr[ents[k].wg];
        if (rg.end == rg.beg) {
            rg.beg = idx;
            rg.mid = idx;
        }
        rg.end = idx + 1;
        if (ents[k].e.kind == 0) rg.mid = idx + 1;
    }
    if (c->host_only) return SBPE_OK;
    if (flat.empty()) flat.push_back(Entry{-1, -1, 0, 0, 0.0, 0.0});
    c->nitems = (int)items.size();
    c->nrecadj = (int)radj.size();
    if (!radj.empty()) {
        HIPCHECK(c, dmalloc(c, &c->d_recadj, radj.size() * sizeof(RecAdj)));
        HIPCHECK(c, hipMemcpy(c->d_recadj, radj.data(), radj.size() * sizeof(RecAdj), hipMemcpyHostToDevice));
    }
    HIPCHECK(c, dmalloc(c, &c->d_entries, flat.size() * sizeof(Entry)));
    HIPCHECK(c, hipMemcpy(c->d_entries, flat.data(), flat.size() * sizeof(Entry), hipMemcpyHostToDevice));
    HIPCHECK(c, dmalloc(c, &c->d_tile_ranges, tr.size() * sizeof(Range)));
    HIPCHECK(c, hipMemcpy(c->d_tile_ranges, tr.data(), tr.size() * sizeof(Range), hipMemcpyHostToDevice));
    HIPCHECK(c, dmalloc(c, &c->d_frame_ranges, fr.size() * sizeof(Range)));
    HIPCHECK(c, hipMemcpy(c->d_frame_ranges, fr.data(), fr.size() * sizeof(Range), hipMemcpyHostToDevice));
    HIPCHECK(c, dmalloc(c, &c->d_items, items.size() * sizeof(TimeFn)));
    HIPCHECK(c, hipMemcpy(c->d_items, items.data(), items.size() * sizeof(TimeFn), hipMemcpyHostToDevice));
    c->tau_cap = 1;
    HIPCHECK(c, dmalloc(c, &c->d_tau, (size_t)c->nitems * 3 * sizeof(double)));
    HIPCHECK(c, hipMemset(c->d_tau, 0, (size_t)c->nitems * 3 * sizeof(double)));
    for (int b = 0; b < nb; ++b) {
        BlockDesc& D = c->desc[b];
        D.dt = 0.0;
        D.beta = c->beta;
        D.tau = c->d_tau;
        D.nitems = c->nitems;
        D.step0 = 0;
        D.entries = c->d_entries;
        D.tile_rng = c->d_tile_ranges + D.tile_beg;
        D.frame_rng = c->d_frame_ranges + D.frame_beg;
        D.rec = nullptr;
        D.rec_stride = (long)c->receivers.size() * 16 * 2;
    }
    HIPCHECK(c, dmalloc(c, &c->d_desc, nb * sizeof(BlockDesc)));
    HIPCHECK(c, hipMemcpy(c->d_desc, c->desc.data(), nb * sizeof(BlockDesc), hipMemcpyHostToDevice));
    c->npartial = 1024;
    HIPCHECK(c, dmalloc(c, &c->d_epart, c->npartial * sizeof(double)));
    HIPCHECK(c, dmalloc(c, &c->d_eout, sizeof(double)));
    return SBPE_OK;
}

static sbpe_status sync_desc(sbpe_ctx* c) {
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        c->desc[b].u = c->blocks[b].u;
        c->desc[b].v = c->blocks[b].v;
    }
    HIPCHECK(c, hipMemcpyAsync(c->d_desc, c->desc.data(), c->desc.size() * sizeof(BlockDesc), hipMemcpyHostToDevice,
                               c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return SBPE_OK;
}

static PassArgs base_args(const sbpe_ctx* c) {
    PassArgs a;
    std::memset(&a, 0, sizeof a);
    a.blocks = c->d_desc;
    a.nblocks = (int)c->blocks.size();
    a.wide = c->op == SBPE_OP_WIDE ? 1 : 0;
    a.floop = c->frame_loop;
    return a;
}

// Per-context sweep data in the block descriptors (time step, time-function
// table, receiver buffer).  Uploaded only when something changed.
static sbpe_status refresh_desc(sbpe_ctx* c, double dt, const double* tau) {
    bool changed = false;
    const long nrec = (long)c->receivers.size();
    for (size_t b = 0; b < c->desc.size(); ++b) {
        BlockDesc& D = c->desc[b];
        double* rec = nrec > 0 ? c->d_rec : nullptr;
        if (D.dt != dt || D.tau != tau || D.rec != rec) changed = true;
        D.dt = dt;
        D.tau = tau;
        D.rec = rec;
    }
    if (!changed) return SBPE_OK;
    HIPCHECK(c, hipStreamSynchronize(c->side));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(c->d_desc, c->desc.data(), c->desc.size() * sizeof(BlockDesc), hipMemcpyHostToDevice));
    return SBPE_OK;
}

static hipEvent_t next_event(sbpe_ctx* c) {
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        c->ev_pool.push_back(e);
    }
    return c->ev_pool[c->ev_used++];
}

// sum the elapsed times of all recorded event pairs (synchronises)
static sbpe_status collect_timing(sbpe_ctx* c) {
    if (c->ev_used == 0) return SBPE_OK;
    HIPCHECK(c, hipStreamSynchronize(c->side));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    for (size_t k = 0; k < c->ev_kind.size(); ++k) {
        float ms = 0.f;
        HIPCHECK(c, hipEventElapsedTime(&ms, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]));
        c->t_sum[c->ev_kind[k]] += ms;
        c->t_cnt[c->ev_kind[k]] += 1;
    }
    c->ev_used = 0;
    c->ev_kind.clear();
    return SBPE_OK;
}

// join the two streams: each waits for the work already enqueued on the other
static sbpe_status join_streams(sbpe_ctx* c) {
    HIPCHECK(c, hipEventRecord(c->ev_main, c->stream));
    HIPCHECK(c, hipStreamWaitEvent(c->side, c->ev_main, 0));
    HIPCHECK(c, hipEventRecord(c->ev_side, c->side));
    HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_side, 0));
    return SBPE_OK;
}

static sbpe_status run_pass(sbpe_ctx* c, const PassArgs& a) {
    // launch kinds: 2 * pass index (RK1 = 0, RK2 = 1, APPLY = 2) + (0 interior, 1 frame)
    const int pk = a.pass == PASS_RK1 ? 0 : a.pass == PASS_RK2 ? 1 : 2;
    sbpe_status s;
    if (c->frame_sp && sweep_fused(c->total_tiles)) {
        // assembled frame operator: frame and interior in one launch on the context stream
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            if (c->ev_kind.size() >= 4096) {
                s = collect_timing(c);
                if (s) return s;
            }
            e0 = next_event(c);
            e1 = next_event(c);
            if (!e0 || !e1) return fail(c, SBPE_EHIP, "hipEventCreate failed");
            HIPCHECK(c, hipEventRecord(e0, c->stream));
        }
        const int e = launch_pass(c->dtype, c->order, a, c->total_tiles, c->total_frame_wg, c->stream);
        if (e != 0) return fail(c, SBPE_EHIP, std::string("kernel launch: ") + hip_error_string(e));
        if (c->timing) {
            HIPCHECK(c, hipEventRecord(e1, c->stream));
            c->ev_kind.push_back(2 * pk);
        }
        return SBPE_OK;
    }
    s = join_streams(c);
    if (s) return s;
    for (int part = 0; part < 2; ++part) {
        hipStream_t st = part == 0 ? c->stream : c->side;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            if (c->ev_kind.size() >= 4096) {
                s = collect_timing(c);
                if (s) return s;
            }
            e0 = next_event(c);
            e1 = next_event(c);
            if (!e0 || !e1) return fail(c, SBPE_EHIP, "hipEventCreate failed");
            HIPCHECK(c, hipEventRecord(e0, st));
        }
        const int e = part == 0  ? launch_interior(c->dtype, c->order, a, c->total_tiles, st)
                      : c->frame_sp ? launch_frame_sp(c->dtype, c->order, a, c->total_frame_wg, st)
                                    : launch_frame(c->dtype, c->order, a, c->total_frame_wg, st);
        if (e != 0) return fail(c, SBPE_EHIP, std::string("kernel launch: ") + hip_error_string(e));
        if (c->timing) {
            HIPCHECK(c, hipEventRecord(e1, st));
            c->ev_kind.push_back(2 * pk + part);
        }
    }
    return SBPE_OK;
}

// make the caller's stream wait for everything enqueued on the side stream
static sbpe_status finish_passes(sbpe_ctx* c) {
    HIPCHECK(c, hipEventRecord(c->ev_side, c->side));
    HIPCHECK(c, hipStreamWaitEvent(c->stream, c->ev_side, 0));
    return SBPE_OK;
}

static bool check_ctx(sbpe_ctx* c) { return c != nullptr; }

// tabulate the time functions of nsteps steps starting at t0 into d_tau
static sbpe_status grow_tau(sbpe_ctx* c, long steps);
static sbpe_status fill_tau(sbpe_ctx* c, int nsteps, double t0, double dt) {
    const sbpe_status s = grow_tau(c, nsteps);
    if (s) return s;
    const int e = launch_tau(c->d_items, c->nitems, nsteps, t0, dt, c->d_tau, c->stream);
    if (e != 0) return fail(c, SBPE_EHIP, std::string("tau launch: ") + hip_error_string(e));
    return SBPE_OK;
}

// receiver record capacity of at least `steps` steps; the recorded rows are
// kept (a reallocation synchronises the stream)
static sbpe_status grow_receivers(sbpe_ctx* c, long steps) {
    const long nrec = (long)c->receivers.size();
    const long slots = nrec * 16 * 2;
    if (nrec == 0 || steps <= c->rec_cap) return SBPE_OK;
    const long cap = std::max<long>(steps, 2 * c->rec_cap);
    double* nd = nullptr;
    if (dmalloc(c, &nd, cap * slots * sizeof(double)) != hipSuccess) return fail(c, SBPE_ENOMEM, "receiver buffer");
    if (c->d_rec && c->rec_steps > 0 &&
        hipMemcpyAsync(nd, c->d_rec, c->rec_steps * slots * sizeof(double), hipMemcpyDeviceToDevice, c->stream) !=
            hipSuccess) {
        dfree(c, nd);
        return fail(c, SBPE_EHIP, "receiver buffer copy");
    }
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dfree(c, c->d_rec);
    c->d_rec = nd;
    c->rec_cap = cap;
    return SBPE_OK;
}

// time-function table capacity of at least `steps` steps (contents not kept)
static sbpe_status grow_tau(sbpe_ctx* c, long steps) {
    if (steps <= c->tau_cap) return SBPE_OK;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    dfree(c, c->d_tau);
    c->d_tau = nullptr;
    c->tau_cap = 0;     // a failed allocation leaves no table behind
    if (dmalloc(c, &c->d_tau, (size_t)steps * c->nitems * 3 * sizeof(double)) != hipSuccess)
        return fail(c, SBPE_ENOMEM, "time-function table");
    c->tau_cap = steps;
    return SBPE_OK;
}

static sbpe_status need_gpu(sbpe_ctx* c) {
    if (c->host_only) return fail(c, SBPE_ESTATE, "host-only context");
    if (!c->finalized) return fail(c, SBPE_ESTATE, "context not finalized");
    return SBPE_OK;
}

static void set_time_fn(int kind, const double* p, TimeFn& tf) {
    tf.kind = kind;
    tf.pad = 0;
    tf.p[0] = p ? p[0] : 0.0;
    tf.p[1] = p ? p[1] : 0.0;
}

// ================================================================ C ABI
extern "C" {

// Frame groups per frame workgroup of a one-launch sweep unless set: measured
// at 513^2 and 1025^2 with the default tiles, 2 (FP64) and 4 (FP32) beat 1 by
// 8-20 %.
static int default_frame_loop(int dtype) { return dtype == SBPE_F32 ? 4 : 2; }

sbpe_status sbpe_create(int device, void* stream, int dtype, int order, double beta, sbpe_ctx_t* out) {
    if (!out) return fail(nullptr, SBPE_EINVAL, "out is NULL");
    if (dtype != SBPE_F64 && dtype != SBPE_F32) return fail(nullptr, SBPE_EINVAL, "dtype must be SBPE_F64 or SBPE_F32");
    if (order != 2 && order != 4 && order != 6) return fail(nullptr, SBPE_EINVAL, "order must be 2, 4 or 6");
    if (!(beta >= 1.0)) return fail(nullptr, SBPE_EINVAL, "beta must be >= 1 (Theorem 2)");
    sbpe_ctx* c = new sbpe_ctx;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->dtype = dtype;
    c->order = order;
    c->frame_loop = default_frame_loop(dtype);
    c->beta = beta;
    c->host_only = device < 0;
    if (!c->host_only) {
        int n = 0;
        if (hipGetDeviceCount(&n) != hipSuccess || device >= n) {
            delete c;
            return fail(nullptr, SBPE_EHIP, "no such HIP device");
        }
        if (hipSetDevice(device) != hipSuccess) {
            delete c;
            return fail(nullptr, SBPE_EHIP, "hipSetDevice failed");
        }
        // device address of the no-allocation scratch on this device (once per device)
        const int se = scratch_init(device);
        if (se != 0) {
            delete c;
            return fail(nullptr, SBPE_EHIP, std::string("scratch symbol lookup: ") + hip_error_string(se));
        }
        if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_main, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&c->ev_side, hipEventDisableTiming) != hipSuccess) {
            delete c;
            return fail(nullptr, SBPE_EHIP, "stream/event creation failed");
        }
    }
    *out = c;
    return SBPE_OK;
}

sbpe_status sbpe_destroy(sbpe_ctx_t c) {
    if (!c) return SBPE_OK;
    // a batch member's fields and tables are referenced by the batch's
    // descriptors and may be in use by its enqueued sweeps
    if (c->batch) return fail(c, SBPE_ESTATE, "context is a member of a batch: sbpe_batch_remove it first");
    if (!c->host_only) {
        (void)hipStreamSynchronize(c->stream);
        (void)hipStreamSynchronize(c->side);
        for (auto& B : c->blocks) {
            dfree(c, B.d_coef);
            dfree(c, B.d_force);
            dfree(c, B.d_a1);
            dfree(c, B.d_a2);
            for (int f = 0; f < 4; ++f)
                for (int k = 0; k < 5; ++k) dfree(c, B.d_face[f][k]);
            dfree(c, B.d_fr_rowptr);
            dfree(c, B.d_fr_col);
            dfree(c, B.d_fr_val);
            dfree(c, B.d_fr_rsum);
        }
        dfree(c, c->d_desc);
        dfree(c, c->d_entries);
        dfree(c, c->d_tile_ranges);
        dfree(c, c->d_frame_ranges);
        dfree(c, c->d_items);
        dfree(c, c->d_recadj);
        dfree(c, c->d_tau);
        dfree(c, c->d_rec);
        dfree(c, c->d_epart);
        dfree(c, c->d_eout);
        dfree(c, c->d_gpart);
        for (auto e : c->ev_pool) (void)hipEventDestroy(e);
        (void)hipStreamSynchronize(c->side);
        (void)hipEventDestroy(c->ev_main);
        (void)hipEventDestroy(c->ev_side);
        (void)hipStreamDestroy(c->side);
    }
    delete c;
    return SBPE_OK;
}

const char* sbpe_last_error(sbpe_ctx_t c) { return c ? c->err.c_str() : g_static_err.c_str(); }

sbpe_status sbpe_set_allocator(sbpe_ctx_t c, sbpe_alloc_fn alloc, sbpe_release_fn release, void* user) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (!alloc != !release) return fail(c, SBPE_EINVAL, "allocate and release callbacks must be given together");
    if (c->finalized || !c->dev_sizes.empty())
        return fail(c, SBPE_ESTATE, "the allocator is set before the context allocates (before sbpe_finalize)");
    c->ualloc = alloc;
    c->urelease = release;
    c->uarg = user;
    return SBPE_OK;
}

sbpe_status sbpe_voigt_to_c10(const double* V, size_t npts, double* C10) {
    if (!V || !C10) return fail(nullptr, SBPE_EINVAL, "NULL array");
    for (size_t p = 0; p < npts; ++p) {
        const double c11 = V[p], c12 = V[npts + p], c16 = V[2 * npts + p], c22 = V[3 * npts + p],
                     c26 = V[4 * npts + p], c66 = V[5 * npts + p];
        // C1111, C1112, C1121, C1122, C1212, C1221, C1222, C2121, C2122, C2222
        const double vals[10] = {c11, c16, c16, c12, c66, c66, c26, c66, c26, c22};
        for (int m = 0; m < 10; ++m) C10[m * npts + p] = vals[m];
    }
    return SBPE_OK;
}

sbpe_status sbpe_add_block(sbpe_ctx_t c, int n1, int n2, const double* X1, const double* X2, const double* rho,
                           const double* C10, int* block_id) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail(c, SBPE_ESTATE, "context already finalized");
    const int nmin = min_points(c->order);
    if (n1 < nmin || n2 < nmin) return fail(c, SBPE_EINVAL, "block too small for the operator order");
    // the kernels address a field with 32-bit byte offsets and the frame operator
    // encodes a partner point in 28 bits: at most 2^28 points per block
    if ((long)n1 * n2 > (1L << 28)) return fail(c, SBPE_EINVAL, "block has more than 2^28 points");
    if (!X1 || !X2 || !rho || !C10) return fail(c, SBPE_EINVAL, "NULL array");
    const long np = (long)n1 * n2;
    for (long p = 0; p < np; ++p)
        if (!(rho[p] > 0.0)) return fail(c, SBPE_EINVAL, "density must be positive");
    HostBlock B;
    B.n1 = n1;
    B.n2 = n2;
    B.X1.assign(X1, X1 + np);
    B.X2.assign(X2, X2 + np);
    B.rho.assign(rho, rho + np);
    B.C10.assign(C10, C10 + 10 * np);
    c->blocks.push_back(std::move(B));
    if (block_id) *block_id = (int)c->blocks.size() - 1;
    return SBPE_OK;
}

static sbpe_status check_face(sbpe_ctx* c, int block, int face) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail(c, SBPE_ESTATE, "context already finalized");
    if (block < 0 || block >= (int)c->blocks.size()) return fail(c, SBPE_EINVAL, "no such block");
    if (face < 0 || face > 3) return fail(c, SBPE_EINVAL, "face must be 0..3");
    return SBPE_OK;
}

sbpe_status sbpe_set_tile_rows(sbpe_ctx_t c, int rows) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail(c, SBPE_ESTATE, "context already finalized");
    if (rows < 0 || rows > 256) return fail(c, SBPE_EINVAL, "tile rows must be 0 (default) or 1..256");
    c->tile_rows = rows;
    return SBPE_OK;
}

sbpe_status sbpe_set_frame_loop(sbpe_ctx_t c, int groups) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (groups < 1 || groups > 64) return fail(c, SBPE_EINVAL, "frame groups per workgroup must be 1..64");
    c->frame_loop = groups;
    c->frame_loop_set = true;
    return SBPE_OK;
}

sbpe_status sbpe_set_operator(sbpe_ctx_t c, int op) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail(c, SBPE_ESTATE, "context already finalized");
    if (op != SBPE_OP_NARROW && op != SBPE_OP_WIDE) return fail(c, SBPE_EINVAL, "operator must be narrow or wide");
    if (op == SBPE_OP_WIDE && c->order == 6)
        return fail(c, SBPE_EINVAL, "the wide-stencil operator is built for orders 2 and 4");
    c->op = op;
    return SBPE_OK;
}

sbpe_status sbpe_set_bc(sbpe_ctx_t c, int block, int face, int bc, const double* U) {
    sbpe_status s = check_face(c, block, face);
    if (s) return s;
    if (bc != SBPE_BC_TRACTION && bc != SBPE_BC_ROBIN && bc != SBPE_BC_DISPLACEMENT)
        return fail(c, SBPE_EINVAL, "bc must be traction, Robin or displacement (use sbpe_connect for interfaces)");
    HostFace& F = c->blocks[block].face[face];
    if (F.kind == BC_INTERFACE) return fail(c, SBPE_ESTATE, "face is part of an interface");
    const int nf = c->blocks[block].nf(face);
    if (bc == SBPE_BC_ROBIN) {
        if (!U) return fail(c, SBPE_EINVAL, "Robin condition needs U");
        for (int t = 0; t < nf; ++t) {
            const double a = U[t], b = U[nf + t], b2 = U[2 * nf + t], d = U[3 * nf + t];
            if (std::fabs(b - b2) > 1e-12 * (std::fabs(a) + std::fabs(d) + 1e-300) || a < 0 || d < 0 ||
                a * d - b * b < -1e-12 * (a * d + 1e-300))
                return fail(c, SBPE_EINVAL, "U must be symmetric positive semidefinite");
        }
        F.U.assign(U, U + 4 * nf);
    } else {
        F.U.clear();
    }
    F.kind = bc;
    return SBPE_OK;
}

// symmetric positive semidefinite 2x2 matrices M[k * nf + t] (row-major JL) at every face point
static bool psd2_field(const double* M, int nf) {
    for (int t = 0; t < nf; ++t) {
        const double a = M[t], b = M[nf + t], b2 = M[2 * nf + t], d = M[3 * nf + t];
        if (std::fabs(b - b2) > 1e-12 * (std::fabs(a) + std::fabs(d) + 1e-300) || a < 0 || d < 0 ||
            a * d - b * b < -1e-12 * (a * d + 1e-300))
            return false;
    }
    return true;
}

sbpe_status sbpe_set_bc_dissipation(sbpe_ctx_t c, int block, int face, const double* V) {
    sbpe_status s = check_face(c, block, face);
    if (s) return s;
    HostFace& F = c->blocks[block].face[face];
    if (F.kind != BC_TRACTION && F.kind != BC_ROBIN)
        return fail(c, SBPE_ESTATE, "a dissipative term needs a traction or Robin face");
    if (!V) {
        F.Dv.clear();
        return SBPE_OK;
    }
    const int nf = c->blocks[block].nf(face);
    if (!psd2_field(V, nf)) return fail(c, SBPE_EINVAL, "V must be symmetric positive semidefinite");
    F.Dv.assign(V, V + 4 * nf);
    return SBPE_OK;
}

sbpe_status sbpe_set_bc_data(sbpe_ctx_t c, int block, int face, const double* g, int time_fn, const double* tp) {
    sbpe_status s = check_face(c, block, face);
    if (s) return s;
    if (time_fn < SBPE_TIME_ZERO || time_fn > SBPE_TIME_RICKER) return fail(c, SBPE_EINVAL, "bad time function");
    HostFace& F = c->blocks[block].face[face];
    const int nf = c->blocks[block].nf(face);
    if (g) F.g.assign(g, g + 2 * nf);
    else F.g.clear();
    set_time_fn(time_fn, tp, F.tf);
    return SBPE_OK;
}

sbpe_status sbpe_connect(sbpe_ctx_t c, int bA, int fA, int bB, int fB, int reversed) {
    sbpe_status s = check_face(c, bA, fA);
    if (s) return s;
    s = check_face(c, bB, fB);
    if (s) return s;
    if (bA == bB && fA == fB) return fail(c, SBPE_EINVAL, "a face cannot be connected to itself");
    HostFace& A = c->blocks[bA].face[fA];
    HostFace& B = c->blocks[bB].face[fB];
    if (A.kind == BC_INTERFACE || B.kind == BC_INTERFACE) return fail(c, SBPE_ESTATE, "face already connected");
    if (c->blocks[bA].nf(fA) != c->blocks[bB].nf(fB)) return fail(c, SBPE_EIFACE, "faces have different point counts");
    A.kind = B.kind = BC_INTERFACE;
    A.partner = bB;
    A.pface = fB;
    B.partner = bA;
    B.pface = fA;
    A.reversed = B.reversed = reversed ? 1 : 0;
    A.side = 0;
    B.side = 1;
    return SBPE_OK;
}

sbpe_status sbpe_set_interface_data(sbpe_ctx_t c, int block, int face, const double* V, const double* Th,
                                    int time_fn, const double* tp) {
    sbpe_status s = check_face(c, block, face);
    if (s) return s;
    if (time_fn < SBPE_TIME_ZERO || time_fn > SBPE_TIME_RICKER) return fail(c, SBPE_EINVAL, "bad time function");
    HostFace& A = c->blocks[block].face[face];
    if (A.kind != BC_INTERFACE) return fail(c, SBPE_ESTATE, "face is not an interface");
    HostFace& B = c->blocks[A.partner].face[A.pface];
    const int nf = c->blocks[block].nf(face);
    // both faces keep V as u(side 0) - u(side 1) and Theta, each in its own order
    const double sv = A.side == 0 ? 1.0 : -1.0;
    auto other = [&](int t) { return A.reversed ? nf - 1 - t : t; };
    A.V.clear();
    B.V.clear();
    A.Th.clear();
    B.Th.clear();
    if (V) {
        A.V.assign(2 * nf, 0.0);
        B.V.assign(2 * nf, 0.0);
        for (int q = 0; q < 2; ++q)
            for (int t = 0; t < nf; ++t) {
                A.V[q * nf + t] = sv * V[q * nf + t];
                B.V[q * nf + other(t)] = sv * V[q * nf + t];
            }
    }
    if (Th) {
        A.Th.assign(Th, Th + 2 * nf);
        B.Th.assign(2 * nf, 0.0);
        for (int q = 0; q < 2; ++q)
            for (int t = 0; t < nf; ++t) B.Th[q * nf + other(t)] = Th[q * nf + t];
    }
    set_time_fn(time_fn, tp, A.jtf);
    B.jtf = A.jtf;
    return SBPE_OK;
}

sbpe_status sbpe_set_forcing(sbpe_ctx_t c, int block, const double* F, int time_fn, const double* tp) {
    sbpe_status s = check_face(c, block, 0);
    if (s) return s;
    if (time_fn < SBPE_TIME_ZERO || time_fn > SBPE_TIME_RICKER) return fail(c, SBPE_EINVAL, "bad time function");
    HostBlock& B = c->blocks[block];
    if (F) B.F.assign(F, F + 2 * B.np());
    else B.F.clear();
    set_time_fn(time_fn, tp, B.ftf);
    return SBPE_OK;
}

sbpe_status sbpe_add_source(sbpe_ctx_t c, int block, double x1, double x2, double f1, double f2, double amp,
                            double peak_hz, double t0) {
    sbpe_status s = check_face(c, block, 0);
    if (s) return s;
    if (!(x1 >= 0 && x1 <= 1 && x2 >= 0 && x2 <= 1)) return fail(c, SBPE_EINVAL, "source outside [0,1]^2");
    c->sources.push_back(Source{block, x1, x2, f1, f2, amp, peak_hz, t0});
    return SBPE_OK;
}

sbpe_status sbpe_add_receivers(sbpe_ctx_t c, int block, int n, const double* x1, const double* x2) {
    sbpe_status s = check_face(c, block, 0);
    if (s) return s;
    if (n < 0 || (n > 0 && (!x1 || !x2))) return fail(c, SBPE_EINVAL, "bad receiver arrays");
    for (int k = 0; k < n; ++k)
        if (!(x1[k] >= 0 && x1[k] <= 1 && x2[k] >= 0 && x2[k] <= 1))
            return fail(c, SBPE_EINVAL, "receiver outside [0,1]^2");
    for (int k = 0; k < n; ++k) c->receivers.push_back(Receiver{block, x1[k], x2[k]});
    return SBPE_OK;
}

// ------------------------------------------------- assembled frame operator
// Probe the frame kernel (the definition of the frame rows) with coloured unit
// fields: colour (i mod P, j mod P) per block and component, so that every
// frame row sees at most one probed point of each colour.  No frame stencil
// of the narrow operator, including the interface terms that reach the
// partner block, spans more than 9 points in either direction (P = 9).  The
// wide operator's closure rows reach one point further (row 5 of order 4
// couples points 0 .. 9 through D_1 b D_1), so it is probed with P = 11,
// whose window (offsets -5 .. 5) holds every row.  Two probes with constant
// fields give the row sums.  The result is checked against the frame kernel
// on a random field.
static int probe_window(int i, int n, int color, int P, int r0) {
    const int back = (P - 1) / 2;
    int lo = i < r0 ? 0 : (i > n - 1 - r0 ? n - P : i - back);
    lo = std::max(0, std::min(lo, std::max(0, n - P)));
    const int p = lo + ((color - lo % P) % P + P) % P;
    return p < n ? p : -1;
}

static sbpe_status assemble_frame(sbpe_ctx* c) {
    // order 6: closure rows reach columns 0..11, so every frame row fits a
    // window of 13 (offsets -6 .. 6 away from the ends)
    const int P = c->order == 6 ? 13 : (c->op == SBPE_OP_WIDE && c->order == 4) ? 11 : 9;
    const int R = frame_of(c->order);
    const int r0 = r0_of(c->order);
    // points next to a face that the displacement / interface SAT reaches (the
    // nonzeros of the first D1 row)
    const int reach = c->order == 6 ? 6 : c->order == 4 ? 4 : 2;
    const int nb = (int)c->blocks.size();
    if (nb > MAX_APPLY_BLOCKS) return SBPE_OK;     // general frame kernel
    const size_t es = esize(c);
    std::vector<void*> X(nb, nullptr), Y(nb, nullptr), G(nb, nullptr), Hh(nb, nullptr);
    sbpe_status st = SBPE_OK;
    auto cleanup = [&]() {
        for (int b = 0; b < nb; ++b) {
            dfree(c, X[b]);
            dfree(c, Y[b]);
            dfree(c, G[b]);
            (void)hipHostFree(Hh[b]);
        }
    };
    for (int b = 0; b < nb; ++b) {
        const long np = c->blocks[b].np();
        const int fn = c->desc[b].frame_n;
        if (dmalloc(c, &X[b], 2 * np * es) != hipSuccess || dmalloc(c, &Y[b], 2 * np * es) != hipSuccess ||
            dmalloc(c, &G[b], 2 * (size_t)std::max(fn, 1) * es) != hipSuccess ||
            hipHostMalloc(&Hh[b], 2 * (size_t)std::max(fn, 1) * es) != hipSuccess) {
            cleanup();
            return fail(c, SBPE_ENOMEM, "frame operator assembly buffers");
        }
    }
    PassArgs pa = base_args(c);
    pa.pass = PASS_APPLY;
    pa.homogeneous = 1;
    for (int b = 0; b < nb; ++b) {
        pa.in[b] = X[b];
        pa.out[b] = Y[b];
    }
    auto val = [&](int b, long idx) -> double {
        return c->dtype == SBPE_F64 ? static_cast<double*>(Hh[b])[idx] : (double)static_cast<float*>(Hh[b])[idx];
    };
    // Probes: for every block bp, component and colour (cx, cy), unit vectors
    // of that colour in block bp (zero elsewhere), the frame kernel, and the
    // frame outputs of every block gathered into G[b] and copied to slice pi
    // of a pinned host buffer per block; then the two constant probes (row
    // sums).  The stream is synchronised every PROBE_CHUNK probes, so at most
    // that many probes (a few hundred small launches) are in flight, and the
    // device holds only the probe, result and gather buffers of each block.
    const int NPC = nb * 2 * P * P;
    const int NPR = NPC + 2;
    constexpr int PROBE_CHUNK = 32;
    std::vector<void*> Ha(nb, nullptr);
    std::vector<size_t> Hbytes(nb, 0);
    auto cleanup_all = [&]() {
        for (int b = 0; b < nb; ++b) (void)hipHostFree(Ha[b]);
        cleanup();
    };
    for (int b = 0; b < nb; ++b) {
        Hbytes[b] = (size_t)NPR * 2 * (size_t)std::max(c->desc[b].frame_n, 1) * es;
        if (hipHostMalloc(&Ha[b], Hbytes[b], hipHostMallocDefault) != hipSuccess) {
            Ha[b] = nullptr;
            cleanup_all();
            return fail(c, SBPE_ENOMEM, "frame operator assembly: pinned host buffers");
        }
    }
    auto probe = [&](int pi, int bp, int comp, int cx, int cy, int period) -> sbpe_status {
        for (int b = 0; b < nb; ++b) {
            const HostBlock& H = c->blocks[b];
            const int e = launch_probe_fill(c->dtype, X[b], H.n1, H.n2, (bp < 0 || bp == b) ? comp : -1, cx, cy,
                                            period, c->stream);
            if (e) return fail(c, SBPE_EHIP, std::string("probe fill: ") + hip_error_string(e));
        }
        int e = launch_frame(c->dtype, c->order, pa, c->total_frame_wg, c->stream);
        if (e) return fail(c, SBPE_EHIP, std::string("probe frame: ") + hip_error_string(e));
        for (int b = 0; b < nb; ++b) {
            const HostBlock& H = c->blocks[b];
            const int fn = c->desc[b].frame_n;
            const size_t slice = 2 * (size_t)fn * es;
            if ((size_t)(pi + 1) * slice > Hbytes[b]) return fail(c, SBPE_EINVAL, "probe slice out of range");
            e = launch_frame_gather(c->dtype, Y[b], H.n1, H.n2, R, fn, G[b], c->stream);
            if (e) return fail(c, SBPE_EHIP, std::string("probe gather: ") + hip_error_string(e));
            if (fn > 0 && hipMemcpyAsync(static_cast<char*>(Ha[b]) + (size_t)pi * slice, G[b], slice,
                                         hipMemcpyDeviceToHost, c->stream) != hipSuccess)
                return fail(c, SBPE_EHIP, "frame operator probe copy");
        }
        if ((pi + 1) % PROBE_CHUNK == 0 && hipStreamSynchronize(c->stream) != hipSuccess)
            return fail(c, SBPE_EHIP, "frame operator probes");
        return SBPE_OK;
    };
    {
        int pi = 0;
        for (int bp = 0; bp < nb && !st; ++bp)
            for (int comp = 0; comp < 2 && !st; ++comp)
                for (int cy = 0; cy < P && !st; ++cy)
                    for (int cx = 0; cx < P && !st; ++cx) st = probe(pi++, bp, comp, cx, cy, P);
        for (int comp = 0; comp < 2 && !st; ++comp) st = probe(NPC + comp, -1, comp, 0, 0, 0);
        if (!st && hipStreamSynchronize(c->stream) != hipSuccess) st = fail(c, SBPE_EHIP, "frame operator probes");
        if (st) {
            (void)hipStreamSynchronize(c->stream);
            cleanup_all();
            return st;
        }
    }
    // value of frame row r (2 k + q) of block b in probe pi
    auto hv = [&](int b, int pi, long r) -> double {
        const size_t idx = (size_t)pi * 2 * (size_t)c->desc[b].frame_n + (size_t)r;
        return c->dtype == SBPE_F64 ? static_cast<const double*>(Ha[b])[idx]
                                    : (double)static_cast<const float*>(Ha[b])[idx];
    };
    // column of the unit vector of probe pi that row (b; i, j) sees, or false
    // if none of its window does (a row reaching beyond the probing period)
    auto column = [&](int b, int i, int j, int pi, int& col) -> bool {
        const int bp = pi / (2 * P * P), comp = (pi / (P * P)) % 2, cy = (pi / P) % P, cx = pi % P;
        const HostBlock& H = c->blocks[b];
        if (b == bp) {
            const int ii = probe_window(i, H.n1, cx, P, r0), jj = probe_window(j, H.n2, cy, P, r0);
            if (ii < 0 || jj < 0) return false;
            col = 2 * (jj * H.n1 + ii) + comp;
            return true;
        }
        const HostBlock& Pb = c->blocks[bp];
        for (int f = 0; f < 4; ++f) {
            const HostFace& F = H.face[f];
            if (F.kind != BC_INTERFACE || F.partner != bp) continue;
            const int dn = f == 0 ? i : f == 1 ? H.n1 - 1 - i : f == 2 ? j : H.n2 - 1 - j;
            if (dn >= reach) continue;
            const int t = f < 2 ? j : i;
            const int nf = f < 2 ? H.n2 : H.n1;
            const int tp = F.reversed ? nf - 1 - t : t;
            int ip, jp;
            if (F.pface < 2) {
                ip = F.pface == 0 ? 0 : Pb.n1 - 1;
                jp = tp;
            } else {
                ip = tp;
                jp = F.pface == 2 ? 0 : Pb.n2 - 1;
            }
            const int ii = probe_window(ip, Pb.n1, cx, P, r0), jj = probe_window(jp, Pb.n2, cy, P, r0);
            if (ii >= 0 && jj >= 0) {
                col = -1 - ((f << 29) | (comp << 28) | (jj * Pb.n1 + ii));
                return true;
            }
        }
        return false;
    };
    // CSR per block: count the nonzeros of each row, then fill each row in
    // probe order and sort it by column
    bool bad = false;
    for (int b = 0; b < nb && !bad; ++b) {
        HostBlock& H = c->blocks[b];
        const int fn = c->desc[b].frame_n;
        const long nr = 2L * fn;
        std::vector<int> rp(nr + 1, 0);
#pragma omp parallel for schedule(static)
        for (long r = 0; r < nr; ++r) {
            int cnt = 0;
            for (int pi = 0; pi < NPC; ++pi) cnt += hv(b, pi, r) != 0.0;
            rp[r + 1] = cnt;
        }
        for (long r = 0; r < nr; ++r) rp[r + 1] += rp[r];
        std::vector<int> cl(std::max(rp[nr], 1), 0);
        std::vector<double> vv(std::max(rp[nr], 1), 0.0);
        std::vector<double> rs(4 * (size_t)std::max(fn, 1), 0.0);
#pragma omp parallel
        {
            std::vector<std::pair<int, double>> row;
#pragma omp for schedule(static)
            for (long r = 0; r < nr; ++r) {
                const int k = (int)(r / 2);
                int i, j;
                frame_ij(k, H.n1, H.n2, R, i, j);
                row.clear();
                for (int pi = 0; pi < NPC; ++pi) {
                    const double v = hv(b, pi, r);
                    if (v == 0.0) continue;
                    int col = 0;
                    if (!column(b, i, j, pi, col)) {
#pragma omp critical
                        bad = true;
                        continue;
                    }
                    row.emplace_back(col, v);
                }
                std::sort(row.begin(), row.end());
                for (size_t e = 0; e < row.size(); ++e) {
                    cl[rp[r] + e] = row[e].first;
                    vv[rp[r] + e] = row[e].second;
                }
                for (int comp = 0; comp < 2; ++comp) rs[2 * r + comp] = hv(b, NPC + comp, r);
            }
        }
        if (bad) break;
        // 2x2 blocks: the two component rows of point k (rows 2k, 2k + 1)
        // merged by neighbouring point; block e holds the column of its
        // point's first component (a partner point's code with the component
        // bit clear) and the values K[row][component] at 4e + 2 row + component
        auto bkey = [](int col) { return col >= 0 ? col >> 1 : -1 - ((-1 - col) & ~(1 << 28)); };
        auto bcomp = [](int col) { return col >= 0 ? col & 1 : ((-1 - col) >> 28) & 1; };
        std::vector<int> bpt(fn + 1, 0);
#pragma omp parallel
        {
            std::vector<int> keys;
#pragma omp for schedule(static)
            for (long k = 0; k < fn; ++k) {
                keys.clear();
                for (int e = rp[2 * k]; e < rp[2 * k + 2]; ++e) keys.push_back(bkey(cl[e]));
                std::sort(keys.begin(), keys.end());
                bpt[k + 1] = (int)(std::unique(keys.begin(), keys.end()) - keys.begin());
            }
        }
        for (long k = 0; k < fn; ++k) bpt[k + 1] += bpt[k];
        std::vector<int> bcl(std::max(bpt[fn], 1), 0);
        std::vector<double> bvv(4 * (size_t)std::max(bpt[fn], 1), 0.0);
#pragma omp parallel
        {
            std::vector<int> keys;
#pragma omp for schedule(static)
            for (long k = 0; k < fn; ++k) {
                keys.clear();
                for (int e = rp[2 * k]; e < rp[2 * k + 2]; ++e) keys.push_back(bkey(cl[e]));
                std::sort(keys.begin(), keys.end());
                keys.erase(std::unique(keys.begin(), keys.end()), keys.end());
                for (size_t m = 0; m < keys.size(); ++m) bcl[bpt[k] + m] = keys[m];
                for (int r = 0; r < 2; ++r)
                    for (int e = rp[2 * k + r]; e < rp[2 * k + r + 1]; ++e) {
                        const long m = std::lower_bound(keys.begin(), keys.end(), bkey(cl[e])) - keys.begin();
                        bvv[4 * (size_t)(bpt[k] + m) + 2 * r + bcomp(cl[e])] += vv[e];
                    }
            }
        }
        if (dmalloc(c, &H.d_fr_rowptr, bpt.size() * sizeof(int)) != hipSuccess ||
            dmalloc(c, &H.d_fr_col, bcl.size() * sizeof(int)) != hipSuccess) {
            cleanup_all();
            return fail(c, SBPE_ENOMEM, "frame operator");
        }
        HIPCHECK(c, hipMemcpy(H.d_fr_rowptr, bpt.data(), bpt.size() * sizeof(int), hipMemcpyHostToDevice));
        HIPCHECK(c, hipMemcpy(H.d_fr_col, bcl.data(), bcl.size() * sizeof(int), hipMemcpyHostToDevice));
        st = upload(c, bvv, &H.d_fr_val);
        if (!st) st = upload(c, rs, &H.d_fr_rsum);
        if (st) {
            cleanup_all();
            return st;
        }
        BlockDesc& D = c->desc[b];
        D.fr_rowptr = H.d_fr_rowptr;
        D.fr_col = H.d_fr_col;
        D.fr_val = H.d_fr_val;
        D.fr_rsum = H.d_fr_rsum;
    }
    for (int b = 0; b < nb; ++b) (void)hipHostFree(Ha[b]);
    Ha.assign(nb, nullptr);
    if (bad) {
        cleanup();
        return fail(c, SBPE_EHIP, "frame operator assembly: a frame row reaches beyond the probe window");
    }
    HIPCHECK(c, hipMemcpy(c->d_desc, c->desc.data(), c->desc.size() * sizeof(BlockDesc), hipMemcpyHostToDevice));
    // check against the frame kernel on a random field
    {
        std::vector<std::vector<double>> ref(nb), got(nb);
        unsigned long long sd = 0x9E3779B97F4A7C15ull;
        for (int b = 0; b < nb; ++b) {
            const long np = c->blocks[b].np();
            std::vector<double> r(2 * np);
            for (auto& x : r) {
                sd ^= sd << 13;
                sd ^= sd >> 7;
                sd ^= sd << 17;
                x = (double)(sd >> 11) * (1.0 / 9007199254740992.0) - 0.5;
            }
            void* tmp = nullptr;
            st = upload(c, r, &tmp);
            if (st) {
                cleanup();
                return st;
            }
            HIPCHECK(c, hipMemcpy(X[b], tmp, 2 * np * es, hipMemcpyDeviceToDevice));
            dfree(c, tmp);
        }
        double scale = 0.0, err = 0.0;
        for (int pass = 0; pass < 2; ++pass) {
            const int e = pass == 0 ? launch_frame(c->dtype, c->order, pa, c->total_frame_wg, c->stream)
                                    : launch_frame_sp(c->dtype, c->order, pa, c->total_frame_wg, c->stream);
            if (e) {
                cleanup();
                return fail(c, SBPE_EHIP, std::string("frame operator check: ") + hip_error_string(e));
            }
            for (int b = 0; b < nb; ++b) {
                const HostBlock& H = c->blocks[b];
                const int fn = c->desc[b].frame_n;
                if (launch_frame_gather(c->dtype, Y[b], H.n1, H.n2, R, fn, G[b], c->stream)) {
                    cleanup();
                    return fail(c, SBPE_EHIP, "frame operator check gather");
                }
                HIPCHECK(c, hipMemcpyAsync(Hh[b], G[b], 2 * (size_t)fn * es, hipMemcpyDeviceToHost, c->stream));
                HIPCHECK(c, hipStreamSynchronize(c->stream));
                auto& dst = pass == 0 ? ref[b] : got[b];
                dst.resize(2 * (size_t)fn);
                for (size_t k = 0; k < dst.size(); ++k) dst[k] = val(b, (long)k);
            }
        }
        // FP64: max norm; FP32: relative L2 over the frame rows, the norm of
        // the library's FP32 accuracy target (rounding of the probed entries
        // and the two summation orders differ by a few units in the last place
        // per row, which the max over ~10^5 rows would amplify)
        double ss_ref = 0.0, ss_err = 0.0;
        for (int b = 0; b < nb; ++b)
            for (size_t k = 0; k < ref[b].size(); ++k) {
                const double d = ref[b][k] - got[b][k];
                scale = std::max(scale, std::fabs(ref[b][k]));
                err = std::max(err, std::fabs(d));
                ss_ref += ref[b][k] * ref[b][k];
                ss_err += d * d;
            }
        const double rel = c->dtype == SBPE_F64 ? err / std::max(scale, 1e-300)
                                                : std::sqrt(ss_err / std::max(ss_ref, 1e-300));
        c->frame_check = rel;
        const double tol = c->dtype == SBPE_F64 ? 1e-11 : 1e-5;
        if (!(rel <= tol)) {
            cleanup();
            char buf[160];
            std::snprintf(buf, sizeof buf, "frame operator assembly check failed: %.3e relative", rel);
            return fail(c, SBPE_EHIP, buf);
        }
    }
    cleanup();
    c->frame_sp = true;
    return SBPE_OK;
}

sbpe_status sbpe_finalize(sbpe_ctx_t c) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail(c, SBPE_ESTATE, "context already finalized");
    if (c->blocks.empty()) return fail(c, SBPE_ESTATE, "no blocks");
    // dissipative terms: traction or Robin faces only; they are applied with
    // the assembled frame operator (at most MAX_APPLY_BLOCKS blocks)
    c->dissipative = false;
    for (const auto& B : c->blocks)
        for (int f = 0; f < 4; ++f) {
            if (B.face[f].Dv.empty()) continue;
            if (B.face[f].kind != BC_TRACTION && B.face[f].kind != BC_ROBIN)
                return fail(c, SBPE_EINVAL, "a dissipative term is set on a face that is no longer traction or Robin");
            c->dissipative = true;
        }
    if (c->dissipative && c->blocks.size() > (size_t)MAX_APPLY_BLOCKS)
        return fail(c, SBPE_EINVAL, "dissipative faces need at most 16 blocks");
    // SBPE_SETUP_TIMING=1 prints the wall time of each setup phase to stderr
    const bool timing = std::getenv("SBPE_SETUP_TIMING") != nullptr;
    const auto t_start = std::chrono::steady_clock::now();
    auto since = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
    double t_metrics = 0, t_upload = 0, t_plan = 0;
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        sbpe_status s = setup_block(c, (int)b);
        if (s) return s;
    }
    t_metrics = since();
    // interfaces: conforming faces must share Jhat (Sec. 6)
    for (size_t b = 0; b < c->blocks.size(); ++b)
        for (int f = 0; f < 4; ++f) {
            const HostFace& F = c->blocks[b].face[f];
            if (F.kind != BC_INTERFACE) continue;
            const HostFace& P = c->blocks[F.partner].face[F.pface];
            const int nf = (int)F.jhat.size();
            for (int t = 0; t < nf; ++t) {
                const double a = F.jhat[t], q = P.jhat[F.reversed ? nf - 1 - t : t];
                if (std::fabs(a - q) > 1e-8 * std::max(a, q))
                    return fail(c, SBPE_EIFACE, "interface faces do not coincide (Jhat differs)");
            }
        }
    if (!c->host_only) {
        if (hipSetDevice(c->device) != hipSuccess) return fail(c, SBPE_EHIP, "hipSetDevice failed");
        for (auto& B : c->blocks) {
            sbpe_status s = upload(c, B.coef, &B.d_coef);
            if (s) return s;
            const long np = B.np();
            if (!B.F.empty()) {
                std::vector<double> JF(2 * np);
                for (long p = 0; p < np; ++p) {
                    JF[p] = B.J[p] * B.F[p];
                    JF[np + p] = B.J[p] * B.F[np + p];
                }
                s = upload(c, JF, &B.d_force);
                if (s) return s;
            }
            if (dmalloc(c, &B.d_a1, 2 * np * esize(c)) != hipSuccess ||
                dmalloc(c, &B.d_a2, 2 * np * esize(c)) != hipSuccess)
                return fail(c, SBPE_ENOMEM, "device allocation failed");
            for (int f = 0; f < 4; ++f) {
                HostFace& F = B.face[f];
                const int nf = B.nf(f);
                const int a = f >> 1;
                const double w = (a == 0 ? B.h1 : B.h2) * norm_weight(c->order, a == 0 ? B.n1 : B.n2, 0);
                if (!F.g.empty() && (F.kind == BC_TRACTION || F.kind == BC_ROBIN || F.kind == BC_DISPLACEMENT)) {
                    std::vector<double> g(F.g);
                    if (F.kind != BC_DISPLACEMENT)
                        for (int t = 0; t < nf; ++t) {
                            g[t] *= F.jhat[t] / w;
                            g[nf + t] *= F.jhat[t] / w;
                        }
                    s = upload(c, g, &B.d_face[f][0]);
                    if (s) return s;
                }
                if (F.kind == BC_ROBIN) {
                    std::vector<double> U(F.U);
                    for (int k = 0; k < 4; ++k)
                        for (int t = 0; t < nf; ++t) U[k * nf + t] *= F.jhat[t] / w;
                    s = upload(c, U, &B.d_face[f][1]);
                    if (s) return s;
                }
                if (!F.Dv.empty()) {
                    std::vector<double> dv(F.Dv);
                    for (int k = 0; k < 4; ++k)
                        for (int t = 0; t < nf; ++t) dv[k * nf + t] *= F.jhat[t] / w;
                    s = upload(c, dv, &B.d_face[f][4]);
                    if (s) return s;
                }
                if (F.kind == BC_INTERFACE && !F.V.empty()) {
                    s = upload(c, F.V, &B.d_face[f][2]);
                    if (s) return s;
                }
                if (F.kind == BC_INTERFACE && !F.Th.empty()) {
                    // the traction-jump SAT adds Jhat H_f Theta / 2 at the face row: Jhat Theta / (2 w)
                    std::vector<double> th(F.Th);
                    for (int t = 0; t < nf; ++t) {
                        th[t] *= 0.5 * F.jhat[t] / w;
                        th[nf + t] *= 0.5 * F.jhat[t] / w;
                    }
                    s = upload(c, th, &B.d_face[f][3]);
                    if (s) return s;
                }
            }
        }
    }
    t_upload = since();
    sbpe_status s = build_plan(c);
    if (s) return s;
    t_plan = since();
    if (!c->host_only) {
        // SBPE_FRAME=stencil leaves the frame operator unassembled: every sweep
        // then runs the frame band with the stencil kernel on the second
        // stream (a measurement switch; contexts with dissipative faces, which
        // only the assembled operator applies, always assemble it)
        const char* fe = std::getenv("SBPE_FRAME");
        const bool stencil = fe && std::strcmp(fe, "stencil") == 0 && !c->dissipative;
        if (!stencil) {
            s = assemble_frame(c);
            if (s) return s;
        }
    }
    if (timing)
        std::fprintf(stderr, "sbpe_finalize: metrics and c %.4f s, uploads %.4f s, plan %.4f s, frame operator %.4f s\n",
                     t_metrics, t_upload - t_metrics, t_plan - t_upload, since() - t_plan);
    c->finalized = true;
    return SBPE_OK;
}

sbpe_status sbpe_dt_cfl(sbpe_ctx_t c, double cfl, double* dt) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail(c, SBPE_ESTATE, "context not finalized");
    if (!dt || !(cfl > 0)) return fail(c, SBPE_EINVAL, "bad arguments");
    double best = INFINITY;
    for (const auto& B : c->blocks) {
        const double v2 = block_vmax2(B);
        best = std::min(best, std::min(B.h1, B.h2) / std::sqrt(v2));
    }
    *dt = cfl * best;
    return SBPE_OK;
}

sbpe_status sbpe_block_size(sbpe_ctx_t c, int block, int* n1, int* n2) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (block < 0 || block >= (int)c->blocks.size()) return fail(c, SBPE_EINVAL, "no such block");
    if (n1) *n1 = c->blocks[block].n1;
    if (n2) *n2 = c->blocks[block].n2;
    return SBPE_OK;
}

sbpe_status sbpe_apply(sbpe_ctx_t c, const void* const* u, void* const* a, double t, int homogeneous) {
    if (c && c->batch) return fail(c, SBPE_ESTATE, "context is a member of a batch");
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    const int nb = (int)c->blocks.size();
    if (nb > MAX_APPLY_BLOCKS) return fail(c, SBPE_EINVAL, "sbpe_apply supports at most 16 blocks");
    if (!u || !a) return fail(c, SBPE_EINVAL, "NULL pointer array");
    for (int b = 0; b < nb; ++b) {
        if (!u[b] || !a[b]) return fail(c, SBPE_EINVAL, "NULL block pointer");
        for (int q = 0; q < nb; ++q)
            if (a[b] == u[q]) return fail(c, SBPE_EINVAL, "output aliases an input");
    }
    if (!homogeneous) {
        sbpe_status s2 = fill_tau(c, 1, t, 0.0);
        if (s2) return s2;
    }
    {
        sbpe_status s2 = refresh_desc(c, c->desc.empty() ? 0.0 : c->desc[0].dt, c->d_tau);
        if (s2) return s2;
    }
    PassArgs pa = base_args(c);
    pa.pass = PASS_APPLY;
    pa.homogeneous = homogeneous ? 1 : 0;
    pa.wa[0] = homogeneous ? 0.0 : 1.0;
    for (int b = 0; b < nb; ++b) {
        pa.in[b] = u[b];
        pa.out[b] = a[b];
    }
    sbpe_status s2 = run_pass(c, pa);
    if (s2) return s2;
    return finish_passes(c);
}

sbpe_status sbpe_bind_state(sbpe_ctx_t c, void* const* u, void* const* v, double t) {
    if (c && c->batch) return fail(c, SBPE_ESTATE, "context is a member of a batch");
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (!u || !v) return fail(c, SBPE_EINVAL, "NULL pointer array");
    for (size_t b = 0; b < c->blocks.size(); ++b)
        if (!u[b] || !v[b] || u[b] == v[b]) return fail(c, SBPE_EINVAL, "bad state pointers");
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        c->blocks[b].u = u[b];
        c->blocks[b].v = v[b];
    }
    s = sync_desc(c);
    if (s) return s;
    c->bound = true;
    c->t = t;
    c->rec_steps = 0;
    return SBPE_OK;
}

static sbpe_status energy_now(sbpe_ctx* c, double* eps) {
    PassArgs pa = base_args(c);
    pa.pass = PASS_APPLY;
    pa.homogeneous = 1;
    for (size_t b = 0; b < c->blocks.size(); ++b) {
        pa.in[b] = c->blocks[b].u;
        pa.out[b] = c->blocks[b].d_a1;
    }
    sbpe_status s = run_pass(c, pa);
    if (s) return s;
    s = finish_passes(c);
    if (s) return s;
    const int e = launch_energy(c->dtype, c->order, c->d_desc, (int)c->blocks.size(), c->d_epart, c->npartial,
                                c->d_eout, c->stream);
    if (e != 0) return fail(c, SBPE_EHIP, std::string("energy launch: ") + hip_error_string(e));
    HIPCHECK(c, hipMemcpyAsync(eps, c->d_eout, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return SBPE_OK;
}

sbpe_status sbpe_energy(sbpe_ctx_t c, double* eps) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (!c->bound) return fail(c, SBPE_ESTATE, "no state bound");
    if (!eps) return fail(c, SBPE_EINVAL, "NULL eps");
    return energy_now(c, eps);
}

sbpe_status sbpe_set_energy_guard(sbpe_ctx_t c, int every, double rel_growth) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (every < 0 || !(rel_growth >= 0)) return fail(c, SBPE_EINVAL, "bad guard parameters");
    c->guard_every = every;
    c->guard_growth = rel_growth;
    return SBPE_OK;
}

// The steps of an advance call once the receiver
// record holds them: the time functions of every step tabulated into `tau`
// (at least nsteps * nitems * 3 doubles), then two sweeps per step.
static sbpe_status advance_steps(sbpe_ctx* c, int nsteps, double dt, double* tau) {
    sbpe_status s;
    double e0 = 0.0;
    if (c->guard_every > 0) {
        s = energy_now(c, &e0);
        if (s) return s;
    }
    if (nsteps > 0) {
        const int e = launch_tau(c->d_items, c->nitems, nsteps, c->t, dt, tau, c->stream);
        if (e != 0) return fail(c, SBPE_EHIP, std::string("tau launch: ") + hip_error_string(e));
        s = refresh_desc(c, dt, tau);
        if (s) return s;
    }
    for (int k = 0; k < nsteps; ++k) {
        PassArgs p1 = base_args(c);
        p1.pass = PASS_RK1;
        p1.step = k;
        p1.rec_base = (int)c->rec_steps;
        p1.wa[0] = 1.0;     // tau(t)
        p1.wb[1] = 1.0;     // tau(t + dt/2)
        s = run_pass(c, p1);
        if (s) return s;
        PassArgs p2 = p1;
        p2.pass = PASS_RK2;
        // 2/dt^2 (tau(t) - 2 tau(t + dt/2) + tau(t + dt)); the kernels apply 2/dt^2
        p2.wa[0] = p2.wa[1] = p2.wa[2] = 0.0;
        p2.wb[0] = 1.0;
        p2.wb[1] = -2.0;
        p2.wb[2] = 1.0;
        s = run_pass(c, p2);
        if (s) return s;
        c->t += dt;
        if (c->guard_every > 0 && (k + 1) % c->guard_every == 0) {
            s = finish_passes(c);
            if (s) return s;
            double e = 0.0;
            s = energy_now(c, &e);
            if (s) return s;
            if (!std::isfinite(e) || e > (1.0 + c->guard_growth) * e0) {
                c->rec_steps += k + 1;
                char buf[160];
                std::snprintf(buf, sizeof buf, "energy guard: energy %.6e after step %d exceeds %.6e", e, k + 1,
                              (1.0 + c->guard_growth) * e0);
                return fail(c, SBPE_EUNSTABLE, buf);
            }
        }
    }
    c->rec_steps += nsteps;
    return finish_passes(c);
}

static sbpe_status check_advance(sbpe_ctx* c, int nsteps, double dt) {
    if (c && c->batch) return fail(c, SBPE_ESTATE, "context is a member of a batch");
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (!c->bound) return fail(c, SBPE_ESTATE, "no state bound");
    if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail(c, SBPE_EINVAL, "bad nsteps or dt");
    return SBPE_OK;
}

sbpe_status sbpe_advance(sbpe_ctx_t c, int nsteps, double dt) {
    sbpe_status s = check_advance(c, nsteps, dt);
    if (s) return s;
    s = grow_receivers(c, c->rec_steps + nsteps);
    if (s) return s;
    if (nsteps > 0) {
        s = grow_tau(c, nsteps);
        if (s) return s;
    }
    return advance_steps(c, nsteps, dt, c->d_tau);
}

sbpe_status sbpe_advance_noalloc(sbpe_ctx_t c, int nsteps, double dt) {
    sbpe_status s = check_advance(c, nsteps, dt);
    if (s) return s;
    const long nrec = (long)c->receivers.size();
    if (nrec > 0 && c->rec_steps + nsteps > c->rec_cap) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "receiver record holds %ld more steps, %d asked: sbpe_reserve_steps first",
                      c->rec_cap - c->rec_steps, nsteps);
        return fail(c, SBPE_ESTATE, buf);
    }
    const size_t per_step = (size_t)c->nitems * 3;
    if ((size_t)nsteps * per_step > NOALLOC_SCRATCH_DOUBLES) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "at most %zu steps per call fit the no-allocation time-function table (%d asked)",
                      NOALLOC_SCRATCH_DOUBLES / std::max<size_t>(per_step, 1), nsteps);
        return fail(c, SBPE_EINVAL, buf);
    }
    double* tau = scratch_ptr(c->device);
    if (!tau) return fail(c, SBPE_ESTATE, "no-allocation scratch not set up on this device");
    return advance_steps(c, nsteps, dt, tau);
}

sbpe_status sbpe_reserve_steps(sbpe_ctx_t c, int nsteps) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (nsteps < 0) return fail(c, SBPE_EINVAL, "negative nsteps");
    s = grow_tau(c, nsteps);
    if (s) return s;
    return grow_receivers(c, c->rec_steps + nsteps);
}

sbpe_status sbpe_device_bytes(sbpe_ctx_t c, long long* held, long long* peak) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (held) *held = (long long)c->dev_held;
    if (peak) *peak = (long long)c->dev_peak;
    return SBPE_OK;
}

sbpe_status sbpe_get_time(sbpe_ctx_t c, double* t) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (!t) return fail(c, SBPE_EINVAL, "NULL t");
    *t = c->t;
    return SBPE_OK;
}

sbpe_status sbpe_read_receivers(sbpe_ctx_t c, double* out, int max_steps, int* nsteps_out) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    const long nrec = (long)c->receivers.size();
    const long n = std::min<long>(c->rec_steps, std::max(max_steps, 0));
    if (nsteps_out) *nsteps_out = (int)n;
    if (nrec == 0 || n == 0 || !out) return SBPE_OK;
    std::vector<double> raw(n * nrec * 32);
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(raw.data(), c->d_rec, raw.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (long st = 0; st < n; ++st)
        for (long r = 0; r < nrec; ++r)
            for (int cmp = 0; cmp < 2; ++cmp) {
                double acc = 0.0;
                for (int sl = 0; sl < 16; ++sl) acc += raw[((st * nrec + r) * 16 + sl) * 2 + cmp];
                out[(st * nrec + r) * 2 + cmp] = acc;
            }
    return SBPE_OK;
}

sbpe_status sbpe_synchronize(sbpe_ctx_t c) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c->host_only) return SBPE_OK;
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    return SBPE_OK;
}

sbpe_status sbpe_set_kernel_timing(sbpe_ctx_t c, int enable) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (!enable) {
        s = collect_timing(c);
        if (s) return s;
    }
    c->timing = enable != 0;
    return SBPE_OK;
}

sbpe_status sbpe_get_kernel_timing(sbpe_ctx_t c, double* ms_avg, int* count) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    s = collect_timing(c);
    if (s) return s;
    for (int k = 0; k < 6; ++k) {
        if (ms_avg) ms_avg[k] = c->t_cnt[k] ? c->t_sum[k] / c->t_cnt[k] : 0.0;
        if (count) count[k] = c->t_cnt[k];
        c->t_sum[k] = 0.0;
        c->t_cnt[k] = 0;
    }
    return SBPE_OK;
}

sbpe_status sbpe_plan_info(sbpe_ctx_t c, long long* info) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail(c, SBPE_ESTATE, "context not finalized");
    if (!info) return fail(c, SBPE_EINVAL, "NULL info");
    const int R = frame_of(c->order);
    long long ip = 0, fp = 0;
    for (const auto& B : c->blocks) {
        ip += (long long)(B.n1 - 2 * R) * (B.n2 - 2 * R);
        fp += (long long)B.n1 * B.n2 - (long long)(B.n1 - 2 * R) * (B.n2 - 2 * R);
    }
    info[0] = ip;
    info[1] = fp;
    info[2] = c->total_tiles;
    info[3] = c->total_frame_wg;
    info[4] = R;
    info[5] = (c->frame_sp && sweep_fused(c->total_tiles)) ? 1 : 0;
    return SBPE_OK;
}

sbpe_status sbpe_host_d1_line(int order, int n, const double* u, double* out) {
    if ((order != 2 && order != 4 && order != 6) || n < min_points(order) || !u || !out)
        return fail(nullptr, SBPE_EINVAL, "bad arguments");
    d1_apply(order, n, 1.0 / (n - 1), u, 1, out, 1);
    return SBPE_OK;
}

sbpe_status sbpe_host_d2fc_line(int order, int n, const double* b, const double* u, double* out) {
    if ((order != 2 && order != 4 && order != 6) || n < min_points(order) || !b || !u || !out)
        return fail(nullptr, SBPE_EINVAL, "bad arguments");
    const int R0 = r0_of(order), W = order == 6 ? O6_W : order == 4 ? O4_W : O2_W;
    std::vector<double> T((size_t)R0 * W * W);
    derive_d2_closure(order, T.data());
    const double ih2 = double(n - 1) * double(n - 1);
    for (int r = 0; r < n; ++r) {
        double acc = 0.0;
        if (r >= R0 && r <= n - 1 - R0) {
            if (order == 6) {
                // interior row of h^2 D2(b) in edge form, b and u on offsets -3 .. 3
                const double* B = b + r;
                const double* U = u + r;
                const double k[6] = {
                    11.0 / 360 * (B[-3] + B[0]) - (B[-2] + B[-1]) / 40,
                    -(B[-3] + B[1]) / 20 + 0.3 * B[-1] - 7.0 / 40 * (B[-2] + B[0]),
                    (B[-3] + B[2]) / 40 + 0.3 * (B[-2] + B[1]) + 17.0 / 40 * (B[-1] + B[0]),
                    (B[-2] + B[3]) / 40 + 0.3 * (B[-1] + B[2]) + 17.0 / 40 * (B[0] + B[1]),
                    -(B[-1] + B[3]) / 20 + 0.3 * B[1] - 7.0 / 40 * (B[0] + B[2]),
                    11.0 / 360 * (B[0] + B[3]) - (B[1] + B[2]) / 40};
                const int off[6] = {-3, -2, -1, 1, 2, 3};
                for (int e = 0; e < 6; ++e) acc += k[e] * (U[off[e]] - U[0]);
            } else if (order == 4) {
                const double* B = b + r;
                const double* U = u + r;
                const double km2 = B[-1] / 6 - 0.125 * (B[-2] + B[0]);
                const double km1 = (B[-2] + B[1]) / 6 + 0.5 * (B[-1] + B[0]);
                const double kp1 = (B[-1] + B[2]) / 6 + 0.5 * (B[0] + B[1]);
                const double kp2 = B[1] / 6 - 0.125 * (B[0] + B[2]);
                acc = km2 * (U[-2] - U[0]) + km1 * (U[-1] - U[0]) + kp1 * (U[1] - U[0]) + kp2 * (U[2] - U[0]);
            } else {
                acc = 0.5 * (b[r - 1] + b[r]) * (u[r - 1] - u[r]) + 0.5 * (b[r] + b[r + 1]) * (u[r + 1] - u[r]);
            }
        } else {
            const bool lo = r < R0;
            const int rr = lo ? r : n - 1 - r;
            for (int m = 0; m < W; ++m)
                for (int s = 0; s < W; ++s) {
                    const double tv = T[((size_t)rr * W + m) * W + s];
                    if (tv != 0.0) acc += tv * b[lo ? s : n - 1 - s] * (u[lo ? m : n - 1 - m] - u[r]);
                }
        }
        out[r] = acc * ih2;
    }
    return SBPE_OK;
}

sbpe_status sbpe_get_block_fields(sbpe_ctx_t c, int block, double* c10, double* J, double* jhat) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail(c, SBPE_ESTATE, "context not finalized");
    if (block < 0 || block >= (int)c->blocks.size()) return fail(c, SBPE_EINVAL, "no such block");
    const HostBlock& B = c->blocks[block];
    if (c10) std::copy(B.c10t.begin(), B.c10t.end(), c10);
    if (J) std::copy(B.J.begin(), B.J.end(), J);
    if (jhat) {
        const int m = std::max(B.n1, B.n2);
        for (int f = 0; f < 4; ++f) std::copy(B.face[f].jhat.begin(), B.face[f].jhat.end(), jhat + (size_t)f * m);
    }
    return SBPE_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ batches
// A batch advances the bound states of several finalized contexts with one
// kernel launch per sweep over the union of their blocks (each block carries
// its own time step, time-function table and receiver buffer).  Members join
// and leave between calls to sbpe_batch_advance.
struct BatchMember {
    sbpe_ctx* ctx;
    double dt;
    int remaining;   // steps still to take
    int step0;       // batch step index at which the member joined
    long rec0;       // receiver row of the member at its first batch step
};

struct sbpe_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t side = nullptr;
    hipEvent_t ev_main = nullptr, ev_side = nullptr;
    int dtype = SBPE_F64, order = 4;
    int op = SBPE_OP_NARROW;     // operator of the members (set by the first member of an empty batch)
    std::string err;
    std::vector<BatchMember> members;
    std::vector<BlockDesc> desc;
    BlockDesc* d_desc = nullptr;
    size_t desc_cap = 0;
    int total_tiles = 0, total_frame_wg = 0;
    int step = 0;
    bool dirty = true;
};

static sbpe_status bfail(sbpe_batch* b, sbpe_status code, const std::string& msg) {
    if (b) b->err = msg;
    else g_static_err = msg;
    return code;
}

#define BHIPCHECK(bt, expr)                                                                        \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return bfail(bt, SBPE_EHIP, std::string(#expr ": ") + hipGetErrorString(e_)); \
    } while (0)

extern "C" {

sbpe_status sbpe_batch_create(int device, void* stream, int dtype, int order, sbpe_batch_t* out) {
    if (!out) return bfail(nullptr, SBPE_EINVAL, "out is NULL");
    if (dtype != SBPE_F64 && dtype != SBPE_F32) return bfail(nullptr, SBPE_EINVAL, "bad dtype");
    if (order != 2 && order != 4 && order != 6) return bfail(nullptr, SBPE_EINVAL, "order must be 2, 4 or 6");
    int n = 0;
    if (device < 0 || hipGetDeviceCount(&n) != hipSuccess || device >= n) return bfail(nullptr, SBPE_EHIP, "no such HIP device");
    if (hipSetDevice(device) != hipSuccess) return bfail(nullptr, SBPE_EHIP, "hipSetDevice failed");
    sbpe_batch* b = new sbpe_batch;
    b->device = device;
    b->stream = static_cast<hipStream_t>(stream);
    b->dtype = dtype;
    b->order = order;
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_main, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_side, hipEventDisableTiming) != hipSuccess) {
        delete b;
        return bfail(nullptr, SBPE_EHIP, "stream/event creation failed");
    }
    *out = b;
    return SBPE_OK;
}

sbpe_status sbpe_batch_destroy(sbpe_batch_t b) {
    if (!b) return SBPE_OK;
    (void)hipStreamSynchronize(b->side);
    (void)hipStreamSynchronize(b->stream);
    for (auto& m : b->members) m.ctx->batch = nullptr;
    (void)hipFree(b->d_desc);
    (void)hipEventDestroy(b->ev_main);
    (void)hipEventDestroy(b->ev_side);
    (void)hipStreamDestroy(b->side);
    delete b;
    return SBPE_OK;
}

const char* sbpe_batch_last_error(sbpe_batch_t b) { return b ? b->err.c_str() : g_static_err.c_str(); }

sbpe_status sbpe_batch_add(sbpe_batch_t b, sbpe_ctx_t c, int nsteps, double dt) {
    if (!b || !c) return bfail(b, SBPE_EINVAL, "NULL batch or context");
    if (c->host_only || !c->finalized || !c->bound) return bfail(b, SBPE_ESTATE, "context must be finalized with a bound state");
    if (c->batch) return bfail(b, SBPE_ESTATE, "context already belongs to a batch");
    if (c->device != b->device || c->dtype != b->dtype || c->order != b->order)
        return bfail(b, SBPE_EINVAL, "context device, dtype or order differs from the batch");
    if (!b->members.empty() && c->op != b->op)
        return bfail(b, SBPE_EINVAL, "context operator (narrow or wide) differs from the batch members'");
    if (nsteps <= 0 || !(dt > 0) || !std::isfinite(dt)) return bfail(b, SBPE_EINVAL, "bad nsteps or dt");
    if (!c->frame_sp)
        return bfail(b, SBPE_EINVAL, "batches sweep the assembled frame operator, which this context does not hold");
    // time functions for all its steps, receiver rows for all its steps
    sbpe_status s = fill_tau(c, nsteps, c->t, dt);
    if (s) return bfail(b, s, c->err);
    const long nrec = (long)c->receivers.size();
    const long slots = nrec * 16 * 2;
    if (nrec > 0 && c->rec_steps + nsteps > c->rec_cap) {
        const long cap = c->rec_steps + nsteps;
        double* nd = nullptr;
        if (dmalloc(c, &nd, cap * slots * sizeof(double)) != hipSuccess) return bfail(b, SBPE_ENOMEM, "receiver buffer");
        if (c->d_rec && c->rec_steps > 0)
            BHIPCHECK(b, hipMemcpyAsync(nd, c->d_rec, c->rec_steps * slots * sizeof(double), hipMemcpyDeviceToDevice,
                                        c->stream));
        BHIPCHECK(b, hipStreamSynchronize(c->stream));
        dfree(c, c->d_rec);
        c->d_rec = nd;
        c->rec_cap = cap;
    }
    // the batch streams wait for everything already enqueued on the context
    BHIPCHECK(b, hipEventRecord(c->ev_main, c->stream));
    BHIPCHECK(b, hipStreamWaitEvent(b->stream, c->ev_main, 0));
    BHIPCHECK(b, hipStreamWaitEvent(b->side, c->ev_main, 0));
    c->batch = b;
    if (b->members.empty()) b->op = c->op;
    b->members.push_back(BatchMember{c, dt, nsteps, b->step, c->rec_steps});
    b->dirty = true;
    return SBPE_OK;
}

sbpe_status sbpe_batch_remove(sbpe_batch_t b, sbpe_ctx_t c) {
    if (!b || !c) return bfail(b, SBPE_EINVAL, "NULL batch or context");
    size_t k = 0;
    while (k < b->members.size() && b->members[k].ctx != c) ++k;
    if (k == b->members.size()) return bfail(b, SBPE_EINVAL, "context is not a member");
    // later work on the context's stream waits for the batch's work
    BHIPCHECK(b, hipEventRecord(b->ev_side, b->side));
    BHIPCHECK(b, hipStreamWaitEvent(c->stream, b->ev_side, 0));
    BHIPCHECK(b, hipEventRecord(b->ev_main, b->stream));
    BHIPCHECK(b, hipStreamWaitEvent(c->stream, b->ev_main, 0));
    c->batch = nullptr;
    b->members.erase(b->members.begin() + k);
    b->dirty = true;
    return SBPE_OK;
}

sbpe_status sbpe_batch_remaining(sbpe_batch_t b, sbpe_ctx_t c, int* remaining) {
    if (!b || !c || !remaining) return bfail(b, SBPE_EINVAL, "NULL argument");
    for (auto& m : b->members)
        if (m.ctx == c) {
            *remaining = m.remaining;
            return SBPE_OK;
        }
    return bfail(b, SBPE_EINVAL, "context is not a member");
}

sbpe_status sbpe_batch_info(sbpe_batch_t b, int* members, int* min_remaining, long long* points) {
    if (!b) return bfail(nullptr, SBPE_EINVAL, "NULL batch");
    int mr = 0;
    long long pts = 0;
    for (size_t k = 0; k < b->members.size(); ++k) {
        mr = k == 0 ? b->members[k].remaining : std::min(mr, b->members[k].remaining);
        for (auto& B : b->members[k].ctx->blocks) pts += (long long)B.n1 * B.n2;
    }
    if (members) *members = (int)b->members.size();
    if (min_remaining) *min_remaining = mr;
    if (points) *points = pts;
    return SBPE_OK;
}

}  // extern "C"

// concatenated descriptors of all members (blocks renumbered, launch ranges rebased)
static sbpe_status batch_rebuild(sbpe_batch* b) {
    b->desc.clear();
    int tiles = 0, fwg = 0;
    for (auto& m : b->members) {
        sbpe_ctx* c = m.ctx;
        const int base = (int)b->desc.size();
        const long nrec = (long)c->receivers.size();
        for (size_t k = 0; k < c->desc.size(); ++k) {
            BlockDesc D = c->desc[k];
            D.tile_beg = tiles;
            tiles += D.tiles_x * D.tiles_y;
            D.frame_beg = fwg;
            fwg += D.frame_wg;
            for (int f = 0; f < 4; ++f)
                if (D.face[f].kind == BC_INTERFACE) D.face[f].partner += base;
            D.dt = m.dt;
            D.tau = c->d_tau;
            D.step0 = m.step0;
            D.rec = nrec > 0 ? c->d_rec + m.rec0 * D.rec_stride : nullptr;
            b->desc.push_back(D);
        }
    }
    b->total_tiles = tiles;
    b->total_frame_wg = fwg;
    if (b->desc.empty()) {
        b->dirty = false;
        return SBPE_OK;
    }
    BHIPCHECK(b, hipStreamSynchronize(b->side));
    BHIPCHECK(b, hipStreamSynchronize(b->stream));
    if (b->desc.size() > b->desc_cap) {
        (void)hipFree(b->d_desc);
        b->d_desc = nullptr;
        const size_t cap = std::max(b->desc.size(), 2 * b->desc_cap);
        b->desc_cap = 0;    // a failed allocation leaves no table behind
        if (hipMalloc(&b->d_desc, cap * sizeof(BlockDesc)) != hipSuccess) return bfail(b, SBPE_ENOMEM, "descriptor table");
        b->desc_cap = cap;
    }
    BHIPCHECK(b, hipMemcpy(b->d_desc, b->desc.data(), b->desc.size() * sizeof(BlockDesc), hipMemcpyHostToDevice));
    b->dirty = false;
    return SBPE_OK;
}

// One sweep over every member: a single launch while the tiles are few,
// otherwise the interior tiles on the batch stream and the frame operator on
// the side stream (each waits for the other's previous sweep).  Either way
// every point is evaluated with the arithmetic of a single-context sweep.
static sbpe_status batch_pass(sbpe_batch* b, const PassArgs& a) {
    int e;
    if (sweep_fused(b->total_tiles)) {
        e = launch_pass(b->dtype, b->order, a, b->total_tiles, b->total_frame_wg, b->stream);
    } else {
        BHIPCHECK(b, hipEventRecord(b->ev_main, b->stream));
        BHIPCHECK(b, hipStreamWaitEvent(b->side, b->ev_main, 0));
        BHIPCHECK(b, hipEventRecord(b->ev_side, b->side));
        BHIPCHECK(b, hipStreamWaitEvent(b->stream, b->ev_side, 0));
        e = launch_interior(b->dtype, b->order, a, b->total_tiles, b->stream);
        if (e == 0) e = launch_frame_sp(b->dtype, b->order, a, b->total_frame_wg, b->side);
    }
    if (e != 0) return bfail(b, SBPE_EHIP, std::string("kernel launch: ") + hip_error_string(e));
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_batch_advance(sbpe_batch_t b, int nsteps) {
    if (!b) return bfail(nullptr, SBPE_EINVAL, "NULL batch");
    if (nsteps < 0) return bfail(b, SBPE_EINVAL, "nsteps < 0");
    for (auto& m : b->members)
        if (m.remaining < nsteps) return bfail(b, SBPE_EINVAL, "nsteps exceeds the remaining steps of a member");
    if (b->members.empty() || nsteps == 0) return SBPE_OK;
    if (hipSetDevice(b->device) != hipSuccess) return bfail(b, SBPE_EHIP, "hipSetDevice failed");
    if (b->dirty) {
        sbpe_status s = batch_rebuild(b);
        if (s) return s;
    }
    for (int k = 0; k < nsteps; ++k) {
        PassArgs p1;
        std::memset(&p1, 0, sizeof p1);
        p1.blocks = b->d_desc;
        p1.nblocks = (int)b->desc.size();
        p1.pass = PASS_RK1;
        p1.wide = b->op == SBPE_OP_WIDE ? 1 : 0;
        p1.floop = default_frame_loop(b->dtype);
        p1.step = b->step + k;
        p1.rec_base = 0;
        p1.wa[0] = 1.0;
        p1.wb[1] = 1.0;
        sbpe_status s = batch_pass(b, p1);
        if (s) return s;
        PassArgs p2 = p1;
        p2.pass = PASS_RK2;
        p2.wa[0] = 0.0;
        p2.wb[0] = 1.0;
        p2.wb[1] = -2.0;
        p2.wb[2] = 1.0;
        s = batch_pass(b, p2);
        if (s) return s;
    }
    BHIPCHECK(b, hipEventRecord(b->ev_side, b->side));
    BHIPCHECK(b, hipStreamWaitEvent(b->stream, b->ev_side, 0));
    b->step += nsteps;
    for (auto& m : b->members) {
        m.remaining -= nsteps;
        m.ctx->t += nsteps * m.dt;
        m.ctx->rec_steps += nsteps;
    }
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_batch_synchronize(sbpe_batch_t b) {
    if (!b) return bfail(nullptr, SBPE_EINVAL, "NULL batch");
    BHIPCHECK(b, hipStreamSynchronize(b->side));
    BHIPCHECK(b, hipStreamSynchronize(b->stream));
    return SBPE_OK;
}

// -------------------------------------------------------------- gradients
// Gradient accumulation of nst stages: stage s takes z[s*nb + b], y[s*nb + b],
// a[s*nb + b], alpha[s], and column tcol[s] of the time functions tabulated at
// (t, dt) (columns: t, t + dt/2, t + dt).
static sbpe_status grad_stages(sbpe_ctx* c, int nst, const void* const* z, const void* const* y,
                               const void* const* a, const double* alpha, const int* tcol, double t, double dt,
                               int homogeneous, void* const* gc, void* const* grt) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (c && c->batch) return fail(c, SBPE_ESTATE, "context is a member of a batch");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (c->dissipative)
        return fail(c, SBPE_EINVAL, "coefficient gradients with dissipative faces are not supported (the scheme is not self-adjoint)");
    if (c->order == 6) return fail(c, SBPE_EINVAL, "coefficient gradients are built for orders 2 and 4");
    const int nb = (int)c->blocks.size();
    if (nb > MAX_APPLY_BLOCKS) return fail(c, SBPE_EINVAL, "at most 16 blocks");
    if (!z || !y || !a || !gc || !grt || !alpha) return fail(c, SBPE_EINVAL, "NULL pointer array");
    for (int b = 0; b < nb; ++b) {
        if (!gc[b] || !grt[b]) return fail(c, SBPE_EINVAL, "NULL block pointer");
        for (int st = 0; st < nst; ++st)
            if (!z[st * nb + b] || !y[st * nb + b] || !a[st * nb + b]) return fail(c, SBPE_EINVAL, "NULL block pointer");
        for (int f = 0; f < 4; ++f)
            if (c->blocks[b].face[f].kind == BC_INTERFACE)
                return fail(c, SBPE_EINVAL, "coefficient gradients across interfaces are not supported");
    }
    GradArgs g;
    std::memset(&g, 0, sizeof g);
    for (int b = 0; b < nb; ++b) {
        g.n1[b] = c->blocks[b].n1;
        g.n2[b] = c->blocks[b].n2;
    }
    if (nst > 1) {
        // band partial sums of the stages
        const long need = (long)nst * GRAD_TERMS * grad_band_points(c->order, g.n1, g.n2, nb);
        if (need > c->gpart_cap) {
            HIPCHECK(c, hipStreamSynchronize(c->stream));
            dfree(c, c->d_gpart);
            c->d_gpart = nullptr;
            c->gpart_cap = 0;
            if (dmalloc(c, &c->d_gpart, (size_t)need * sizeof(double)) != hipSuccess)
                return fail(c, SBPE_ENOMEM, "gradient partial sums");
            c->gpart_cap = need;
        }
    }
    if (!homogeneous) {
        s = fill_tau(c, 1, t, dt);
        if (s) return s;
    }
    g.blocks = c->d_desc;
    g.nblocks = nb;
    g.nstages = nst;
    g.homogeneous = homogeneous ? 1 : 0;
    g.wide = c->op == SBPE_OP_WIDE ? 1 : 0;
    g.tau = c->d_tau;
    g.part = c->d_gpart;
    for (int st = 0; st < nst; ++st) {
        g.alpha[st] = alpha[st];
        g.tcol[st] = tcol[st];
        for (int b = 0; b < nb; ++b) {
            g.z[st][b] = z[st * nb + b];
            g.y[st][b] = y[st * nb + b];
            g.a[st][b] = a[st * nb + b];
        }
    }
    for (int b = 0; b < nb; ++b) {
        g.gc[b] = static_cast<double*>(gc[b]);
        g.grt[b] = static_cast<double*>(grt[b]);
    }
    const int e = launch_grad(c->dtype, c->order, g, c->stream);
    if (e != 0) return fail(c, SBPE_EHIP, std::string("gradient launch: ") + hip_error_string(e));
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_grad_accumulate(sbpe_ctx_t c, const void* const* z, const void* const* y,
                                            const void* const* a, double alpha, double t, int homogeneous,
                                            void* const* gc, void* const* grt) {
    const int tcol = 0;
    return grad_stages(c, 1, z, y, a, &alpha, &tcol, t, 0.0, homogeneous, gc, grt);
}

extern "C" sbpe_status sbpe_grad_accumulate_rk4(sbpe_ctx_t c, const void* const* z, const void* const* y,
                                                const void* const* a, const double* alpha, double t, double dt,
                                                int homogeneous, void* const* gc, void* const* grt) {
    static const int tcol[4] = {0, 1, 1, 2};     // stage times t, t + dt/2, t + dt/2, t + dt
    return grad_stages(c, 4, z, y, a, alpha, tcol, t, dt, homogeneous, gc, grt);
}

extern "C" sbpe_status sbpe_stage_slopes(sbpe_ctx_t c, int block, void** a1, void** a2) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail(c, SBPE_ESTATE, "call sbpe_finalize first");
    if (block < 0 || block >= (int)c->blocks.size()) return fail(c, SBPE_EINVAL, "no such block");
    if (!a1 || !a2) return fail(c, SBPE_EINVAL, "NULL pointer");
    *a1 = c->blocks[block].d_a1;
    *a2 = c->blocks[block].d_a2;
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_grad_to_physical(sbpe_ctx_t c, int block, const void* gc, const void* grt,
                                             double* g_c10, double* g_rho) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (block < 0 || block >= (int)c->blocks.size()) return fail(c, SBPE_EINVAL, "no such block");
    if (!gc || !grt || !g_c10 || !g_rho) return fail(c, SBPE_EINVAL, "NULL pointer");
    const HostBlock& B = c->blocks[block];
    const long np = B.np();
    std::vector<double> hg((size_t)10 * np), hr(np);
    HIPCHECK(c, hipStreamSynchronize(c->stream));
    HIPCHECK(c, hipMemcpy(hg.data(), gc, hg.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIPCHECK(c, hipMemcpy(hr.data(), grt, hr.size() * sizeof(double), hipMemcpyDeviceToHost));
    // stored coefficient k = c_{ijkl} with these representative indices
    static const int REP[10][4] = {{0, 0, 0, 0}, {0, 0, 0, 1}, {0, 1, 0, 1}, {1, 0, 1, 0}, {1, 0, 1, 1},
                                   {1, 1, 1, 1}, {0, 0, 1, 0}, {0, 0, 1, 1}, {0, 1, 1, 0}, {0, 1, 1, 1}};
    int m_of[4][4];
    for (int m = 0; m < 10; ++m) {
        m_of[C10P[m][0]][C10P[m][1]] = m;
        m_of[C10P[m][1]][C10P[m][0]] = m;
    }
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        double out[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        const double J = B.J[p];
        double F[2][2];
        for (int q = 0; q < 4; ++q) F[q >> 1][q & 1] = B.Fm[(size_t)q * np + p];
        // c_ijkl = J F_Ii C_IjKl F_Kk: d c_ijkl / d C_(Ij)(Kl) = J F_Ii F_Kk
        for (int k = 0; k < 10; ++k) {
            const double gk = hg[(size_t)k * np + p];
            const int i = REP[k][0], j = REP[k][1], kk = REP[k][2], l = REP[k][3];
            for (int I = 0; I < 2; ++I)
                for (int K = 0; K < 2; ++K) out[m_of[2 * I + j][2 * K + l]] += gk * J * F[I][i] * F[K][kk];
        }
        for (int m = 0; m < 10; ++m) g_c10[(size_t)m * np + p] = out[m];
        g_rho[p] = J * hr[p];     // rho~ = J rho
    }
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_lincomb(sbpe_ctx_t c, int nterms, const double* coefs, const void* const* x, void* y,
                                    long long count) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (nterms < 1 || nterms > LINCOMB_MAX || !coefs || !x || !y || count < 0)
        return fail(c, SBPE_EINVAL, "bad arguments");
    for (int k = 0; k < nterms; ++k)
        if (!x[k]) return fail(c, SBPE_EINVAL, "NULL input");
    const int e = launch_lincomb(c->dtype, nterms, coefs, x, y, (long)count, c->stream);
    if (e != 0) return fail(c, SBPE_EHIP, std::string("lincomb launch: ") + hip_error_string(e));
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_rk4_stages(sbpe_ctx_t c, const void* u0, const void* v0, const void* u1, const void* v1,
                                       const void* a1, const void* a2, double dt, void* const* out,
                                       long long count) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    if (!u0 || !v0 || !a1 || !a2 || !out || count < 0 || !(dt > 0.0)) return fail(c, SBPE_EINVAL, "bad arguments");
    Rk4StageArgs a;
    a.u0 = u0;
    a.v0 = v0;
    a.u1 = u1;
    a.v1 = v1;
    a.a1 = a1;
    a.a2 = a2;
    a.dt = dt;
    for (int k = 0; k < 7; ++k) a.out[k] = out[k];
    if ((out[5] || out[6]) && (!u1 || !v1)) return fail(c, SBPE_EINVAL, "the slopes a3, a4 need u1 and v1");
    const int e = launch_rk4_stages(c->dtype, a, (long)count, c->stream);
    if (e != 0) return fail(c, SBPE_EHIP, std::string("rk4 stages launch: ") + hip_error_string(e));
    return SBPE_OK;
}

extern "C" sbpe_status sbpe_receiver_adjoint(sbpe_ctx_t c, const void* r, void* const* u, double scale) {
    if (!check_ctx(c)) return fail(nullptr, SBPE_EINVAL, "NULL context");
    sbpe_status s = need_gpu(c);
    if (s) return s;
    const int nb = (int)c->blocks.size();
    if (nb > MAX_APPLY_BLOCKS) return fail(c, SBPE_EINVAL, "at most 16 blocks");
    if (!r || !u) return fail(c, SBPE_EINVAL, "NULL pointer");
    RecAdjArgs a;
    std::memset(&a, 0, sizeof a);
    for (int b = 0; b < nb; ++b) {
        if (!u[b]) return fail(c, SBPE_EINVAL, "NULL block pointer");
        a.u[b] = u[b];
        a.np[b] = c->blocks[b].np();
    }
    a.scale = scale;
    const int e = launch_rec_adjoint(c->dtype, c->d_recadj, c->nrecadj, static_cast<const double*>(r), a, c->stream);
    if (e != 0) return fail(c, SBPE_EHIP, std::string("receiver adjoint launch: ") + hip_error_string(e));
    return SBPE_OK;
}

// ================================================================ 3-D
// One curvilinear 3-D block (include/sbpe3.h): setup on the host (metric,
// c = F J C F, face scale factors), then the point kernel of sbpe3_kernels.hip.

struct sbpe3_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    int dtype = SBPE_F64, order = 4;
    double beta = 1.0;
    std::string err;
    int n[3] = {0, 0, 0};
    double h[3] = {0, 0, 0};
    std::vector<double> X[3], rho, C81;
    struct Face {
        int kind = BC_TRACTION;
        std::vector<double> g;     // [3][nf] as given
        TimeFn tf{TF_ZERO, 0, {0.0, 0.0}};
    } face[6];
    std::vector<double> force;     // [3][np] as given
    TimeFn ftf{TF_ZERO, 0, {0.0, 0.0}};
    std::vector<double> coef;      // host copy of the stored coefficients [46][np]
    void* d_coef = nullptr;
    void* d_force = nullptr;
    void* d_g[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    void* d_a1 = nullptr;
    void* d_a2 = nullptr;
    void* d_flux = nullptr;         // mixed-term fluxes of a pass's two fields [2][9][np]
    hipStream_t side = nullptr;     // the edge and corner points of a pass run here
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    double w[6] = {0, 0, 0, 0, 0, 0};
    bool finalized = false, bound = false;
    void* u = nullptr;
    void* v = nullptr;
    double t = 0.0;
    long np() const { return (long)n[0] * n[1] * n[2]; }
    int nf(int f) const {
        const int a = f >> 1;
        return a == 0 ? n[1] * n[2] : (a == 1 ? n[0] * n[2] : n[0] * n[1]);
    }
};

static sbpe_status fail3(sbpe3_ctx* c, sbpe_status code, const std::string& msg) {
    if (c) c->err = msg;
    else g_static_err = msg;
    return code;
}

static double tf_host(const TimeFn& f, double t) {
    switch (f.kind) {
        case TF_ONE: return 1.0;
        case TF_COS: return std::cos(f.p[0] * t + f.p[1]);
        case TF_RICKER: {
            const double a = (M_PI * f.p[0] * (t - f.p[1])) * (M_PI * f.p[0] * (t - f.p[1]));
            return (1.0 - 2.0 * a) * std::exp(-a);
        }
        default: return 0.0;
    }
}

// positive semidefinite test of a symmetric m x m matrix (pivoted Cholesky)
static bool psd_n(std::vector<double> a, int m, double tol_rel) {
    double dmax = 0.0;
    for (int i = 0; i < m; ++i) dmax = std::max(dmax, a[(size_t)i * m + i]);
    const double tol = tol_rel * std::max(1.0, dmax);
    std::vector<int> perm(m);
    for (int i = 0; i < m; ++i) perm[i] = i;
    for (int k = 0; k < m; ++k) {
        int p = k;
        for (int i = k + 1; i < m; ++i)
            if (a[(size_t)i * m + i] > a[(size_t)p * m + p]) p = i;
        if (p != k) {
            for (int j = 0; j < m; ++j) std::swap(a[(size_t)k * m + j], a[(size_t)p * m + j]);
            for (int i = 0; i < m; ++i) std::swap(a[(size_t)i * m + k], a[(size_t)i * m + p]);
        }
        const double d = a[(size_t)k * m + k];
        if (d <= tol) {
            for (int i = k; i < m; ++i)
                for (int j = k; j < m; ++j)
                    if (std::fabs(a[(size_t)i * m + j]) > tol) return false;
            return true;
        }
        for (int i = k + 1; i < m; ++i) {
            const double l = a[(size_t)i * m + k] / d;
            for (int j = k + 1; j < m; ++j) a[(size_t)i * m + j] -= l * a[(size_t)k * m + j];
        }
    }
    return true;
}

// largest eigenvalue of a symmetric 3 x 3 matrix (trigonometric closed form)
static double lmax3(const double G[3][3]) {
    const double p1 = G[0][1] * G[0][1] + G[0][2] * G[0][2] + G[1][2] * G[1][2];
    const double q = (G[0][0] + G[1][1] + G[2][2]) / 3.0;
    if (p1 == 0.0) return std::max(G[0][0], std::max(G[1][1], G[2][2]));
    const double p2 = (G[0][0] - q) * (G[0][0] - q) + (G[1][1] - q) * (G[1][1] - q) + (G[2][2] - q) * (G[2][2] - q) +
                      2.0 * p1;
    const double p = std::sqrt(p2 / 6.0);
    double B[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = (G[i][j] - (i == j ? q : 0.0)) / p;
    const double r = 0.5 * (B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) -
                            B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
                            B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0]));
    const double phi = r <= -1.0 ? M_PI / 3.0 : (r >= 1.0 ? 0.0 : std::acos(r) / 3.0);
    return q + 2.0 * p * std::cos(phi);
}

static int f3N(int i, int j, int l) {
    const int a = std::min(j, l), b = std::max(j, l);
    return 6 * i + (a == 0 ? b : (a == 1 ? 2 + b : 5));
}
static int f3M(int i, int k, int j, int l) {
    const int a = std::min(i, k), b = std::max(i, k);
    const int P = a == 0 ? (b == 1 ? 0 : 1) : 2;
    return i < k ? 18 + 9 * P + 3 * j + l : 18 + 9 * P + 3 * l + j;
}

template <typename P>
static hipError_t d3malloc(P** p, size_t bytes) {
    void* v = nullptr;
    const hipError_t e = hipMalloc(&v, bytes);
    *p = static_cast<P*>(v);
    return e;
}

static sbpe_status upload3(sbpe3_ctx* c, const double* h, size_t n, void** d) {
    const size_t es = c->dtype == SBPE_F64 ? 8 : 4;
    if (d3malloc(d, n * es) != hipSuccess) return fail3(c, SBPE_ENOMEM, "device allocation failed");
    hipError_t e;
    if (c->dtype == SBPE_F64) {
        e = hipMemcpy(*d, h, n * 8, hipMemcpyHostToDevice);
    } else {
        std::vector<float> f(n);
        for (size_t k = 0; k < n; ++k) f[k] = (float)h[k];
        e = hipMemcpy(*d, f.data(), n * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return fail3(c, SBPE_EHIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
    return SBPE_OK;
}

extern "C" {

sbpe_status sbpe3_create(int device, void* stream, int dtype, int order, double beta, sbpe3_ctx_t* out) {
    if (!out) return fail3(nullptr, SBPE_EINVAL, "NULL output");
    *out = nullptr;
    if (dtype != SBPE_F64 && dtype != SBPE_F32) return fail3(nullptr, SBPE_EINVAL, "bad dtype");
    if (order != 2 && order != 4) return fail3(nullptr, SBPE_EINVAL, "3-D blocks take orders 2 and 4");
    if (!(beta >= 1.0)) return fail3(nullptr, SBPE_EINVAL, "beta must be >= 1");
    if (device < 0) return fail3(nullptr, SBPE_EINVAL, "bad device");
    if (hipSetDevice(device) != hipSuccess) return fail3(nullptr, SBPE_EHIP, "hipSetDevice failed");
    auto* c = new sbpe3_ctx;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->dtype = dtype;
    c->order = order;
    c->beta = beta;
    // side stream of the edge and corner points (default priority)
    if (hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess) {
        sbpe3_destroy(c);
        return fail3(nullptr, SBPE_EHIP, "stream/event creation failed");
    }
    *out = c;
    return SBPE_OK;
}

sbpe_status sbpe3_destroy(sbpe3_ctx_t c) {
    if (!c) return SBPE_OK;
    // a finalize that failed part way may have left some of these behind
    if (c->finalized) (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->d_coef);
    (void)hipFree(c->d_force);
    for (int f = 0; f < 6; ++f) (void)hipFree(c->d_g[f]);
    (void)hipFree(c->d_a1);
    (void)hipFree(c->d_a2);
    (void)hipFree(c->d_flux);
    if (c->side) {
        (void)hipStreamSynchronize(c->side);
        (void)hipStreamDestroy(c->side);
    }
    if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
    if (c->ev_join) (void)hipEventDestroy(c->ev_join);
    delete c;
    return SBPE_OK;
}

const char* sbpe3_last_error(sbpe3_ctx_t c) { return c ? c->err.c_str() : g_static_err.c_str(); }

sbpe_status sbpe3_set_block(sbpe3_ctx_t c, int n1, int n2, int n3, const double* X1, const double* X2,
                            const double* X3, const double* rho, const double* C81) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail3(c, SBPE_ESTATE, "context already finalized");
    const int nmin = min_points(c->order);
    if (n1 < nmin || n2 < nmin || n3 < nmin) return fail3(c, SBPE_EINVAL, "block too small for the operator order");
    if ((long)n1 * n2 * n3 > (1L << 28)) return fail3(c, SBPE_EINVAL, "block has more than 2^28 points");
    if (!X1 || !X2 || !X3 || !rho || !C81) return fail3(c, SBPE_EINVAL, "NULL array");
    c->n[0] = n1;
    c->n[1] = n2;
    c->n[2] = n3;
    const long np = c->np();
    c->X[0].assign(X1, X1 + np);
    c->X[1].assign(X2, X2 + np);
    c->X[2].assign(X3, X3 + np);
    c->rho.assign(rho, rho + np);
    c->C81.assign(C81, C81 + 81 * np);
    for (int f = 0; f < 6; ++f) c->face[f] = sbpe3_ctx::Face{};
    c->force.clear();
    return SBPE_OK;
}

sbpe_status sbpe3_set_bc(sbpe3_ctx_t c, int face, int bc, const double* g, int time_fn, const double* tp) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail3(c, SBPE_ESTATE, "context already finalized");
    if (c->n[0] == 0) return fail3(c, SBPE_ESTATE, "no block");
    if (face < 0 || face > 5) return fail3(c, SBPE_EINVAL, "bad face");
    if (bc != SBPE_BC_TRACTION && bc != SBPE_BC_DISPLACEMENT)
        return fail3(c, SBPE_EINVAL, "3-D faces are traction or displacement");
    if (time_fn < SBPE_TIME_ZERO || time_fn > SBPE_TIME_RICKER) return fail3(c, SBPE_EINVAL, "bad time function");
    auto& F = c->face[face];
    F.kind = bc;
    if (g) F.g.assign(g, g + 3L * c->nf(face));
    else F.g.clear();
    set_time_fn(time_fn, tp, F.tf);
    return SBPE_OK;
}

sbpe_status sbpe3_set_forcing(sbpe3_ctx_t c, const double* F, int time_fn, const double* tp) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail3(c, SBPE_ESTATE, "context already finalized");
    if (c->n[0] == 0) return fail3(c, SBPE_ESTATE, "no block");
    if (time_fn < SBPE_TIME_ZERO || time_fn > SBPE_TIME_RICKER) return fail3(c, SBPE_EINVAL, "bad time function");
    if (F) c->force.assign(F, F + 3 * c->np());
    else c->force.clear();
    set_time_fn(time_fn, tp, c->ftf);
    return SBPE_OK;
}

sbpe_status sbpe3_finalize(sbpe3_ctx_t c) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (c->finalized) return fail3(c, SBPE_ESTATE, "context already finalized");
    if (c->n[0] == 0) return fail3(c, SBPE_ESTATE, "no block");
    const int o = c->order;
    const long np = c->np();
    const int* n = c->n;
    const long st[3] = {1, n[0], (long)n[0] * n[1]};
    for (int i = 0; i < 3; ++i) c->h[i] = 1.0 / (n[i] - 1);
    // A[i][I] = dX_I / dx_i along every line of direction i
    std::vector<hvec> A(9);
    for (auto& a : A) a.resize(np);
    for (int i = 0; i < 3; ++i) {
        const int j1 = (i + 1) % 3, j2 = (i + 2) % 3;
#pragma omp parallel for schedule(static) collapse(2)
        for (int b = 0; b < n[j2]; ++b)
            for (int a = 0; a < n[j1]; ++a) {
                const long s0 = (long)a * st[j1] + (long)b * st[j2];
                for (int I = 0; I < 3; ++I)
                    d1_apply(o, n[i], c->h[i], &c->X[I][s0], st[i], &A[3 * i + I][s0], st[i]);
            }
    }
    c->coef.assign((size_t)NCOEF3 * np, 0.0);
    std::vector<double> Jv(np);
    long bad_j = -1, bad_c = -1;
#pragma omp parallel for schedule(static)
    for (long p = 0; p < np; ++p) {
        double M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int I = 0; I < 3; ++I) M[i][I] = A[3 * i + I][p];
        const double J = M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) -
                         M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
                         M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0]);
        if (!(J > 0.0)) {
#pragma omp critical
            bad_j = (bad_j < 0 || p < bad_j) ? p : bad_j;
            continue;
        }
        Jv[p] = J;
        // F[I][i] = dx_i / dX_I = (M^{-1})[I][i]
        double F[3][3];
        for (int I = 0; I < 3; ++I)
            for (int i = 0; i < 3; ++i) {
                const int r1 = (i + 1) % 3, r2 = (i + 2) % 3, c1 = (I + 1) % 3, c2 = (I + 2) % 3;
                F[I][i] = (M[r1][c1] * M[r2][c2] - M[r1][c2] * M[r2][c1]) / J;
            }
        const double* C = c->C81.data();
        std::vector<double> Cm(81);
        for (int k = 0; k < 81; ++k) Cm[k] = C[(long)k * np + p];
        bool sym = true;
        for (int a = 0; a < 9 && sym; ++a)
            for (int b = 0; b < 9; ++b)
                if (std::fabs(Cm[a * 9 + b] - Cm[b * 9 + a]) > 1e-12 * (std::fabs(Cm[a * 9 + b]) + 1.0)) sym = false;
        if (!sym || !psd_n(Cm, 9, 1e-10)) {
#pragma omp critical
            bad_c = (bad_c < 0 || p < bad_c) ? p : bad_c;
            continue;
        }
        // c_ijkl = J F_Ii C_IjKl F_Kk
        auto cc = [&](int i, int j, int k, int l) {
            double s = 0.0;
            for (int I = 0; I < 3; ++I)
                for (int K = 0; K < 3; ++K) s += F[I][i] * Cm[((I * 3 + j) * 3 + K) * 3 + l] * F[K][k];
            return J * s;
        };
        double* q = c->coef.data();
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int l = j; l < 3; ++l) q[(long)f3N(i, j, l) * np + p] = cc(i, j, i, l);
        for (int i = 0; i < 3; ++i)
            for (int k = i + 1; k < 3; ++k)
                for (int j = 0; j < 3; ++j)
                    for (int l = 0; l < 3; ++l) q[(long)f3M(i, k, j, l) * np + p] = cc(i, j, k, l);
        q[(long)45 * np + p] = 1.0 / (J * c->rho[p]);
    }
    if (bad_j >= 0) return fail3(c, SBPE_ENONPOS_J, "discrete Jacobian <= 0 at point " + std::to_string(bad_j));
    if (bad_c >= 0)
        return fail3(c, SBPE_ENOT_PSD, "stiffness not major symmetric positive semidefinite at point " + std::to_string(bad_c));
    if (hipSetDevice(c->device) != hipSuccess) return fail3(c, SBPE_EHIP, "hipSetDevice failed");
    sbpe_status s = upload3(c, c->coef.data(), c->coef.size(), &c->d_coef);
    if (s) return s;
    if (!c->force.empty()) {
        std::vector<double> JF(3 * np);
        for (int j = 0; j < 3; ++j)
            for (long p = 0; p < np; ++p) JF[(size_t)j * np + p] = Jv[p] * c->force[(size_t)j * np + p];
        s = upload3(c, JF.data(), JF.size(), &c->d_force);
        if (s) return s;
    }
    // faces: first norm weight of the normal direction, Jhat = |a_t1 x a_t2|
    for (int f = 0; f < 6; ++f) {
        const int a = f >> 1, t1 = a == 0 ? 1 : 0, t2 = a == 2 ? 1 : 2;
        c->w[f] = c->h[a] * norm_weight(o, n[a], 0);
        auto& F = c->face[f];
        if (F.g.empty()) continue;
        const int nf = c->nf(f);
        std::vector<double> g(F.g);
        if (F.kind == SBPE_BC_TRACTION) {
            const int cn = (f & 1) ? n[a] - 1 : 0;
            for (int b = 0; b < n[t2]; ++b)
                for (int aa = 0; aa < n[t1]; ++aa) {
                    const long p = (long)cn * st[a] + (long)aa * st[t1] + (long)b * st[t2];
                    const double x[3] = {A[3 * t1][p], A[3 * t1 + 1][p], A[3 * t1 + 2][p]};
                    const double y[3] = {A[3 * t2][p], A[3 * t2 + 1][p], A[3 * t2 + 2][p]};
                    const double cr[3] = {x[1] * y[2] - x[2] * y[1], x[2] * y[0] - x[0] * y[2], x[0] * y[1] - x[1] * y[0]};
                    const double jh = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
                    const int t = aa + n[t1] * b;
                    for (int j = 0; j < 3; ++j) g[(size_t)j * nf + t] *= jh / c->w[f];
                }
        }
        s = upload3(c, g.data(), g.size(), &c->d_g[f]);
        if (s) return s;
    }
    const size_t es = c->dtype == SBPE_F64 ? 8 : 4;
    if (d3malloc(&c->d_a1, 3 * np * es) != hipSuccess || d3malloc(&c->d_a2, 3 * np * es) != hipSuccess ||
        d3malloc(&c->d_flux, 2 * 9 * np * es) != hipSuccess)
        return fail3(c, SBPE_ENOMEM, "device allocation failed");
    c->finalized = true;
    return SBPE_OK;
}

// dt = cfl min h / v_max, v_max^2 = max over directions xi and points of
// lambda_max(xi_i c_ijkl xi_k) / rho~ (2000 directions of a Fibonacci sphere)
sbpe_status sbpe3_dt_cfl(sbpe3_ctx_t c, double cfl, double* dt) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail3(c, SBPE_ESTATE, "context not finalized");
    if (!dt || !(cfl > 0)) return fail3(c, SBPE_EINVAL, "bad arguments");
    const long np = c->np();
    const int ndir = 2000;
    std::vector<double> xi(3 * ndir);
    for (int d = 0; d < ndir; ++d) {
        const double k = d + 0.5, z = 1.0 - 2.0 * k / ndir, r = std::sqrt(1.0 - z * z);
        const double ph = M_PI * (1.0 + std::sqrt(5.0)) * k;
        xi[3 * d] = r * std::cos(ph);
        xi[3 * d + 1] = r * std::sin(ph);
        xi[3 * d + 2] = z;
    }
    const double* q = c->coef.data();
    double best = 0.0;
#pragma omp parallel for schedule(static) reduction(max : best)
    for (long p = 0; p < np; ++p) {
        double cc[3][3][3][3];
        for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k)
                for (int j = 0; j < 3; ++j)
                    for (int l = 0; l < 3; ++l)
                        cc[i][j][k][l] = i == k ? q[(long)f3N(i, j, l) * np + p] : q[(long)f3M(i, k, j, l) * np + p];
        const double irho = q[(long)45 * np + p];
        for (int d = 0; d < ndir; ++d) {
            double G[3][3];
            for (int j = 0; j < 3; ++j)
                for (int l = 0; l < 3; ++l) {
                    double s = 0.0;
                    for (int i = 0; i < 3; ++i)
                        for (int k = 0; k < 3; ++k) s += xi[3 * d + i] * cc[i][j][k][l] * xi[3 * d + k];
                    G[j][l] = s;
                }
            best = std::max(best, lmax3(G) * irho);
        }
    }
    *dt = cfl * std::min(c->h[0], std::min(c->h[1], c->h[2])) / std::sqrt(best);
    return SBPE_OK;
}

static Args3 args3(const sbpe3_ctx* c) {
    Args3 a;
    std::memset(&a, 0, sizeof a);
    a.n1 = c->n[0];
    a.n2 = c->n[1];
    a.n3 = c->n[2];
    a.h1 = c->h[0];
    a.h2 = c->h[1];
    a.h3 = c->h[2];
    a.beta = c->beta;
    a.coef = c->d_coef;
    a.force = c->d_force;
    for (int f = 0; f < 6; ++f) {
        a.face[f].kind = c->face[f].kind;
        a.face[f].nf = c->nf(f);
        a.face[f].w = c->w[f];
        a.face[f].g = c->d_g[f];
    }
    a.a1 = c->d_a1;
    a.a2 = c->d_a2;
    a.flux = c->d_flux;
    return a;
}

// time values of the 6 face items and the forcing at time t
static void tvals3(const sbpe3_ctx* c, double t, double out[7]) {
    for (int f = 0; f < 6; ++f) out[f] = c->face[f].g.empty() ? 0.0 : tf_host(c->face[f].tf, t);
    out[6] = c->force.empty() ? 0.0 : tf_host(c->ftf, t);
}

sbpe_status sbpe3_apply(sbpe3_ctx_t c, const void* u, void* a, double t, int homogeneous) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail3(c, SBPE_ESTATE, "context not finalized");
    if (!u || !a || u == a) return fail3(c, SBPE_EINVAL, "bad operands");
    Args3 A = args3(c);
    A.pass = PASS_APPLY;
    A.in = u;
    A.out = a;
    if (!homogeneous) tvals3(c, t, A.tfa);
    const int e = launch_point3(c->dtype, c->order, A, c->stream, c->side, c->ev_fork, c->ev_join);
    if (e) return fail3(c, SBPE_EHIP, std::string("kernel launch: ") + hip_error_string(e));
    return SBPE_OK;
}

sbpe_status sbpe3_bind_state(sbpe3_ctx_t c, void* u, void* v, double t) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->finalized) return fail3(c, SBPE_ESTATE, "context not finalized");
    if (!u || !v || u == v) return fail3(c, SBPE_EINVAL, "bad state buffers");
    c->u = u;
    c->v = v;
    c->t = t;
    c->bound = true;
    return SBPE_OK;
}

// classical RK4 in the two sweeps of sbpe_internal.h, data at t, t + dt/2, t + dt
sbpe_status sbpe3_advance(sbpe3_ctx_t c, int nsteps, double dt) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (!c->bound) return fail3(c, SBPE_ESTATE, "no bound state");
    if (nsteps < 0 || !(dt > 0) || !std::isfinite(dt)) return fail3(c, SBPE_EINVAL, "bad nsteps or dt");
    for (int k = 0; k < nsteps; ++k) {
        const double t = c->t;
        double v0[7], vh[7], v1[7];
        tvals3(c, t, v0);
        tvals3(c, t + 0.5 * dt, vh);
        tvals3(c, t + dt, v1);
        Args3 A = args3(c);
        A.dt = dt;
        A.u = c->u;
        A.v = c->v;
        A.uo = c->u;
        A.vo = c->v;
        A.pass = PASS_RK1;
        for (int q = 0; q < 7; ++q) {
            A.tfa[q] = v0[q];
            A.tfb[q] = vh[q];
        }
        int e = launch_point3(c->dtype, c->order, A, c->stream, c->side, c->ev_fork, c->ev_join);
        if (e) return fail3(c, SBPE_EHIP, std::string("kernel launch: ") + hip_error_string(e));
        A.pass = PASS_RK2;
        for (int q = 0; q < 7; ++q) {
            A.tfa[q] = 0.0;
            A.tfb[q] = 2.0 / (dt * dt) * (v0[q] - 2.0 * vh[q] + v1[q]);
        }
        e = launch_point3(c->dtype, c->order, A, c->stream, c->side, c->ev_fork, c->ev_join);
        if (e) return fail3(c, SBPE_EHIP, std::string("kernel launch: ") + hip_error_string(e));
        c->t = t + dt;
    }
    return SBPE_OK;
}

sbpe_status sbpe3_get_time(sbpe3_ctx_t c, double* t) {
    if (!c || !t) return fail3(c, SBPE_EINVAL, "NULL argument");
    *t = c->t;
    return SBPE_OK;
}

sbpe_status sbpe3_synchronize(sbpe3_ctx_t c) {
    if (!c) return fail3(nullptr, SBPE_EINVAL, "NULL context");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail3(c, SBPE_EHIP, "hipStreamSynchronize failed");
    return SBPE_OK;
}

}  // extern "C"
