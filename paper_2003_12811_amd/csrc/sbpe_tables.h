// Coefficients of the one-dimensional diagonal-norm SBP operators used by the
// library (Sec. 4 of Almquist & Dunham, arXiv 2003.12811), and the derivation
// of the boundary-closure table of the adapted fully compatible narrow second
// derivative D2^FC(b) (Sec. 4.1) from its SBP form
//
//   H D2^FC(b) = -D1^T H b D1 - R(b) - e0 b0 e0^T D1 + eN bN eN^T D1,
//   R(b)       = (1/h) sum_windows gamma_w B_w(b) d_w d_w^T      (eq. B_structure_1d).
//
// All coefficients are dimensionless (h = 1); kernels scale by 1/h or 1/h^2.
//
// Order 4: the classical diagonal norm 17/48, 59/48, 43/48, 49/48 and its
// first-derivative boundary rows; remainder windows d3 = (-1,3,-3,1) with
// weight 1/18 (B = mean of the two middle b values) and d4 = (1,-4,6,-4,1)
// with weight 1/144 (B = centre b).  The three d3 windows touching each end
// carry the weights 181507/1719312, 293/4214, 185/3528, which make rows 1..5
// of D2^FC second-order accurate for variable b (row 0 keeps the end-point
// order of the adapted operators).  Order 2: norm 1/2 at the ends,
// D1 boundary rows (-1, 1), windows d2 = (1,-2,1) with weight 1/4 and B = centre b.
// Order 6: see the order-6 block below.
#pragma once

namespace sbpe {

// ---- order 4 ---------------------------------------------------------------
constexpr int O4_NB = 4;                 // number of D1 / H boundary rows
constexpr int O4_R0 = 6;                 // number of D2^FC closure rows
constexpr int O4_W = 8;                  // closure row width (u and b indices 0..7)
constexpr double O4_H[O4_NB] = {17.0 / 48.0, 59.0 / 48.0, 43.0 / 48.0, 49.0 / 48.0};
constexpr double O4_D1B[O4_NB][6] = {
    {-24.0 / 17.0, 59.0 / 34.0, -4.0 / 17.0, -3.0 / 34.0, 0.0, 0.0},
    {-0.5, 0.0, 0.5, 0.0, 0.0, 0.0},
    {4.0 / 43.0, -59.0 / 86.0, 0.0, 59.0 / 86.0, -4.0 / 43.0, 0.0},
    {3.0 / 98.0, 0.0, -59.0 / 98.0, 0.0, 32.0 / 49.0, -4.0 / 49.0}};
constexpr double O4_D1I[5] = {1.0 / 12.0, -2.0 / 3.0, 0.0, 2.0 / 3.0, -1.0 / 12.0};
constexpr double O4_G3_BND[3] = {181507.0 / 1719312.0, 293.0 / 4214.0, 185.0 / 3528.0};
constexpr double O4_G3 = 1.0 / 18.0;
constexpr double O4_G4 = 1.0 / 144.0;

// ---- order 2 ---------------------------------------------------------------
constexpr int O2_NB = 1;
constexpr int O2_R0 = 1;
constexpr int O2_W = 2;
constexpr double O2_H[O2_NB] = {0.5};
constexpr double O2_D1B[O2_NB][6] = {{-1.0, 1.0, 0.0, 0.0, 0.0, 0.0}};
constexpr double O2_D1I[3] = {-0.5, 0.0, 0.5};
constexpr double O2_G2 = 0.25;

// ---- order 6 ---------------------------------------------------------------
// The unique diagonal norm of a six-row closure of boundary order 3; the
// first-derivative closure rows D1 = H^{-1} Q with the one free entry Q_45 of
// Q set to the minimiser of the H-weighted squared degree-4 residual of the
// closure rows (rounded from exact rationals).  Remainder windows of orders 4,
// 5, 6: d4 with weight 1/80 (B = mean of the three middle b values), d5 with
// 1/600 (B = mean of the two middle ones), d6 with 1/3600 (B = centre b); the
// five d4 windows touching each end are scaled by O6_G4_BND, which makes rows
// 1..8 of D2^FC third-order accurate for variable b.
constexpr int O6_NB = 6;
constexpr int O6_R0 = 9;
constexpr int O6_W = 12;
constexpr int O6_D1W = 9;                // columns of a D1 closure row
constexpr double O6_H[O6_NB] = {13649.0 / 43200.0, 12013.0 / 8640.0, 2711.0 / 4320.0,
                                5359.0 / 4320.0, 7877.0 / 8640.0, 43801.0 / 43200.0};
constexpr double O6_D1B[O6_NB][O6_D1W] = {
    {-1.5825335189391163, 2.0448904424171728, -0.18755991361085947, -0.3813277242792929, 0.058441014418055957, 0.048089699994040239, 0.0, 0.0, 0.0},
    {-0.46467509612173458, 0.0, 0.31341762788401262, 0.20649807756530805, -0.02987355817398105, -0.025367051153605054, 0.0, 0.0, 0.0},
    {0.094430293650852856, -0.69440906746046549, 0.0, 0.72215146825426424, -0.13881813492093095, 0.016645440476279281, 0.0, 0.0, 0.0},
    {0.097121517236202062, -0.23144816251092049, -0.36532051323704245, 0.0, 0.54958194598842858, -0.063370129891297269, 0.013435342414629596, 0.0, 0.0},
    {-0.020252923848979199, 0.045559356905425202, 0.095553120165200914, -0.74779983459489363, 0.0, 0.77318885316453778, -0.1645296432652025, 0.018281071473911389, 0.0},
    {-0.01498541848858828, 0.034786236102858095, -0.010302456366565406, 0.077532596536029341, -0.69523624990035204, 0.0, 0.73970913906075209, -0.1479418278121504, 0.016437980868016712}};
constexpr double O6_D1I[7] = {-1.0 / 60.0, 3.0 / 20.0, -0.75, 0.0, 0.75, -3.0 / 20.0, 1.0 / 60.0};
constexpr double O6_G4 = 1.0 / 80.0;
constexpr double O6_G5 = 1.0 / 600.0;
constexpr double O6_G6 = 1.0 / 3600.0;
constexpr double O6_G4_BND[5] = {7.5209690064828418, 7.1872878387387704, 1.5548122877553581, 0.77018733107015991, 1.0580948577597769};

// Number of points adjacent to each face that need boundary-aware treatment
// (closure rows or displacement/interface SAT reach); the rest is interior.
template <int ORD> struct Frame;
template <> struct Frame<4> { static constexpr int R = 6; };
template <> struct Frame<2> { static constexpr int R = 2; };
template <> struct Frame<6> { static constexpr int R = 9; };

// ---- closure tables, derived at compile time --------------------------------
// T[r][m][s] (r < R0, m, s < W) with h^2 (D2^FC(b) u)_r = sum_{m,s} T[r][m][s] b_s u_m
// on the lower end of a line (rows r < R0); the upper end follows by reflection:
// (D2^FC u)_{N-r} uses b_{N-s}, u_{N-m}.  Derived on a 32-point line from
//   -H^{-1} ( D1^T H b D1 + R(b) + e0 b0 e0^T D1 )   restricted to rows r < R0.
template <int R0, int W> struct D2Table {
    double t[R0][W][W];
};

constexpr double table_norm(int order, int n, int k) {
    if (order == 6) return k < O6_NB ? O6_H[k] : (k > n - 1 - O6_NB ? O6_H[n - 1 - k] : 1.0);
    if (order == 4) return k < O4_NB ? O4_H[k] : (k > n - 1 - O4_NB ? O4_H[n - 1 - k] : 1.0);
    return k < O2_NB ? O2_H[k] : (k > n - 1 - O2_NB ? O2_H[n - 1 - k] : 1.0);
}

constexpr D2Table<O4_R0, O4_W> make_d2_table4() {
    constexpr int n = 32;
    double D[n][n] = {};
    for (int r = 0; r < O4_NB; ++r)
        for (int c = 0; c < 6; ++c) {
            D[r][c] = O4_D1B[r][c];
            D[n - 1 - r][n - 1 - c] = -O4_D1B[r][c];
        }
    for (int r = O4_NB; r < n - O4_NB; ++r)
        for (int k = 0; k < 5; ++k) D[r][r - 2 + k] = O4_D1I[k];
    const double d3[4] = {-1, 3, -3, 1};
    const double d4[5] = {1, -4, 6, -4, 1};
    D2Table<O4_R0, O4_W> T{};
    for (int r = 0; r < O4_R0; ++r)
        for (int m = 0; m < O4_W; ++m)
            for (int s = 0; s < O4_W; ++s) {
                double v = -D[s][r] * table_norm(4, n, s) * D[s][m];
                const int n3 = n - 3;
                for (int c = 0; c < n3; ++c) {          // d3 windows, B = (b_{c+1} + b_{c+2}) / 2
                    if (r < c || r > c + 3 || m < c || m > c + 3) continue;
                    double g = O4_G3;
                    if (c < 3) g = O4_G3_BND[c];
                    else if (n3 - 1 - c < 3) g = O4_G3_BND[n3 - 1 - c];
                    if (s == c + 1 || s == c + 2) v -= g * 0.5 * d3[r - c] * d3[m - c];
                }
                for (int c = 0; c + 4 < n; ++c) {       // d4 windows, B = b_{c+2}
                    if (r < c || r > c + 4 || m < c || m > c + 4) continue;
                    if (s == c + 2) v -= O4_G4 * d4[r - c] * d4[m - c];
                }
                if (r == 0 && s == 0) v -= D[0][m];     // boundary derivative = D1 (fully compatible)
                T.t[r][m][s] = v / table_norm(4, n, r);
            }
    return T;
}

constexpr D2Table<O2_R0, O2_W> make_d2_table2() {
    constexpr int n = 16;
    double D[n][n] = {};
    D[0][0] = O2_D1B[0][0];
    D[0][1] = O2_D1B[0][1];
    D[n - 1][n - 1] = -O2_D1B[0][0];
    D[n - 1][n - 2] = -O2_D1B[0][1];
    for (int r = 1; r < n - 1; ++r)
        for (int k = 0; k < 3; ++k) D[r][r - 1 + k] = O2_D1I[k];
    const double d2[3] = {1, -2, 1};
    D2Table<O2_R0, O2_W> T{};
    for (int r = 0; r < O2_R0; ++r)
        for (int m = 0; m < O2_W; ++m)
            for (int s = 0; s < O2_W; ++s) {
                double v = -D[s][r] * table_norm(2, n, s) * D[s][m];
                for (int c = 0; c + 2 < n; ++c) {       // d2 windows, B = b_{c+1}
                    if (r < c || r > c + 2 || m < c || m > c + 2) continue;
                    if (s == c + 1) v -= O2_G2 * d2[r - c] * d2[m - c];
                }
                if (r == 0 && s == 0) v -= D[0][m];
                T.t[r][m][s] = v / table_norm(2, n, r);
            }
    return T;
}

constexpr D2Table<O6_R0, O6_W> make_d2_table6() {
    constexpr int n = 40;
    double D[n][n] = {};
    for (int r = 0; r < O6_NB; ++r)
        for (int c = 0; c < O6_D1W; ++c) {
            D[r][c] = O6_D1B[r][c];
            D[n - 1 - r][n - 1 - c] = -O6_D1B[r][c];
        }
    for (int r = O6_NB; r < n - O6_NB; ++r)
        for (int k = 0; k < 7; ++k) D[r][r - 3 + k] = O6_D1I[k];
    const double d4[5] = {1, -4, 6, -4, 1};
    const double d5[6] = {-1, 5, -10, 10, -5, 1};
    const double d6[7] = {1, -6, 15, -20, 15, -6, 1};
    D2Table<O6_R0, O6_W> T{};
    for (int r = 0; r < O6_R0; ++r)
        for (int m = 0; m < O6_W; ++m)
            for (int s = 0; s < O6_W; ++s) {
                double v = -D[s][r] * table_norm(6, n, s) * D[s][m];
                // windows starting at c hold r and m, and (for these rows, far
                // from the upper end) are full windows of the lower end
                for (int c = (r > 4 ? r - 4 : 0); c <= r; ++c) {   // d4, B = (b_{c+1} + b_{c+2} + b_{c+3}) / 3
                    if (m < c || m > c + 4 || s < c + 1 || s > c + 3) continue;
                    const double g = c < 5 ? O6_G4 * O6_G4_BND[c] : O6_G4;
                    v -= g * d4[r - c] * d4[m - c] / 3.0;
                }
                for (int c = (r > 5 ? r - 5 : 0); c <= r; ++c) {   // d5, B = (b_{c+2} + b_{c+3}) / 2
                    if (m < c || m > c + 5 || (s != c + 2 && s != c + 3)) continue;
                    v -= O6_G5 * 0.5 * d5[r - c] * d5[m - c];
                }
                for (int c = (r > 6 ? r - 6 : 0); c <= r; ++c) {   // d6, B = b_{c+3}
                    if (m < c || m > c + 6 || s != c + 3) continue;
                    v -= O6_G6 * d6[r - c] * d6[m - c];
                }
                if (r == 0 && s == 0) v -= D[0][m];     // boundary derivative = D1 (fully compatible)
                T.t[r][m][s] = v / table_norm(6, n, r);
            }
    return T;
}

constexpr D2Table<O4_R0, O4_W> D2T4 = make_d2_table4();
constexpr D2Table<O2_R0, O2_W> D2T2 = make_d2_table2();
constexpr D2Table<O6_R0, O6_W> D2T6 = make_d2_table6();

// Host copies of the derived closure tables (T[r][m][s], row-major).
void derive_d2_closure(int order, double* T);
// Dimensionless norm weight of point k on a line of n points.
double norm_weight(int order, int n, int k);
// Dense dimensionless D1 of n points (row-major n*n), for host-side setup.
void dense_d1(int order, int n, double* D);

}  // namespace sbpe
