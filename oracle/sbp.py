"""One-dimensional diagonal-norm SBP operators (oracle, test infrastructure only).

Definitions followed (Almquist & Dunham, arXiv 2003.12811):

* Norm H = diag(h_1, h_2, ..., h_2, h_1), first derivative D1 with
  H D1 + D1^T H = -e0 e0^T + eN eN^T                       (Sec. 4, eq. structure_H, el_er)
* Compatible second derivative in SBP form
  H D2(b) = -D1^T H b D1 - R(b) - e0 e0^T b S + eN eN^T b S (Sec. 4, eq. sbp_property_2nd_der)
  with the remainder R(b) = sum_alpha D_alpha^T B_alpha(b) D_alpha, each B_alpha a
  diagonal of non-negative combinations of b                 (Sec. 4, eq. B_structure_1d)
* The adapted fully compatible operator replaces the boundary derivative S by D1
  (Sec. 4.1), so
  D2^FC(b) = H^{-1} ( -D1^T H b D1 - R(b) - e0 b_0 e0^T D1 + eN b_N eN^T D1 ).

The paper cites, but does not print, the coefficients.  Readings used here:

* 2nd order: H = h diag(1/2, 1, ..., 1, 1/2); D1 = (-1/2, 0, 1/2)/h inside,
  (-1, 1)/h at both ends; R(b) = (1/4h) sum_c b_c d2_c d2_c^T over every
  full 3-point window d2 = (1, -2, 1) centred at c = 1..N-1.  This is the
  classical second-order operator written in the paper's R form.
* 4th order: the classical diagonal-norm operator,
  H = h diag(17/48, 59/48, 43/48, 49/48, 1, ...), boundary rows of D1 as in
  ``_D1_CLOSURE_4``, interior (1/12, -2/3, 0, 2/3, -1/12)/h.
  R(b) = (1/h) [ sum_c g_c (b_{c+1}+b_{c+2})/2 d3_c d3_c^T
               + sum_c (1/144) b_{c+2} d4_c d4_c^T ]
  over all full 4-point windows d3 = (-1, 3, -3, 1) and 5-point windows
  d4 = (1, -4, 6, -4, 1) starting at c.  g_c = 1/18 inside (this makes the
  interior stencil five points wide and fourth-order accurate); the three
  windows touching each end use g_0 = 181507/1719312, g_1 = 293/4214,
  g_2 = 185/3528, the unique values that make rows 1..5 of D2^FC exact for all
  (b, u) polynomial pairs of total degree <= 3 (second-order closure) while row
  0 keeps the end-point order q-1 of the adapted operators.  All weights are
  positive, so every dR/db_s is positive semidefinite (Lemma 1 holds).
* 6th order: the diagonal norm of a six-row closure with boundary order 3,
  H = h diag(13649/43200, 12013/8640, 2711/4320, 5359/4320, 7877/8640,
  43801/43200, 1, ...), which the order conditions fix uniquely; they leave
  one free entry of Q = H D1, set to the minimiser of the H-weighted squared
  degree-4 residual of the closure rows (``_Q6_UPPER``); interior
  (-1/60, 3/20, -3/4, 0, 3/4, -3/20, 1/60)/h.  R(b) has windows of differences
  of orders 4, 5, 6 with B the mean of the three middle b values (weight
  1/80), of the two middle ones (1/600) and the centre value (1/3600): the
  unique non-negative weights that give a seven-point sixth-order interior.
  The five order-4 windows at each end are scaled by ``_G4_BND``, the unique
  factors making rows 1..8 exact for (b, u) pairs of total degree <= 4 (a
  third-order closure); all are positive.

Parity status: pinned (tests/test_oracle_sbp.py checks the SBP identities in
exact rational arithmetic, polynomial exactness, symmetry and positive
semidefiniteness of R, and the constant-coefficient textbook stencils;
tests/test_oracle_sixth.py re-derives every order-6 choice in exact
arithmetic and checks the 2-D operator's self-adjointness and convergence).
"""
from fractions import Fraction as Fr

import numpy as np
import scipy.sparse as sps

ORDERS = (2, 4, 6)

# ---------------------------------------------------------------- norms
_H_CLOSURE = {
    2: [Fr(1, 2)],
    4: [Fr(17, 48), Fr(59, 48), Fr(43, 48), Fr(49, 48)],
    # the unique diagonal norm of a 6-row closure with third-order boundary rows
    6: [Fr(13649, 43200), Fr(12013, 8640), Fr(2711, 4320), Fr(5359, 4320), Fr(7877, 8640), Fr(43801, 43200)],
}

# ------------------------------------------------------ first derivative
_D1_CLOSURE = {
    2: [[Fr(-1), Fr(1)]],
    4: [[Fr(-24, 17), Fr(59, 34), Fr(-4, 17), Fr(-3, 34)],
        [Fr(-1, 2), Fr(0), Fr(1, 2)],
        [Fr(4, 43), Fr(-59, 86), Fr(0), Fr(59, 86), Fr(-4, 43)],
        [Fr(3, 98), Fr(0), Fr(-59, 98), Fr(0), Fr(32, 49), Fr(-4, 49)]],
}
_D1_INTERIOR = {
    2: (1, [Fr(-1, 2), Fr(0), Fr(1, 2)]),
    4: (2, [Fr(1, 12), Fr(-2, 3), Fr(0), Fr(2, 3), Fr(-1, 12)]),
    6: (3, [Fr(-1, 60), Fr(3, 20), Fr(-3, 4), Fr(0), Fr(3, 4), Fr(-3, 20), Fr(1, 60)]),
}

# Order 6: Q = H D1 on the six closure rows.  The order conditions
# (D1 x^k = k x^(k-1), k <= 3, on rows 0..5) with Q + Q^T = diag(-1, 0, ...)
# fix H uniquely and leave one free entry, Q_45.  It is set to the minimiser of
# the H-weighted square of the degree-4 residuals of the closure rows,
# sum_r H_r ((D1 x^4)_r - 4 x_r^3)^2, inside the interval where every boundary
# weight of the remainder below is non-negative.  Entries (r, c), r < c < 6;
# Q_rr = 0 except Q_00 = -1/2; Q_rc = -Q_cr; columns 6..8 follow from the
# interior rows by skew symmetry.
_Q6_UPPER = {
    (0, 1): Fr(5124475092222703052468879, 7931626489314500743872000),
    (0, 2): Fr(-14688227387107654735453, 247863327791078148246000),
    (0, 3): Fr(-159267246833799759813661, 1321937748219083457312000),
    (0, 4): Fr(18306575045382041159483, 991453311164312592984000),
    (0, 5): Fr(120512309461734500607719, 7931626489314500743872000),
    (1, 2): Fr(345639531999877949576339, 793162648931450074387200),
    (1, 3): Fr(28465971813079192963909, 99145331116431259298400),
    (1, 4): Fr(-21963203401877827569241, 528775099287633382924800),
    (1, 5): Fr(-34968740224280558358577, 991453311164312592984000),
    (2, 3): Fr(179724104434047613799819, 396581324465725037193600),
    (2, 4): Fr(-8637026328486517498841, 99145331116431259298400),
    (2, 5): Fr(13808676868217278023299, 1321937748219083457312000),
    (3, 4): Fr(540747751505546378368499, 793162648931450074387200),
    (3, 5): Fr(-9742420893013796487329, 123931663895539074123000),
    (4, 5): Fr(5591070156686698065364559, 7931626489314500743872000)
}


def _d1_closure_6():
    H = _H_CLOSURE[6]
    half, st = _D1_INTERIOR[6]
    rows = []
    for r in range(6):
        row = []
        for c in range(9):
            if c < 6:
                q = Fr(-1, 2) if (r, c) == (0, 0) else (Fr(0) if r == c else
                                                        (_Q6_UPPER[(r, c)] if r < c else -_Q6_UPPER[(c, r)]))
            else:
                k = r - c                # Q_rc = -Q_cr, row c interior: Q_cr = d_{r-c}
                q = -st[k + half] if -half <= k <= half else Fr(0)
            row.append(q / H[r])
        while row and row[-1] == 0:
            row.pop()
        rows.append(row)
    return rows


_D1_CLOSURE[6] = _d1_closure_6()

# remainder windows: (difference stencil, interior weight, boundary weights,
#                     list of (offset within window, share) defining B)
_R_WINDOWS = {
    2: [([1, -2, 1], Fr(1, 4), [], [(1, Fr(1))])],
    4: [([-1, 3, -3, 1], Fr(1, 18),
         [Fr(181507, 1719312), Fr(293, 4214), Fr(185, 3528)],
         [(1, Fr(1, 2)), (2, Fr(1, 2))]),
        ([1, -4, 6, -4, 1], Fr(1, 144), [], [(2, Fr(1))])],
    # order 6: windows of widths 5, 6, 7 (alpha = 4, 5, 6); the interior
    # weights are the unique ones that make the interior stencil seven points
    # wide and sixth-order accurate; the five width-5 windows at each end are
    # scaled by the factors _G4_BND, the unique ones that make rows 1.. of
    # D2^FC exact for all (b, u) polynomial pairs of total degree <= 4 (a
    # third-order closure) given the D1 above; every factor is positive
    6: [([1, -4, 6, -4, 1], Fr(1, 80), None, [(1, Fr(1, 3)), (2, Fr(1, 3)), (3, Fr(1, 3))]),
        ([-1, 5, -10, 10, -5, 1], Fr(1, 600), [], [(2, Fr(1, 2)), (3, Fr(1, 2))]),
        ([1, -6, 15, -20, 15, -6, 1], Fr(1, 3600), [], [(3, Fr(1))])],
}
_G4_BND = [Fr(237685172925523195733757321662141117118767, 31602998592421529376702770327325284401500), Fr(227139847450989727703237846776878932224483, 31602998592421529376702770327325284401500), Fr(23788947390956941843, 15300205419202354830), Fr(53028109694882963204, 68850924386410596735), Fr(145701618090536539739, 137701848772821193470)]
_R_WINDOWS[6][0] = (_R_WINDOWS[6][0][0], _R_WINDOWS[6][0][1], [g * _R_WINDOWS[6][0][1] for g in _G4_BND],
                    _R_WINDOWS[6][0][3])

MIN_POINTS = {2: 3, 4: 13, 6: 19}


def _check(n, order):
    if order not in ORDERS:
        raise ValueError("order must be 2, 4 or 6")
    if n < MIN_POINTS[order]:
        raise ValueError(f"need at least {MIN_POINTS[order]} points for order {order}")


def norm_exact(n, order):
    """Diagonal of H/h as exact fractions (Sec. 4, eq. structure_H)."""
    _check(n, order)
    w = [Fr(1)] * n
    for i, v in enumerate(_H_CLOSURE[order]):
        w[i] = v
        w[n - 1 - i] = v
    return w


def d1_exact(n, order):
    """h*D1 as a dense list of exact fractions (Sec. 4)."""
    _check(n, order)
    D = [[Fr(0)] * n for _ in range(n)]
    clos = _D1_CLOSURE[order]
    for r, row in enumerate(clos):
        for c, v in enumerate(row):
            D[r][c] = v
            D[n - 1 - r][n - 1 - c] = -v
    half, st = _D1_INTERIOR[order]
    for r in range(len(clos), n - len(clos)):
        for o, v in zip(range(-half, half + 1), st):
            D[r][r + o] = v
    return D


def windows_exact(n, order):
    """All remainder windows of R(b)*h, exactly.

    Returns a list of (start, stencil, gamma, [(point index, share)]) so that
    h R(b) = sum over windows gamma * (sum share*b[point]) * d d^T with d the
    stencil placed at points start..start+len-1 (Sec. 4, eq. B_structure_1d).
    """
    _check(n, order)
    out = []
    for st, g_in, g_bnd, avg in _R_WINDOWS[order]:
        k = len(st)
        nwin = n - k + 1
        for c in range(nwin):
            g = g_in
            if c < len(g_bnd):
                g = g_bnd[c]
            elif nwin - 1 - c < len(g_bnd):
                g = g_bnd[nwin - 1 - c]
            out.append((c, st, g, [(c + o, s) for o, s in avg]))
    return out


# ------------------------------------------------------- float operators
def norm(n, h, order):
    """Diagonal of H as a float array."""
    return h * np.array([float(v) for v in norm_exact(n, order)])


def d1(n, h, order):
    """D1 as a CSR matrix."""
    D = d1_exact(n, order)
    rows, cols, vals = [], [], []
    for r in range(n):
        for c in range(n):
            if D[r][c] != 0:
                rows.append(r)
                cols.append(c)
                vals.append(float(D[r][c]) / h)
    return sps.csr_matrix((vals, (rows, cols)), shape=(n, n))


class _Windows:
    """Remainder windows as sparse operators: h R(b) = Delta^T diag(g * A b) Delta."""

    def __init__(self, n, order):
        wins = windows_exact(n, order)
        m = len(wins)
        dr, dc, dv, ar, ac, av, g = [], [], [], [], [], [], []
        for w, (c, st, gam, avg) in enumerate(wins):
            for o, v in enumerate(st):
                dr.append(w)
                dc.append(c + o)
                dv.append(float(v))
            for p, s in avg:
                ar.append(w)
                ac.append(p)
                av.append(float(s))
            g.append(float(gam))
        self.delta = sps.csr_matrix((dv, (dr, dc)), shape=(m, n))
        self.avg = sps.csr_matrix((av, (ar, ac)), shape=(m, n))
        self.gamma = np.array(g)


_CACHE = {}


def _ops(n, h, order):
    key = (n, float(h), order)
    if key not in _CACHE:
        _CACHE[key] = (norm(n, h, order), d1(n, h, order), _Windows(n, order))
    return _CACHE[key]


def remainder(b, h, order):
    """R(b) as a CSR matrix (Sec. 4, eq. B_structure_1d)."""
    n = len(b)
    _, _, W = _ops(n, h, order)
    B = W.gamma * (W.avg @ b)
    return (W.delta.T @ sps.diags(B) @ W.delta / h).tocsr()


def d2fc(b, h, order):
    """Adapted fully compatible D2^FC(b) as a CSR matrix (Sec. 4.1)."""
    b = np.asarray(b, dtype=float)
    n = len(b)
    Hd, D, _ = _ops(n, h, order)
    M = D.T @ sps.diags(Hd * b) @ D + remainder(b, h, order)
    E0 = sps.csr_matrix(([1.0], ([0], [0])), shape=(n, n))
    EN = sps.csr_matrix(([1.0], ([n - 1], [n - 1])), shape=(n, n))
    bnd = -E0 @ sps.diags(b) @ D + EN @ sps.diags(b) @ D
    return (sps.diags(1.0 / Hd) @ (-M + bnd)).tocsr()


# ----------------------------------------------- line-wise application
def _along(A, U, axis):
    """Apply the sparse 1-D operator A along ``axis`` of the 2-D array U."""
    if axis == 0:
        return np.asarray(A @ U)
    return np.asarray((A @ U.T).T)


def apply_d1(U, h, order, axis):
    """D1 along one axis of a 2-D grid function (Sec. 4.3, tensor products)."""
    n = U.shape[axis]
    _, D, _ = _ops(n, h, order)
    return _along(D, U, axis)


def apply_d2fc(U, Bc, h, order, axis):
    """D2^FC(b) along every grid line of one axis (Sec. 4.4).

    U, Bc are 2-D arrays of the same shape; line k of Bc is the coefficient for
    line k of U.  Literal SBP form: H^{-1}(-D1^T H b D1 u - R(b) u + boundary).
    """
    n = U.shape[axis]
    Hd, D, W = _ops(n, h, order)
    sh = [1, 1]
    sh[axis] = n
    Hb = Hd.reshape(sh)
    DU = _along(D, U, axis)
    wide = _along(D.T, Hb * Bc * DU, axis)
    shw = [1, 1]
    shw[axis] = -1
    gam = W.gamma.reshape(shw)
    rem = _along(W.delta.T, gam * _along(W.avg, Bc, axis) * _along(W.delta, U, axis), axis) / h
    out = -wide - rem
    if axis == 0:
        out[0, :] -= Bc[0, :] * DU[0, :]
        out[-1, :] += Bc[-1, :] * DU[-1, :]
    else:
        out[:, 0] -= Bc[:, 0] * DU[:, 0]
        out[:, -1] += Bc[:, -1] * DU[:, -1]
    return out / Hb
