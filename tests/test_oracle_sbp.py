"""Pins of the 1-D SBP operators of the oracle against what the paper fixes.

Sec. 4: diagonal norm, H D1 + D1^T H = -e0 e0^T + eN eN^T, interior order 2q and
boundary order q; the second-derivative remainder R(b) is symmetric, zero to the
order of accuracy and built from non-negative combinations of b (Lemma 1 needs
every dR/db_s positive semidefinite); the adapted fully compatible operator
loses one order at the end point only (Sec. 4.1).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import sbp

ORD = [2, 4, 6]
R0 = {2: 1, 4: 6, 6: 9}          # closure rows of D2^FC (rows that differ from the interior stencil)


@pytest.mark.parametrize("order", ORD)
@pytest.mark.parametrize("n", [19, 24, 29])
def test_sbp_identity_exact(order, n):
    H = sbp.norm_exact(n, order)
    D = sbp.d1_exact(n, order)
    for i in range(n):
        for j in range(n):
            q = H[i] * D[i][j] + H[j] * D[j][i]
            e = Fr(-1) if i == j == 0 else Fr(1) if i == j == n - 1 else Fr(0)
            assert q == e, (i, j, q)
    assert sum(H) == n - 1          # H integrates 1 over [0, N] exactly


@pytest.mark.parametrize("order", ORD)
def test_d1_accuracy_exact(order):
    n = 20
    q = order // 2
    D = sbp.d1_exact(n, order)
    x = [Fr(k) for k in range(n)]
    nb = len(sbp._D1_CLOSURE[order])
    for p in range(order + 1):
        for r in range(n):
            val = sum(D[r][c] * x[c] ** p for c in range(n))
            ex = p * x[r] ** (p - 1) if p > 0 else Fr(0)
            interior = nb <= r < n - nb
            if p <= q or (interior and p <= order):
                assert val == ex, (p, r)


@pytest.mark.parametrize("order", ORD)
def test_quadrature_exact(order):
    n = 20
    H = sbp.norm_exact(n, order)
    for p in range(order):
        s = sum(H[k] * Fr(k) ** p for k in range(n))
        assert s == Fr((n - 1) ** (p + 1), p + 1), p


def _d2_exact_vs_poly(order, n, pb, pu, rows):
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    b = x ** pb
    u = x ** pu
    D2 = sbp.d2fc(b, h, order).toarray()
    ex = pu * (pb + pu - 1) * x ** (pb + pu - 2) if pb + pu >= 2 and pu >= 1 else 0 * x
    return np.abs(D2[rows] @ u - ex[rows]).max()


@pytest.mark.parametrize("order", ORD)
def test_d2fc_polynomial_orders(order):
    """Interior exact for deg b + deg u <= 2q+1 (order 2q); closure rows other than
    the end point exact for total degree <= q+1 (order q); the end point for
    total degree <= q (order q-1, the adapted operator, Sec. 4.1)."""
    n = 25
    q = order // 2
    r0 = R0[order]
    interior = list(range(r0, n - r0))
    closure = list(range(1, r0)) + list(range(n - r0, n - 1))
    ends = [0, n - 1]
    tol = 1e-8
    for tot in range(0, 2 * q + 2):
        for pb in range(0, tot + 1):
            pu = tot - pb
            if pu == 0:
                continue
            assert _d2_exact_vs_poly(order, n, pb, pu, interior) < tol, (pb, pu)
            if tot <= q + 1 and closure:
                assert _d2_exact_vs_poly(order, n, pb, pu, closure) < tol, (pb, pu)
            if tot <= q:
                assert _d2_exact_vs_poly(order, n, pb, pu, ends) < tol, (pb, pu)
    # and the end point is genuinely of lower order (orders 4 and 6)
    if order >= 4:
        assert _d2_exact_vs_poly(order, n, 0, q + 1, ends) > 1e-6


@pytest.mark.parametrize("order", ORD)
def test_remainder_structure(order):
    """R(b) symmetric, every dR/db_s PSD (Lemma 1), R 1 = R x = 0."""
    n = 25
    h = 1.0 / (n - 1)
    x = np.arange(n) * h
    rng = np.random.default_rng(0)
    b = 1.0 + rng.uniform(0, 1, n)
    R = sbp.remainder(b, h, order).toarray()
    assert np.abs(R - R.T).max() < 1e-13 * np.abs(R).max()
    assert np.abs(R @ np.ones(n)).max() < 1e-12 * np.abs(R).max()
    assert np.abs(R @ x).max() < 1e-12 * np.abs(R).max()
    for s in range(n):
        e = np.zeros(n)
        e[s] = 1.0
        Rs = sbp.remainder(e, h, order).toarray()
        assert np.linalg.eigvalsh(Rs).min() > -1e-12 * max(1.0, np.abs(Rs).max())


@pytest.mark.parametrize("order", ORD)
def test_constant_coefficient_textbook(order):
    n = 31
    h = 1.0 / (n - 1)
    D2 = sbp.d2fc(np.ones(n), h, order).toarray() * h * h
    st = {2: [1.0, -2.0, 1.0], 4: [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12],
          6: [1 / 90, -3 / 20, 3 / 2, -49 / 18, 3 / 2, -3 / 20, 1 / 90]}[order]
    k = len(st) // 2
    for r in range(R0[order], n - R0[order]):
        row = np.zeros(n)
        row[r - k:r + k + 1] = st
        assert np.allclose(D2[r], row, atol=1e-12)


@pytest.mark.parametrize("order", ORD)
def test_fully_compatible_ibp(order):
    """u^T H D2(b) v = -(D1 u)^T H b D1 v - u^T R v + u_N b_N (D1 v)_N - u_0 b_0 (D1 v)_0,
    the fully compatible SBP property (Sec. 4.1 with S = D1); hence the
    'integration by parts twice' antisymmetric part is a pure boundary term."""
    n = 19
    h = 1.0 / (n - 1)
    rng = np.random.default_rng(3)
    b = 1 + rng.uniform(0, 1, n)
    u, v = rng.normal(size=n), rng.normal(size=n)
    H = np.diag(sbp.norm(n, h, order))
    D1 = sbp.d1(n, h, order).toarray()
    D2 = sbp.d2fc(b, h, order).toarray()
    R = sbp.remainder(b, h, order).toarray()
    lhs = u @ H @ D2 @ v
    rhs = -(D1 @ u) @ H @ (b * (D1 @ v)) - u @ R @ v + u[-1] * b[-1] * (D1 @ v)[-1] - u[0] * b[0] * (D1 @ v)[0]
    assert abs(lhs - rhs) < 1e-10 * (abs(lhs) + 1)
    anti = u @ H @ D2 @ v - v @ H @ D2 @ u
    bnd = (u[-1] * b[-1] * (D1 @ v)[-1] - u[0] * b[0] * (D1 @ v)[0]) - (v[-1] * b[-1] * (D1 @ u)[-1] - v[0] * b[0] * (D1 @ u)[0])
    assert abs(anti - bnd) < 1e-10 * (abs(anti) + 1)


def test_boundary_window_weights_are_the_order_conditions():
    """The three boundary weights of the 4th-order d3 windows are the unique
    solution of the closure order conditions (rows 1..5 exact for the cubic
    with constant b); re-derived here in exact arithmetic from D1 and H alone."""
    import sympy as spy
    n = 25
    H = sbp.norm_exact(n, 4)
    D = sbp.d1_exact(n, 4)
    x = [Fr(k) for k in range(n)]
    e = [sum(D[r][c] * x[c] ** 3 for c in range(n)) - 3 * x[r] ** 2 for r in range(n)]
    target = [H[r] * sum(D[r][c] * e[c] for c in range(n)) for r in range(n)]
    g = spy.symbols('g0:3')
    d3 = [-1, 3, -3, 1]
    eqs = []
    for r in range(1, 9):
        expr = 0
        for c in range(0, r + 1):
            if r - c > 3:
                continue
            gam = g[c] if c < 3 else spy.Rational(1, 18)
            expr += 6 * gam * d3[r - c]
        eqs.append(expr - spy.Rational(target[r].numerator, target[r].denominator))
    sol = spy.solve(eqs, g, dict=True)
    assert len(sol) == 1
    got = [Fr(str(sol[0][gi])) for gi in g]
    assert got == sbp._R_WINDOWS[4][0][2]
    assert all(v > 0 for v in got)
