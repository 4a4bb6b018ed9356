"""Pins of the oracle's wide-stencil operator D_i c D_i (the operator the
narrow-stencil D2^FC(c) of Sec. 4.1 is compared with in Sec. 7.1).

* Constant coefficient: every interior row is the first-derivative stencil
  convolved with itself (a textbook identity of the wide second derivative).
* The two operators differ by the SBP remainder: H (D1 b D1 - D2^FC(b)) is
  symmetric positive semidefinite for positive b (the construction of
  D2^FC(b) in Sec. 4 subtracts a positive semidefinite R(b)).
* The 2-D operator with traction SATs is H-symmetric and negative
  semidefinite (brute force), like the narrow one.
* The C1 manufactured solution converges at fourth order with the wide
  operator as well, and the narrow operator is the more accurate one: slightly
  at second order, by an order of magnitude at fourth order on the finest grid
  (the comparison of Sec. 7.1).
* The narrow operator has the larger spectral radius (Sec. 7.1).  With
  displacement SATs on every face the penalty sets the largest eigenvalue and
  the two differ by a few per cent, as the paper reports for its domain with a
  displacement-bounded scatterer; with traction faces only the narrow
  operator's grid-scale interior mode, which the wide operator does not see,
  makes the difference tens of per cent.
"""
import numpy as np
import pytest

from oracle import elastic as E, material as M, sbp, timestep as T
from oracle.geometry import face_index
from paper_2003_12811_amd import workloads as W


@pytest.mark.parametrize("order", [4, 2])
def test_wide_interior_row_is_squared_first_derivative(order):
    n, h = 41, 0.1
    D = sbp.d1(n, h, order)
    D = D.toarray() if hasattr(D, 'toarray') else np.asarray(D)
    Wd = D @ D                      # D1 c D1 with c = 1
    row = n // 2
    # the interior first-derivative stencil, and its square by convolution
    half = 2 if order == 4 else 1
    s1 = D[row, row - half: row + half + 1]
    s2 = np.convolve(s1, s1)
    got = Wd[row, row - 2 * half: row + 2 * half + 1]
    assert np.allclose(got, s2, rtol=0, atol=1e-12 / h ** 2)
    assert np.allclose(s1 * h, [1 / 12, -2 / 3, 0, 2 / 3, -1 / 12] if order == 4 else [-0.5, 0, 0.5], atol=1e-14)


@pytest.mark.parametrize("order", [4, 2])
def test_wide_minus_narrow_is_the_psd_remainder(order):
    rng = np.random.default_rng(4)
    n, h = 30, 1.0 / 29
    b = rng.uniform(0.5, 2.0, n)
    D = sbp.d1(n, h, order)
    D = D.toarray() if hasattr(D, 'toarray') else np.asarray(D)
    Hd = sbp.norm(n, h, order)
    wide = D @ np.diag(b) @ D
    narrow = sbp.d2fc(b, h, order)
    narrow = narrow.toarray() if hasattr(narrow, 'toarray') else np.asarray(narrow)
    Rm = np.diag(Hd) @ (wide - narrow)
    assert np.allclose(Rm, Rm.T, atol=1e-9 * np.abs(Rm).max())
    lam = np.linalg.eigvalsh(0.5 * (Rm + Rm.T))
    assert lam.min() > -1e-9 * lam.max()
    assert lam.max() > 0        # the operators do differ


def _wide_problem(order, n1=16, n2=15, seed=2):
    X1, X2 = W.grid(W.SineWarp(0.06), n1, n2)
    rho, C10 = W.paper_random_material((n2, n1), seed)
    B = E.Block(X1, X2, rho, M.full_from_c10(C10), order=order, operator='wide')
    return E.Problem([B])


@pytest.mark.parametrize("order", [4, 2])
def test_wide_operator_self_adjoint_negative_semidefinite(order):
    P = _wide_problem(order)
    A = P.assemble()              # diag(JH) D^tot, traction on every face
    assert np.allclose(A, A.T, atol=1e-9 * np.abs(A).max())
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam.max() < 1e-9 * np.abs(lam).max()


def _mms_error(order, n, operator, T_end=0.5):
    C10 = W.voigt_to_c10(np.array(W.VOIGT_C1))
    X1, X2 = W.grid(W.Identity(), n, n)
    mm = W.mms_c1(X1, X2, C10)
    B = E.Block(X1, X2, 1.0, mm['C'][..., None, None], order=order, operator=operator)
    P = E.Problem([B])
    w = mm['omega']
    tf = lambda t: np.cos(w * t)
    for f in range(4):
        g = W.traction_data(mm, face_index(f, n, n), W.outward_normal(W.Identity(), f, n, n))
        P.set_bc(0, f, E.TRACTION, g=g, tfun=tf)
    P.forcing[0] = (mm['f'], tf)
    nst, dt = T.steps_for(T_end, T.dt_cfl(P, 0.5))
    u, v, t = [mm['u'].copy()], [np.zeros_like(mm['u'])], 0.0
    for _ in range(nst):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
    ex = mm['u'] * np.cos(w * t)
    return np.sqrt(np.sum(B.J * B.H * ((u[0] - ex) ** 2).sum(0)))


def test_wide_mms_convergence_and_narrow_is_more_accurate():
    wide = [_mms_error(4, n, 'wide') for n in (17, 33, 65)]
    rates = [np.log2(wide[i] / wide[i + 1]) for i in range(2)]
    assert min(rates) > 3.0, (wide, rates)
    narrow = [_mms_error(4, n, 'narrow') for n in (33, 65)]
    ratio = [w / n for w, n in zip(wide[1:], narrow)]
    assert ratio[1] > 8 and ratio[1] > ratio[0], ratio
    ratio2 = _mms_error(2, 33, 'wide') / _mms_error(2, 33, 'narrow')
    assert 1.1 < ratio2 < 3, ratio2


def _spectral_radius(order, operator, displacement):
    n = 25
    C10 = W.voigt_to_c10(np.array(W.VOIGT_C1))
    X1, X2 = W.grid(W.SineWarp(0.06), n, n)
    C = M.full_from_c10(np.broadcast_to(C10[..., None, None], C10.shape + (n, n)).copy())
    P = E.Problem([E.Block(X1, X2, 1.0, C, order=order, operator=operator)])
    if displacement:
        for f in range(4):
            P.set_bc(0, f, E.DISPLACEMENT)
    A = P.assemble()
    m = np.concatenate([np.tile((B.J * B.H * B.rho).ravel(), 2) for B in P.blocks])
    s = 1.0 / np.sqrt(m)
    return np.abs(np.linalg.eigvalsh(0.5 * (s[:, None] * (A + A.T) * s[None, :]))).max()


@pytest.mark.parametrize("order,bound", [(4, 0.05), (2, 0.15)])
def test_narrow_spectral_radius_slightly_larger(order, bound):
    rn, rw = (_spectral_radius(order, op, True) for op in ('narrow', 'wide'))
    assert 0 < (rn - rw) / rw < bound, (rn, rw)
    tn, tw = (_spectral_radius(order, op, False) for op in ('narrow', 'wide'))
    assert (tn - tw) / tw > 0.2, (tn, tw)
