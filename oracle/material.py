"""Stiffness tensors and their transformation (oracle, test infrastructure only).

* Generalised Hooke's law with major symmetry only, C_IJKL = C_KLIJ
  (Sec. 3, eq. hooke, symmetry_phys).
* Transformed density and stiffness rho~ = J rho, c_ijkl = F_Ii J C_IjKl F_Kk
  (Sec. 3.2.1, eq. transf_density_stiffness).
* Isotropic stiffness lambda d_IJ d_KL + mu (d_IK d_JL + d_IL d_JK) (Sec. 3.3.1).

Layouts.  A full 2-D tensor field is an array C[I, J, K, L, ...] with indices
0/1.  The compact major-symmetric form ("C10") lists the upper triangle of the
4x4 matrix C_(IJ)(KL) with pair order 11, 12, 21, 22:
C1111, C1112, C1121, C1122, C1212, C1221, C1222, C2121, C2122, C2222.
Voigt form (normal materials with minor symmetry) is c11, c12, c16, c22, c26,
c66 with index 1 <-> 11, 2 <-> 22, 6 <-> 12 and no factor 2.

Parity status: pinned (tests/test_oracle_2d.py: major symmetry and
semidefiniteness of c, isotropic closed form of Sec. 3.3.1).
"""
import numpy as np

PAIRS = [(0, 0), (0, 1), (1, 0), (1, 1)]
C10_ORDER = [(p, q) for p in range(4) for q in range(p, 4)]


def full_from_c10(C10):
    """C10 (10, ...) -> full tensor (2, 2, 2, 2, ...)."""
    C10 = np.asarray(C10, dtype=float)
    shp = C10.shape[1:]
    C = np.zeros((2, 2, 2, 2) + shp)
    for m, (p, q) in enumerate(C10_ORDER):
        I, J = PAIRS[p]
        K, L = PAIRS[q]
        C[I, J, K, L] = C10[m]
        C[K, L, I, J] = C10[m]
    return C


def c10_from_full(C):
    return np.stack([C[PAIRS[p] + PAIRS[q]] for p, q in C10_ORDER])


def full_from_voigt(V):
    """Voigt (6, ...) = c11, c12, c16, c22, c26, c66 -> full tensor."""
    V = np.asarray(V, dtype=float)
    c11, c12, c16, c22, c26, c66 = V
    vidx = {(0, 0): 0, (1, 1): 1, (0, 1): 2, (1, 0): 2}
    M = {(0, 0): c11, (0, 1): c12, (0, 2): c16, (1, 1): c22, (1, 2): c26, (2, 2): c66}
    C = np.zeros((2, 2, 2, 2) + V.shape[1:])
    for I in range(2):
        for J in range(2):
            for K in range(2):
                for L in range(2):
                    a, b = vidx[(I, J)], vidx[(K, L)]
                    C[I, J, K, L] = M[(min(a, b), max(a, b))]
    return C


def isotropic(lam, mu):
    d = np.eye(2)
    lam = np.asarray(lam, dtype=float)
    mu = np.asarray(mu, dtype=float)
    C = np.zeros((2, 2, 2, 2) + lam.shape)
    for I in range(2):
        for J in range(2):
            for K in range(2):
                for L in range(2):
                    C[I, J, K, L] = lam * d[I, J] * d[K, L] + mu * (d[I, K] * d[J, L] + d[I, L] * d[J, K])
    return C


def transform(C, F, J):
    """c_ijkl = F_Ii J C_IjKl F_Kk (eq. transf_density_stiffness).

    F[I, i, ...] = dx_i/dX_I, J = det(dX/dx).
    """
    return np.einsum('Ii...,IjKl...,Kk...->ijkl...', F, C, F) * J
