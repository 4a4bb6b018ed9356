"""Discrete metric terms of a curvilinear block (oracle, test infrastructure only).

Follows Sec. 3.2 and Sec. 3.3 of the paper:

* F^{-1}_{iI} = dX_I/dx_i is computed with the first-derivative SBP operator of
  the same order as the scheme, applied to the grid coordinates.
* J = det(F^{-1}) and F its inverse; blocks with J <= 0 are rejected.
* On a face with reference normal nu (nu_a = -1 on x_a = 0, +1 on x_a = 1)
  the surface scale factor is the length of the tangential covariant basis
  vector (eq. surfj_app_2d) and the physical normal follows from Nanson's
  formula, Jhat n_I = J F_Ii nu_i (eq. nanson).

Array convention: grid functions have shape (n2, n1), x1 is the fast index;
x_1 = i h1, x_2 = j h2 with h_a = 1/(n_a - 1).

Parity status: pinned (tests/test_oracle_2d.py: affine maps give exact F,
Nanson's formula, unit normals, J > 0 detection).
"""
import numpy as np

from .sbp import apply_d1

# faces: (axis index a in 0/1 for x1/x2, side 0 = lower / 1 = upper)
FACES = [(0, 0), (0, 1), (1, 0), (1, 1)]


def face_index(face, n1, n2):
    """Flat grid indices of the points of a face, ordered along the face."""
    a, s = FACES[face]
    if a == 0:
        i = 0 if s == 0 else n1 - 1
        return np.arange(n2) * n1 + i
    j = 0 if s == 0 else n2 - 1
    return j * n1 + np.arange(n1)


def metrics(X1, X2, order):
    X1 = np.asarray(X1, dtype=float)
    X2 = np.asarray(X2, dtype=float)
    n2, n1 = X1.shape
    h1, h2 = 1.0 / (n1 - 1), 1.0 / (n2 - 1)
    # A[i][I] = dX_I / dx_i
    A = np.empty((2, 2, n2, n1))
    A[0, 0] = apply_d1(X1, h1, order, axis=1)
    A[0, 1] = apply_d1(X2, h1, order, axis=1)
    A[1, 0] = apply_d1(X1, h2, order, axis=0)
    A[1, 1] = apply_d1(X2, h2, order, axis=0)
    J = A[0, 0] * A[1, 1] - A[0, 1] * A[1, 0]
    if np.any(J <= 0):
        raise ValueError("non-positive discrete Jacobian")
    F = np.empty((2, 2, n2, n1))      # F[I][i] = dx_i / dX_I
    F[0, 0] = A[1, 1] / J
    F[0, 1] = -A[0, 1] / J
    F[1, 0] = -A[1, 0] / J
    F[1, 1] = A[0, 0] / J
    faces = []
    for f, (a, s) in enumerate(FACES):
        idx = face_index(f, n1, n2)
        t = 1 - a                       # tangential reference direction
        at = np.stack([A[t, 0].ravel()[idx], A[t, 1].ravel()[idx]])
        Jhat = np.sqrt(at[0] ** 2 + at[1] ** 2)
        nu = -1.0 if s == 0 else 1.0
        Jf = J.ravel()[idx]
        n = np.stack([Jf * F[I, a].ravel()[idx] * nu / Jhat for I in range(2)])
        faces.append(dict(idx=idx, axis=a, side=s, nu=nu, Jhat=Jhat, n=n))
    return dict(A=A, J=J, F=F, h=(h1, h2), faces=faces)
