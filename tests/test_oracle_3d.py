"""Pins of the 3-D oracle (oracle/elastic3d.py) against what the paper and the
mathematics fix, independently of the GPU path:

* affine maps: exact metric, J, face normals, and the two routes to the face
  scale factor (|a_t1 x a_t2| of Sec. 3.2.2 and J |F_.a| from Nanson's
  formula) agree;
* the H-weighted operator diag(JH) D^tot is symmetric and negative
  semidefinite (Sec. 5, Theorems 1-2) for traction, mixed and displacement
  faces on a curved block with a random major-symmetric stiffness: brute force
  at second order, random bilinear forms and a Lanczos bound at fourth order;
* constant fields span the traction-only null space;
* an extruded plane-strain block reduces exactly to the pinned 2-D operator
  (with beta scaled by 2/3, since the penalty carries d);
* manufactured-solution convergence with traction and displacement data.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import elastic as E2
from oracle import elastic3d as E3
from oracle import timestep as T


def _grid(n1, n2, n3, eps=0.0):
    x1, x2, x3 = np.meshgrid(np.linspace(0, 1, n1), np.linspace(0, 1, n2), np.linspace(0, 1, n3), indexing='ij')
    x1, x2, x3 = (np.transpose(a, (2, 1, 0)) for a in (x1, x2, x3))     # (n3, n2, n1)
    bump = eps * np.sin(np.pi * x1) * np.sin(np.pi * x2) * np.sin(np.pi * x3)
    return x1 + bump, x2 + 0.6 * bump + eps * x3 * x1, x3 - 0.8 * bump


def _random_C(seed, shape, minor=False):
    """Major-symmetric positive definite stiffness, spatially varying."""
    rng = np.random.default_rng(seed)
    if minor:
        Q = rng.normal(size=(6, 6))
        V = Q @ Q.T + 2 * np.eye(6)
        vi = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
        M = np.zeros((9, 9))
        for a, (i, j) in enumerate(vi):
            for b, (k, l) in enumerate(vi):
                for (p, q) in {(i, j), (j, i)}:
                    for (r, s) in {(k, l), (l, k)}:
                        M[3 * p + q, 3 * r + s] = V[a, b]
    else:
        Q = rng.normal(size=(9, 9))
        M = Q @ Q.T + 2 * np.eye(9)
    C0 = M.reshape(3, 3, 3, 3)
    var = 1.0 + 0.2 * np.sin(np.arange(np.prod(shape)).reshape(shape) * 0.37)
    return C0[..., None, None, None] * var, 1.0 + 0.3 * np.cos(np.arange(np.prod(shape)).reshape(shape) * 0.11)


def _problem(n, order, kinds, eps=0.04, seed=3, minor=False):
    X1, X2, X3 = _grid(*n, eps=eps)
    C, rho = _random_C(seed, X1.shape, minor)
    P = E3.Problem3D(E3.Block3D(X1, X2, X3, rho, C, order=order))
    for f, k in enumerate(kinds):
        P.set_bc(f, k)
    return P


TRACTION_ONLY = [E3.TRACTION] * 6
MIXED = [E3.DISPLACEMENT, E3.TRACTION, E3.TRACTION, E3.DISPLACEMENT, E3.TRACTION, E3.DISPLACEMENT]
CLAMPED = [E3.DISPLACEMENT] * 6


def test_affine_metrics_and_normals():
    n1, n2, n3 = 6, 7, 5
    M = np.array([[1.2, 0.3, -0.1], [0.2, 0.9, 0.25], [-0.15, 0.1, 1.1]])
    x1, x2, x3 = _grid(n1, n2, n3)
    X = [M[I, 0] * x1 + M[I, 1] * x2 + M[I, 2] * x3 + 0.3 * I for I in range(3)]
    B = E3.Block3D(*X, 1.0, np.eye(9).reshape(3, 3, 3, 3), order=2)
    # A[i][I] = dX_I/dx_i = M[I, i] exactly (D1 is exact for linear functions)
    for i in range(3):
        for I in range(3):
            assert np.allclose(B.A[i, I], M[I, i], atol=1e-12)
    assert np.allclose(B.J, np.linalg.det(M), atol=1e-12)
    Minv = np.linalg.inv(M)            # dx/dX
    for f, (a, s) in enumerate(E3.FACES3):
        fo = B.faces[f]
        nu = -1.0 if s == 0 else 1.0
        n_exact = nu * Minv[a] / np.linalg.norm(Minv[a])     # gradient of x_a, outward
        assert np.allclose(fo['n'], n_exact[:, None], atol=1e-12)
        # |a_t1 x a_t2| = J |grad x_a| (cofactor identity), two independent routes
        assert np.allclose(fo['Jhat'], np.linalg.det(M) * np.linalg.norm(Minv[a]), rtol=1e-12)
        t1, t2 = [t for t in range(3) if t != a]
        assert np.allclose(fo['Hf'].sum(), 1.0)             # face quadrature of the unit square
        assert fo['Hf'].shape == (B.n[t1] * B.n[t2],)


@pytest.mark.parametrize("kinds,minor", [(TRACTION_ONLY, False), (MIXED, False), (CLAMPED, False), (MIXED, True)])
def test_second_order_operator_is_self_adjoint_and_stable(kinds, minor):
    P = _problem((5, 6, 4), 2, kinds, minor=minor)
    A = P.assemble()
    nrm = np.abs(A).max()
    assert np.abs(A - A.T).max() / nrm < 1e-13
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam[-1] < 1e-12 * np.abs(lam).max()
    if kinds is TRACTION_ONLY:
        # translations are in the null space: three zero eigenvalues
        assert np.sum(np.abs(lam) < 1e-10 * np.abs(lam).max()) >= 3
    else:
        assert lam[-1] < -1e-6 * np.abs(lam).max()


@pytest.mark.parametrize("kinds", [TRACTION_ONLY, MIXED])
def test_fourth_order_operator_is_self_adjoint_and_stable(kinds):
    P = _problem((13, 14, 13), 4, kinds)
    B = P.block
    shp = (3,) + B.J.shape
    w = np.tile((B.J * B.H).ravel(), 3)
    Aop = lambda x: w * P.total_operator(np.asarray(x).reshape(shp)).ravel()
    rng = np.random.default_rng(5)
    scale = None
    for _ in range(3):
        x, y = rng.normal(size=(2, 3 * B.npts))
        ax, ay = Aop(x), Aop(y)
        scale = np.abs(x) @ np.abs(ay)
        assert abs(y @ ax - x @ ay) < 1e-13 * scale
        assert x @ ax < 0
    if kinds is MIXED:
        # strictly negative definite with displacement faces (Lanczos; the
        # traction-only operator's null space makes its largest eigenvalue 0,
        # which the null-space test pins instead)
        lop = spla.LinearOperator((3 * B.npts,) * 2, matvec=Aop, dtype=float)
        lmax = spla.eigsh(lop, k=1, which='LA', return_eigenvectors=False, tol=1e-8, maxiter=3000)[0]
        assert lmax < 0


def test_constants_are_the_traction_only_null_space():
    P = _problem((13, 13, 13), 4, TRACTION_ONLY)
    B = P.block
    for L in range(3):
        u = np.zeros((3,) + B.J.shape)
        u[L] = 1.0
        r = P.total_operator(u)
        assert np.abs(r).max() < 1e-9 * np.abs(B.c).max() / min(B.h) ** 2


@pytest.mark.parametrize("order", [2, 4])
def test_extruded_plane_strain_block_is_the_2d_operator(order):
    n1, n2, n3 = 15, 13, 7 if order == 2 else 13
    x1, x2 = np.meshgrid(np.linspace(0, 1, n1), np.linspace(0, 1, n2))
    X1 = x1 + 0.05 * np.sin(np.pi * x1) * np.sin(np.pi * x2)
    X2 = x2 + 0.1 * np.exp(-((x1 - 0.5) / 0.2) ** 2) * (1 - x2)
    rng = np.random.default_rng(9)
    Q = rng.normal(size=(4, 4))
    C2 = (Q @ Q.T + np.eye(4)).reshape(2, 2, 2, 2)       # major symmetric, no minor symmetry
    var = 1.0 + 0.2 * np.sin(3 * X1 + 2 * X2)
    rho2 = 1.0 + 0.1 * np.cos(X1 - X2)
    C3 = np.zeros((3, 3, 3, 3, n2, n1))
    C3[:2, :2, :2, :2] = C2[..., None, None] * var
    C3[2, 2, 2, 2] = 2.5 * var
    for a in range(2):
        C3[2, a, 2, a] = (1.3 + 0.2 * a) * var
        C3[a, 2, a, 2] = (0.9 + 0.3 * a) * var
    ext = lambda A: np.repeat(A[None], n3, axis=0) if A.ndim == 2 else np.repeat(A[..., None, :, :], n3, axis=-3)
    X3 = np.repeat(np.linspace(0, 1, n3)[:, None, None], n2, axis=1).repeat(n1, axis=2)
    B3 = E3.Block3D(ext(X1), ext(X2), X3, ext(rho2), ext(C3), order=order, beta=2.0 / 3.0)
    P3 = E3.Problem3D(B3, beta=2.0 / 3.0)
    B2 = E2.Block(X1, X2, rho2, C2[..., None, None] * var, order=order)
    P2 = E2.Problem([B2])
    kinds2 = [E2.TRACTION, E2.DISPLACEMENT, E2.DISPLACEMENT, E2.TRACTION]
    for f, k in enumerate(kinds2):
        P2.set_bc(0, f, k)
        P3.set_bc(f, E3.DISPLACEMENT if k == E2.DISPLACEMENT else E3.TRACTION)
    u2 = rng.normal(size=(2, n2, n1))
    u3 = np.zeros((3, n3, n2, n1))
    u3[:2] = u2[:, None]
    r2 = P2.total_operator([u2])[0].reshape(2, n2, n1)
    r3 = P3.total_operator(u3).reshape(3, n3, n2, n1)
    sc = np.abs(r2).max()
    assert np.abs(r3[2]).max() < 1e-12 * sc
    for k in range(n3):
        assert np.abs(r3[:2, k] - r2).max() < 1e-11 * sc


class _MMS:
    """u_L = sin(kX1 + a_L) sin(kX2 + b_L) sin(kX3 + c_L) cos(w t), constant C, rho."""

    def __init__(self, C, rho, k=np.pi):
        self.C, self.rho, self.k = C, rho, k
        self.ph = np.array([[0.3, 1.1, 0.7], [1.4, 0.2, 0.9], [0.5, 0.8, 1.6]])
        cmax = np.abs(C).max()
        self.w = k * np.sqrt(cmax / rho)

    def parts(self, X, L):
        s = [np.sin(self.k * X[m] + self.ph[L, m]) for m in range(3)]
        c = [np.cos(self.k * X[m] + self.ph[L, m]) for m in range(3)]
        return s, c

    def u(self, X):
        return np.stack([np.prod(self.parts(X, L)[0], axis=0) for L in range(3)])

    def grad(self, X):
        """d u_L / d X_m, shape (3 L, 3 m, ...)"""
        out = []
        for L in range(3):
            s, c = self.parts(X, L)
            out.append([self.k * c[m] * np.prod([s[q] for q in range(3) if q != m], axis=0) for m in range(3)])
        return np.array(out)

    def forcing(self, X):
        """rho u_tt - d_I (C_IJKL d_K u_L) at t = 0 (times cos(w t))."""
        k = self.k
        f = -self.rho * self.w ** 2 * self.u(X)
        for L in range(3):
            s, c = self.parts(X, L)
            for I in range(3):
                for K in range(3):
                    if I == K:
                        d2 = -k * k * np.prod(s, axis=0)
                    else:
                        q = 3 - I - K
                        d2 = k * k * c[I] * c[K] * s[q]
                    for J in range(3):
                        f[J] -= self.C[I, J, K, L] * d2
        return f


def _mms_error(n, order, T_end=0.1):
    X = _grid(n, n, n, eps=0.0)
    rng = np.random.default_rng(1)
    Q = rng.normal(size=(6, 6))
    V = Q @ Q.T / 6 + np.eye(6)
    vi = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    C = np.zeros((3, 3, 3, 3))
    for a, (i, j) in enumerate(vi):
        for b, (kk, l) in enumerate(vi):
            for (p, q) in {(i, j), (j, i)}:
                for (r, s) in {(kk, l), (l, kk)}:
                    C[p, q, r, s] = V[a, b]
    rho = 1.3
    m = _MMS(C, rho)
    B = E3.Block3D(*X, rho, C, order=order)
    P = E3.Problem3D(B)
    cosw = lambda t: np.cos(m.w * t)
    P.forcing = (m.forcing(X) / 1.0, cosw)
    G = m.grad(X)
    for f, (a, s) in enumerate(E3.FACES3):
        fo = B.faces[f]
        if f in (1, 4):
            g = m.u(X).reshape(3, -1)[:, fo['idx']]
            P.set_bc(f, E3.DISPLACEMENT, g=g, tfun=cosw)
        else:
            Gf = G.reshape(3, 3, -1)[..., fo['idx']]
            g = np.einsum('If,IJKL,LKf->Jf', fo['n'], C, Gf)
            P.set_bc(f, E3.TRACTION, g=g, tfun=cosw)
    dtm = E3.dt_cfl(B, 0.5)
    nst = int(np.ceil(T_end / dtm))
    dt = T_end / nst
    u, v = [m.u(X)], [np.zeros_like(m.u(X))]
    t = 0.0
    for _ in range(nst):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
    e = u[0] - m.u(X) * np.cos(m.w * T_end)
    return np.sqrt(np.sum((B.J * B.H) * (e ** 2).sum(0)))


@pytest.mark.parametrize("order,ns,rate", [(2, (9, 13, 17), 1.8), (4, (13, 17, 21), 3.3)])
def test_manufactured_solution_converges(order, ns, rate):
    errs = [_mms_error(n, order) for n in ns]
    hs = [1.0 / (n - 1) for n in ns]
    rates = [np.log(errs[i] / errs[i + 1]) / np.log(hs[i] / hs[i + 1]) for i in range(len(ns) - 1)]
    print('3-D manufactured solution, order %d: errors %s, rates %s' % (order, errs, rates))
    assert min(rates) > rate, (errs, rates)
