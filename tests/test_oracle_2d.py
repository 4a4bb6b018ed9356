"""Pins of the oracle's 2-D operator, metric terms and SATs.

What the paper fixes (and what a plausible mistake would break):
* Theorems 3 and 5 (Sec. 5.3, 6.1) and the experiment of Sec. 7.2: the total
  operator is self-adjoint, A = diag(JH, JH) D^tot symmetric to round-off, and
  A is negative semidefinite (energy stability) for Robin/traction,
  displacement and interface SATs, with random Cosserat materials.
* Traction-only blocks conserve translations: D^tot applied to a constant is 0.
* Constant coefficients on the identity map reduce to textbook
  constant-coefficient Kronecker stencils.
* Sec. 3.3.1: transformed isotropic stiffness in closed form.
* Sec. 3.3: affine maps give exact metric terms; Nanson's formula.
* eq. n-C_conversion: Jhat T_jl = nu_i c_ijkl D_k (the reference-frame traction).
* eq. borrowing_phys (Sec. 4.5): the volume quadrature bounds h_1/d times the
  face quadrature, sharply at corners; this fixes the weights of the
  displacement and interface penalties.
"""
import numpy as np
import pytest

from oracle import elastic as E, material as M, sbp
from oracle.geometry import metrics
from paper_2003_12811_amd import workloads as W


def _block(order, n1, n2, seed, mapping=None, lim1=(0, 1), lim2=(0, 1)):
    mapping = mapping or W.SineWarp(0.08)
    X1, X2 = W.grid(mapping, n1, n2, lim1, lim2)
    rho, C10 = W.paper_random_material((n2, n1), seed)
    return E.Block(X1, X2, rho, M.full_from_c10(C10), order=order)


CASES = [(0, 0, 0, 0), (2, 0, 0, 0), (0, 2, 2, 0), (2, 2, 2, 2), (1, 2, 0, 1)]


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("bcs", CASES)
def test_self_adjoint_negative_semidefinite(order, bcs):
    B = _block(order, 14, 13, seed=11)
    P = E.Problem([B])
    rng = np.random.default_rng(5)
    for f, k in enumerate(bcs):
        U = None
        if k == E.ROBIN:
            Q = rng.uniform(0, 1, (2, 2, 13 if f < 2 else 14))
            U = np.einsum('ikf,jkf->ijf', Q, Q)          # symmetric PSD U_JL
        P.set_bc(0, f, k, U=U)
    A = P.assemble()
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() / scale < 1e-14
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < 1e-12 * scale
    if E.DISPLACEMENT in bcs or E.ROBIN in bcs:
        assert ev.max() < -1e-6 * scale


@pytest.mark.parametrize("order", [2, 4])
@pytest.mark.parametrize("reverse", [False, True])
def test_interface_self_adjoint(order, reverse):
    n = 13
    A_ = _block(order, n, n, 2, W.SineWarp(0.05), (0, 0.5), (0, 1))
    if not reverse:
        B_ = _block(order, n, n, 3, W.SineWarp(0.05), (0.5, 1), (0, 1))
        itf = E.Interface(0, 1, 1, 0)
    else:
        # second block parameterised with x2 running downwards: its face x1=0
        # is traversed in the opposite direction
        class Flip(W.Mapping):
            def __call__(self, x1, x2):
                return W.SineWarp(0.05)(x1, 1.0 - x2)
        X1, X2 = W.grid(Flip(), n, n, (0.5, 1), (0, 1))
        X1, X2 = X1[:, :], X2[:, :]
        # keep a right-handed parameterisation: reflect x1 as well
        X1, X2 = X1[:, ::-1], X2[:, ::-1]
        rho, C10 = W.paper_random_material((n, n), 3)
        B_ = E.Block(X1, X2, rho, M.full_from_c10(C10), order=order)
        itf = E.Interface(0, 1, 1, 1, reversed=True)
    P = E.Problem([A_, B_], [itf])
    P.set_bc(0, 0, E.DISPLACEMENT)
    A = P.assemble()
    scale = np.abs(A).max()
    assert np.abs(A - A.T).max() / scale < 1e-14
    ev = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert ev.max() < -1e-8 * scale


@pytest.mark.parametrize("order", [2, 4])
def test_traction_translation_null_space(order):
    B = _block(order, 15, 13, seed=4)
    P = E.Problem([B])
    for comp in range(2):
        u = np.zeros((2, 13, 15))
        u[comp] = 1.0
        r = P.total_operator([u])[0]
        assert np.abs(r).max() < 1e-10


@pytest.mark.parametrize("order", [2, 4])
def test_constant_coefficients_textbook(order):
    """Identity map, constant C: interior rows equal
    C_1j1l D2x u_l + C_2j2l D2y u_l + (C_1j2l + C_2j1l) Dx Dy u_l with the
    classical constant-coefficient stencils."""
    n1, n2 = 23, 21
    X1, X2 = W.grid(W.Identity(), n1, n2)
    rng = np.random.default_rng(0)
    C10 = rng.uniform(0, 1, 10)
    C10[[0, 4, 7, 9]] += 4
    C = M.full_from_c10(C10)
    B = E.Block(X1, X2, 1.0, C[..., None, None], order=order)
    u = rng.normal(size=(2, n2, n1))
    r = B.volume(u)
    h1, h2 = 1.0 / (n1 - 1), 1.0 / (n2 - 1)
    d2 = {2: [1, -2, 1], 4: [-1 / 12, 4 / 3, -5 / 2, 4 / 3, -1 / 12]}[order]
    d1 = {2: [-0.5, 0, 0.5], 4: [1 / 12, -2 / 3, 0, 2 / 3, -1 / 12]}[order]
    k = len(d2) // 2
    sl = (slice(8, n2 - 8), slice(8, n1 - 8))

    def sh(a, dj, di):
        return np.roll(np.roll(a, -dj, 0), -di, 1)[sl]

    for j in range(2):
        ref = np.zeros_like(r[j][sl])
        for l in range(2):
            for m, w in zip(range(-k, k + 1), d2):
                ref += C[0, j, 0, l] * w * sh(u[l], 0, m) / h1 ** 2
                ref += C[1, j, 1, l] * w * sh(u[l], m, 0) / h2 ** 2
            for m1, w1 in zip(range(-k, k + 1), d1):
                for m2, w2 in zip(range(-k, k + 1), d1):
                    ref += (C[0, j, 1, l] + C[1, j, 0, l]) * w1 * w2 * sh(u[l], m2, m1) / (h1 * h2)
        assert np.allclose(r[j][sl], ref, rtol=1e-12, atol=1e-9 * np.abs(ref).max())


def test_isotropic_transform_closed_form():
    """Sec. 3.3.1: c_ijkl = J [lam F_ji F_lk + mu (F_Ki d_jl F_Kk + F_li F_jk)]."""
    n = 15
    X1, X2 = W.grid(W.SineWarp(0.1), n, n)
    g = metrics(X1, X2, 4)
    F, J = g['F'], g['J']
    lam, mu = 2.3, 0.7
    c = M.transform(M.isotropic(lam, mu), F, J)
    d = np.eye(2)
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    ref = J * (lam * F[j, i] * F[l, k]
                               + mu * (sum(F[K, i] * F[K, k] for K in range(2)) * d[j, l]
                                       + F[l, i] * F[j, k]))
                    assert np.allclose(c[i, j, k, l], ref, rtol=1e-13, atol=1e-13)


def test_affine_metric_exact_and_nanson():
    n1, n2 = 17, 14
    x1, x2 = W.reference_grid(n1, n2)
    Amat = np.array([[1.3, 0.4], [-0.2, 0.9]])         # X_I = Amat[I, i] x_i
    X1 = Amat[0, 0] * x1 + Amat[0, 1] * x2 + 0.5
    X2 = Amat[1, 0] * x1 + Amat[1, 1] * x2 - 1.0
    g = metrics(X1, X2, 4)
    Finv = np.linalg.inv(Amat)                          # dx_i/dX_I = Finv[i, I]
    for I in range(2):
        for i in range(2):
            assert np.allclose(g['F'][I, i], Finv[i, I], atol=1e-12)
    assert np.allclose(g['J'], np.linalg.det(Amat), atol=1e-12)
    for f in g['faces']:
        a = f['axis']
        t = 1 - a
        assert np.allclose(f['Jhat'], np.hypot(Amat[0, t], Amat[1, t]), atol=1e-12)
        assert np.allclose(np.hypot(*f['n']), 1.0, atol=1e-12)
        # Nanson: Jhat n_I = J F_Ia nu_a
        for I in range(2):
            ref = g['J'].ravel()[f['idx']] * g['F'][I, a].ravel()[f['idx']] * f['nu']
            assert np.allclose(f['Jhat'] * f['n'][I], ref, atol=1e-12)


def test_nonpositive_jacobian_rejected():
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    with pytest.raises(ValueError):
        metrics(X1[:, ::-1], X2, 4)


def test_transformed_stiffness_symmetric_psd():
    B = _block(4, 17, 15, seed=9)
    c = B.c.reshape(4, 4, -1)          # (ij),(kl)
    assert np.abs(c - c.transpose(1, 0, 2)).max() < 1e-12 * np.abs(c).max()
    ev = np.linalg.eigvalsh(np.moveaxis(c, -1, 0))
    assert ev.min() > 0


@pytest.mark.parametrize("order", [2, 4])
def test_reference_frame_traction_identity(order):
    """eq. n-C_conversion with D_K = F_Kk D_k: Jhat T_jl u_l = nu_a c_ajkl D_k u_l."""
    B = _block(order, 16, 14, seed=7)
    rng = np.random.default_rng(1)
    u = rng.normal(size=(2, 14, 16))
    Du = np.stack([np.stack([sbp.apply_d1(u[l], B.h1, order, 1),
                             sbp.apply_d1(u[l], B.h2, order, 0)]) for l in range(2)])   # [l, k]
    for f in range(4):
        fo = B._face_ops[f]
        a = [0, 0, 1, 1][f]
        nu = [-1, 1, -1, 1][f]
        idx = fo['idx']
        ref = np.einsum('jklf,lkf->jf', B.c[a].reshape(2, 2, 2, -1)[..., idx],
                        Du.reshape(2, 2, -1)[..., idx]) * nu
        got = fo['Jhat'] * B.traction(f, u)
        assert np.allclose(got, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


@pytest.mark.parametrize("order", [2, 4])
def test_positivity_property_fixes_the_penalty_weights(order):
    """eq. borrowing_phys (Sec. 4.5): for any nonnegative energy density
    q = s_IJ C_IJKL s_KL, the volume quadrature of J q bounds (1/d) times the
    sum over faces of h_1 (the first norm weight along the face normal) times
    the face quadrature of J q.  The bound is attained at a single corner
    point, where faces of both axes meet, and is off by exactly d = 2 inside
    one face: together these pin d, each axis' h_1 (n1 != n2) and the face
    quadrature that the displacement and interface penalties are built from."""
    B = _block(order, 23, 31, seed=7)
    C = B.C.reshape(2, 2, 2, 2, -1)

    def density(s):
        return np.einsum('IJp,IJKLp,KLp->p', s, C, s)

    def vol(q):
        return np.sum((B.J * B.H).ravel() * q)

    def bound(q):
        return sum(fo['h_1'] * np.sum(fo['Hf'] * fo['Jf'] * q[fo['idx']]) for fo in B._face_ops) / E.DIM

    rng = np.random.default_rng(1)
    s = rng.normal(size=(2, 2, B.npts))
    q = density(s)
    assert q.min() > -1e-12 * q.max()
    assert vol(q) > bound(q) > 0
    n1 = B.n1
    for p, ratio in ((0, 1.0), (n1 - 1, 1.0), (B.npts - 1, 1.0), (7 * n1, 2.0), (n1 - 1 + 11 * n1, 2.0),
                     (9, 2.0), (B.npts - 5, 2.0)):
        m = np.zeros(B.npts)
        m[p] = 1.0
        q = density(s * m)
        assert vol(q) == pytest.approx(ratio * bound(q), rel=1e-13), p
    m = np.zeros(B.npts)
    m[5 * n1 + 6] = 1.0
    assert bound(density(s * m)) == 0.0 and vol(density(s * m)) > 0
