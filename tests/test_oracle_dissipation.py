"""Pins of the oracle's dissipative Robin term V u_t (the remark after
eq. sat_traction in Sec. 5.1: Robin conditions T u + U u + V u_t = g with V
symmetric positive semidefinite, imposed by the Robin SAT with the V term
added).

* Energy: with homogeneous data the semidiscrete energy of Sec. 5.1 (with its
  U surface term) changes at exactly the rate -sum_f Jhat H_f v.V v over the
  dissipative faces, at any state (u, v).
* Impedance: for a plane P wave hitting a face with T u + V u_t = 0, the
  continuum reflection coefficient is R = (Z - V)/(Z + V), Z = rho c_P (a
  textbook closed form).  With lambda = 0 the plane wave along x1 is exact on a
  block with traction-free x2 faces; the energy left after the pulse has met
  the face is R^2 of the initial one: nearly 0 for V = Z, 1/9 for V = 2 Z and
  for V = Z/2, 1 for V = 0.
"""
import numpy as np
import pytest

from oracle import elastic as E, material as M, timestep as T
from oracle.geometry import face_index
from paper_2003_12811_amd import workloads as W


def _psd_field(rng, nf, scale=1.0):
    Q = rng.uniform(-1, 1, (2, 2, nf))
    return scale * np.einsum('ikf,jkf->ijf', Q, Q)


@pytest.mark.parametrize("order", [4, 2])
def test_energy_rate_is_the_dissipation(order):
    n1, n2 = 17, 15
    X1, X2 = W.grid(W.GaussianTopography(0.12, 0.2), n1, n2)
    rho, C10 = W.paper_random_material((n2, n1), 3)
    B = E.Block(X1, X2, rho, M.full_from_c10(C10), order=order)
    P = E.Problem([B])
    rng = np.random.default_rng(7)
    nf = [n2, n2, n1, n1]
    V1 = _psd_field(rng, nf[1])
    V3 = _psd_field(rng, nf[3])
    P.set_bc(0, 0, E.DISPLACEMENT)
    P.set_bc(0, 1, E.ROBIN, U=_psd_field(rng, nf[1]), V=V1)
    P.set_bc(0, 3, E.TRACTION, V=V3)
    u = rng.normal(size=(2, n2, n1))
    v = rng.normal(size=(2, n2, n1))
    # dE/dt = v^T (rho J H) a - v^T A u, with A = diag(JH) D^tot symmetric
    a = P.rhs([u], 0.0, [v])[0].reshape(2, -1)
    A = P.assemble()
    M_ = np.tile((B.rho * B.J * B.H).ravel(), 2)
    vf, uf = v.ravel(), u.ravel()
    rate = float(vf @ (M_ * a.ravel()) - vf @ (A @ uf))
    # the dissipation, from the face quadrature directly
    diss = 0.0
    for f, V in ((1, V1), (3, V3)):
        fo = B._face_ops[f]
        vv = B.face_values(f, v)
        diss += float(np.sum(fo['Jhat'] * fo['Hf'] * np.einsum('Jf,JLf,Lf->f', vv, V, vv)))
    assert diss > 0
    assert rate == pytest.approx(-diss, rel=1e-10)


def _pulse_energy_ratio(Vscale, n=81, sigma=0.08):
    lam, mu, rho = 0.0, 1.0, 1.0
    cp, cs = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
    X1, X2 = W.grid(W.Identity(), n, n)
    C10 = W.voigt_to_c10(np.array([lam + 2 * mu, lam, 0.0, lam + 2 * mu, 0.0, mu]))
    C10 = C10[:, None, None] * np.ones((1, n, n))
    B = E.Block(X1, X2, rho * np.ones((n, n)), M.full_from_c10(C10), order=4)
    P = E.Problem([B])
    # x1 = 1: T u + V u_t = 0 with V = Vscale diag(rho c_P, rho c_S) (normal (1, 0))
    V = np.zeros((2, 2, n))
    V[0, 0], V[1, 1] = Vscale * rho * cp, Vscale * rho * cs
    P.set_bc(0, 1, E.TRACTION, V=V)
    g = np.exp(-((X1 - 0.5) / sigma) ** 2)
    u0 = np.stack([g, np.zeros_like(g)])
    v0 = np.stack([cp * (2 * (X1 - 0.5) / sigma ** 2) * g, np.zeros_like(g)])    # u = g(x1 - c_P t): right-going
    e0 = P.energy([u0], [v0])
    nst, dt = T.steps_for(0.62, T.dt_cfl(P, 0.5))
    u, v = [u0], [v0]
    for k in range(nst):
        u, v = T.rk4_step(P, u, v, k * dt, dt)
    return P.energy(u, v) / e0


def test_impedance_face_reflects_the_textbook_fraction():
    # R^2 = ((1 - s) / (1 + s))^2 for V = s Z: 0 at s = 1, 1/9 at s = 2 and at s = 1/2
    r_match = _pulse_energy_ratio(1.0)
    r_double = _pulse_energy_ratio(2.0)
    r_half = _pulse_energy_ratio(0.5)
    r_free = _pulse_energy_ratio(0.0)
    assert r_match < 1e-5, r_match
    assert abs(r_double - 1.0 / 9.0) < 2e-3, r_double
    assert abs(r_half - 1.0 / 9.0) < 2e-3, r_half
    # a traction face reflects everything (RK4 at CFL 0.5 loses a few 1e-5)
    assert abs(r_free - 1.0) < 1e-4, r_free
