"""Pins of the oracle's discrete adjoint (oracle/adjoint.py).

* The C-gradient of the bilinear form w^T D^tot(C) Y is compared with unit
  probes of C: the form is linear in C, so B(C + e) - B(C) is the exact
  derivative along e.  Probes cover corners, faces of every covered type,
  closure rows and interior points, and all 16 tensor entries, for the
  narrow and the wide-stencil operator.
* The misfit gradient (reverse pass of the RK4 map) is compared with central
  finite differences of J along random directions in rho and C.
"""
import numpy as np
import pytest

from oracle import adjoint as AD
from oracle import elastic as E
from oracle import material as M
from oracle import sources as Src
from oracle.geometry import metrics
from paper_2003_12811_amd import workloads as W


def _problem(n1, n2, order, seed, C=None, rho=None, operator='narrow'):
    X1, X2 = W.grid(W.GaussianTopography(0.12, 0.2), n1, n2)
    rho0, C10 = W.paper_random_material((n2, n1), seed)
    Cf = M.full_from_c10(C10) if C is None else C
    rho = rho0 if rho is None else rho
    B = E.Block(X1, X2, rho, Cf, order=order, operator=operator)
    P = E.Problem([B])
    rng = np.random.default_rng(seed)
    P.set_bc(0, 0, E.DISPLACEMENT, g=rng.normal(size=(2, n2)), tfun=lambda t: np.cos(3 * t + 0.2))
    P.set_bc(0, 1, E.TRACTION, g=rng.normal(size=(2, n2)), tfun=lambda t: np.sin(2 * t))
    P.set_bc(0, 2, E.DISPLACEMENT)
    P.set_bc(0, 3, E.TRACTION)
    return P, X1, X2, rho, Cf


def _form(P, w, Y, t):
    return float(np.sum(w.reshape(2, -1) * P.total_operator([Y], t, homogeneous=False)[0]))


@pytest.mark.parametrize("order,n1,n2,operator", [(4, 13, 14, 'narrow'), (2, 7, 8, 'narrow'),
                                                   (4, 14, 15, 'wide'), (2, 7, 8, 'wide')])
def test_coef_gradient_matches_unit_probes(order, n1, n2, operator):
    P, X1, X2, rho, C = _problem(n1, n2, order, 5, operator=operator)
    rng = np.random.default_rng(1)
    w = rng.normal(size=(2, n2, n1))
    Y = rng.normal(size=(2, n2, n1))
    t = 0.37
    g = AD.coef_gradient(P, 0, w, Y, t, homogeneous=False)
    base = _form(P, w, Y, t)
    pts = [(0, 0), (0, n1 - 1), (n2 - 1, 0), (n2 - 1, n1 - 1), (0, 3), (n2 - 1, 4), (5, 0), (6, n1 - 1),
           (1, 1), (2, 4), (n2 // 2, n1 // 2), (3, n1 - 2)]
    worst = 0.0
    scale = np.abs(g).max()
    for (j, i) in pts:
        for comp in [(0, 0, 0, 0), (0, 1, 1, 0), (1, 0, 0, 1), (1, 1, 1, 1), (0, 0, 1, 1), (1, 0, 1, 0),
                     (0, 1, 0, 0), (1, 1, 0, 1)]:
            C2 = C.copy()
            C2[comp + (j, i)] += 1.0
            P2 = _problem(n1, n2, order, 5, C=C2, rho=rho, operator=operator)[0]
            d = _form(P2, w, Y, t) - base
            worst = max(worst, abs(d - g[comp + (j, i)]) / scale)
    assert worst < 1e-10, worst


def _receivers_spec(n):
    return dict(receivers=[(0, np.array([0.3, 0.55, 0.62]), np.array([0.4, 0.62, 0.95]))])


def _source(P, B):
    P.sources.append(Src.point_source(0, B, 0.45, 0.5, (0.3, -1.0), 1.0, 12.0, 0.03))


def test_misfit_gradient_matches_finite_differences():
    n, order, steps = 13, 4, 24
    P, X1, X2, rho, C = _problem(n, n, order, 2)
    _source(P, P.blocks[0])
    spec = _receivers_spec(n)
    dt = 2e-3
    # observed data from a perturbed model
    blob = np.exp(-((X1 - 0.5) ** 2 + (X2 - 0.5) ** 2) / 0.02)
    Pobs = _problem(n, n, order, 2, C=C * (1 + 0.3 * blob), rho=rho * (1 - 0.2 * blob))[0]
    _source(Pobs, Pobs.blocks[0])
    d_obs = AD.forward_receivers(Pobs, spec, steps, dt)
    Jv, g_rho, g_C = AD.misfit_gradient(P, spec, steps, dt, d_obs)
    assert Jv == pytest.approx(AD.misfit(P, spec, steps, dt, d_obs), rel=1e-12)
    assert Jv > 1e-5 * float(np.sum(d_obs ** 2))      # the model change is visible at the receivers
    rng = np.random.default_rng(4)

    def J_of(rho_, C_):
        Pp = _problem(n, n, order, 2, C=C_, rho=rho_)[0]
        _source(Pp, Pp.blocks[0])
        return AD.misfit(Pp, spec, steps, dt, d_obs)

    for trial in range(3):
        drho = rng.normal(size=rho.shape) * (trial != 1)
        dC10 = rng.normal(size=(10,) + rho.shape) * (trial != 0)
        dC = M.full_from_c10(dC10)
        # central differences at eps and eps/2, Richardson-extrapolated (J is
        # strongly curved: the misfit compares nearly equal traces)
        def cd(e):
            return (J_of(rho + e * drho, C + e * dC) - J_of(rho - e * drho, C - e * dC)) / (2 * e)
        eps = 1e-4
        fd = (4.0 * cd(0.5 * eps) - cd(eps)) / 3.0
        ad = float(np.sum(g_rho * drho) + np.sum(g_C * dC))
        assert ad == pytest.approx(fd, rel=1e-8), (trial, ad, fd)
