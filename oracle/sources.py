"""Point sources, receivers and the Ricker wavelet (oracle, test infrastructure only).

* Ricker wavelet W(t) = (1 - 2 pi^2 a^2 (t - t0)^2) exp(-pi^2 a^2 (t - t0)^2)
  with peak frequency a (Sec. 7.4).
* Point force f_J = dir_J amp W(t) delta(X - X0) (Sec. 7.4).  The paper cites a
  discrete delta function without printing it; the reading used here is the
  tensor product of 1-D weights on the four nearest grid points of each
  reference direction (shifted inward at faces) that satisfy the moment
  conditions sum_m w_m x_m^p = x0^p, p = 0..3.  In the physical inner product
  the discrete delta is d_p = w_p / (J_p H_p), so that sum_p J_p H_p d_p phi_p
  = sum_p w_p phi_p.  Receivers sample sum_p w_p u_p, the adjoint of the source.
  Locations are given in reference coordinates x in [0, 1]^2.

Parity status: pinned (tests/test_oracle_time.py: moment conditions, exactness
for cubic polynomials, source/receiver adjointness, alpha_M / alpha_P = 2.40 of
Sec. 7.4).
"""
import numpy as np


def ricker(t, fpeak, t0):
    a = (np.pi * fpeak * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def weights_1d(x0, n):
    """Four-point moment-matching weights at reference position x0 on n points."""
    h = 1.0 / (n - 1)
    m0 = int(np.floor(x0 / h)) - 1
    m0 = min(max(m0, 0), n - 4)
    idx = np.arange(m0, m0 + 4)
    # the moment conditions are solved in local coordinates xi = (x - x_m0)/h,
    # which span the same cubic polynomials and keep the system well conditioned
    xi = np.arange(4.0)
    xi0 = (x0 - m0 * h) / h
    V = np.vstack([xi ** p for p in range(4)])
    w = np.linalg.solve(V, np.array([xi0 ** p for p in range(4)]))
    return idx, w


def weights_2d(x1, x2, n1, n2):
    i, wi = weights_1d(x1, n1)
    j, wj = weights_1d(x2, n2)
    idx = (j[:, None] * n1 + i[None, :]).ravel()
    w = (wj[:, None] * wi[None, :]).ravel()
    return idx, w


def point_source(block_id, block, x1, x2, direction, amp, fpeak, t0):
    idx, w = weights_2d(x1, x2, block.n1, block.n2)
    return dict(block=block_id, idx=idx, w=w, dir=np.asarray(direction, dtype=float),
                tfun=lambda t: amp * ricker(t, fpeak, t0))


def sample(u, x1, x2):
    """Receiver value sum_p w_p u_p for a field u of shape (2, n2, n1)."""
    n2, n1 = u.shape[1:]
    idx, w = weights_2d(x1, x2, n1, n2)
    return np.array([np.dot(w, u[c].ravel()[idx]) for c in range(2)])
