"""Time integration and time-step selection (oracle, test infrastructure only).

* Classical fourth-order Runge-Kutta on the first-order system
  (u, v = u_t)' = (v, a(u, v, t)), with forcing and boundary data evaluated at
  the stage times t, t + dt/2, t + dt/2, t + dt (Sec. 7.1); v enters a only
  through dissipative Robin terms.
* dt = CFL * min over grid points of h / v_max, with v_max the largest
  quasi-P speed of the transformed material (rho~, c) in the reference domain,
  i.e. the square root of the largest eigenvalue of rho~^{-1} xi_i c_ijkl xi_k
  maximised over unit directions xi (Sec. 3.1 eq. christoffel, Sec. 7).  The
  paper maximises with fmincon; here a dense sweep over directions followed by a
  parabolic refinement of the best direction.  Blocks whose two reference
  spacings differ use the smaller one.

Parity status: pinned (tests/test_oracle_time.py: isotropic closed form
v_P = sqrt((lambda + 2 mu)/rho), RK4 energy decay, manufactured-solution
convergence rates).
"""
import numpy as np


def rk4_step(problem, us, vs, t, dt):
    """One classical RK4 step on (u, v); returns (u_new, v_new)."""
    a1 = problem.rhs(us, t, vs)
    u2 = [u + 0.5 * dt * v for u, v in zip(us, vs)]
    v2 = [v + 0.5 * dt * a for v, a in zip(vs, a1)]
    a2 = problem.rhs(u2, t + 0.5 * dt, v2)
    u3 = [u + 0.5 * dt * v for u, v in zip(us, v2)]
    v3 = [v + 0.5 * dt * a for v, a in zip(vs, a2)]
    a3 = problem.rhs(u3, t + 0.5 * dt, v3)
    u4 = [u + dt * v for u, v in zip(us, v3)]
    v4 = [v + dt * a for v, a in zip(vs, a3)]
    a4 = problem.rhs(u4, t + dt, v4)
    un = [u + dt / 6.0 * (v1 + 2 * vb + 2 * vc + vd)
          for u, v1, vb, vc, vd in zip(us, vs, v2, v3, v4)]
    vn = [v + dt / 6.0 * (p + 2 * q + 2 * r + s)
          for v, p, q, r, s in zip(vs, a1, a2, a3, a4)]
    return un, vn


def christoffel_vmax2(rho_t, c, nang=720):
    """Pointwise max over directions of the largest eigenvalue of xi c xi / rho~."""
    shp = rho_t.shape
    cf = c.reshape(2, 2, 2, 2, -1)
    r = rho_t.ravel()

    def lam(th):
        x = np.array([np.cos(th) + 0.0 * r, np.sin(th) + 0.0 * r])
        G = np.einsum('ip,ijklp,kp->jlp', x, cf, x)
        tr = G[0, 0] + G[1, 1]
        disc = np.sqrt(np.maximum((G[0, 0] - G[1, 1]) ** 2 + 4 * G[0, 1] * G[1, 0], 0.0))
        return 0.5 * (tr + disc) / r

    ths = np.linspace(0.0, np.pi, nang, endpoint=False)
    vals = np.stack([lam(t) for t in ths])
    k = np.argmax(vals, axis=0)
    best = vals[k, np.arange(vals.shape[1])]
    dth = np.pi / nang
    # parabolic refinement around the best sampled direction
    th0 = ths[k]
    fm, f0, fp = lam(th0 - dth), best, lam(th0 + dth)
    den = fm - 2 * f0 + fp
    off = np.where(den < 0, 0.5 * (fm - fp) / np.where(den < 0, den, 1.0), 0.0)
    off = np.clip(off, -1.0, 1.0)
    refined = lam(th0 + off * dth)
    return np.maximum(best, refined).reshape(shp)


def dt_cfl(problem, cfl):
    """dt = CFL * min h / v_max over all blocks (Sec. 7)."""
    best = np.inf
    for B in problem.blocks:
        v2 = christoffel_vmax2(B.rho * B.J, B.c)
        h = min(B.h1, B.h2)
        best = min(best, h / np.sqrt(v2.max()))
    return cfl * best


def steps_for(T, dtmax):
    """Number of equal steps reaching T without exceeding dtmax, and the step."""
    n = int(np.ceil(T / dtmax - 1e-12))
    return n, T / n
