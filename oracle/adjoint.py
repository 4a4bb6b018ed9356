"""Discrete adjoint of the receiver misfit (oracle, test infrastructure only).

Misfit of a forward run with classical RK4 (Sec. 7.1) and receivers sampled
after every step:

    J = 1/2 sum_{n=1..N} sum_r |S_r u_n - d_{n,r}|^2.

Parameters are the density rho and the stiffness C (every entry C_IJKL
treated as independent; a major-symmetric perturbation puts the same value at
IJKL and KLIJ).  The semidiscrete right-hand side is

    a(u, t) = rho^{-1} (D^tot(C) u + f(t) + sources(t)),

with D^tot = J^{-1} DD_ik(c_ijkl) + SAT (Sec. 5), linear in C through the
transformed stiffness c = F J C F (Sec. 3.2.1) and through the SATs.

The gradient is the exact derivative of the discrete map:

* reverse pass of the RK4 step written as y_{n+1} = y_n + dt sum b_i k_i,
  k_i = f(y_n + dt c_i k_{i-1}), f(u, v) = (v, a(u)); the state adjoint uses
  the transpose of the assembled operator (dense, small grids only);
* parameter terms: for a stage with adjoint weight z (the v-part of the
  stage-slope adjoint) and stage displacement Y,
  d/drho: -z . a / rho pointwise; d/dC: the gradient of the bilinear form
  (z/rho)^T D^tot(C) Y, written out term by term from the definitions:
    - narrow terms: w^T D2^FC(b) y with D2^FC(b) = H^{-1}(-D1^T H b D1 - R(b)
      - e0 b0 e0^T D1 + eN bN eN^T D1) and R(b) = sum_w gamma_w B_w(b) d_w d_w^T / h
      (Sec. 4, eq. sbp_property_2nd_der, B_structure_1d; Sec. 4.1); with the
      wide-stencil operator D_i b D_i (Sec. 7.1) these terms take the form of
      the mixed ones, (D_i^T w) (D_i y);
    - mixed terms: w^T D_i (c D_k y) -> (D_i^T w) (D_k y) (Sec. 4.6);
    - traction SAT: -(JH)^{-1} e_f Jhat H_f n_I C_IJKL D_K y_L (Sec. 5.1);
    - displacement SAT: (JH)^{-1} (T^T - Z^T) e_f Jhat H_f delta (Sec. 5.2).

Interfaces are not covered (NotImplementedError).

Parity status: pinned (tests/test_oracle_adjoint.py: the C-gradient of the
bilinear form against exact unit probes of C, which are exact because the form
is linear in C, at interior, closure and face points of every covered face
type; the misfit gradient against central finite differences of J).
"""
import numpy as np

from . import sbp
from . import timestep as T
from .elastic import TRACTION, ROBIN, DISPLACEMENT, INTERFACE, DIM


# ----------------------------------------------------------- bilinear forms
def d2fc_coef_grad(W, Y, h, order, axis):
    """d/db of sum over lines of w^T D2^FC(b) y, for every line of ``axis``."""
    n = W.shape[axis]
    Hd, D, Win = sbp._ops(n, h, order)
    sh = [1, 1]
    sh[axis] = n
    Hb = Hd.reshape(sh)
    Z = W / Hb                                       # H^{-1} w
    DZ = sbp._along(D, Z, axis)
    DY = sbp._along(D, Y, axis)
    g = -Hb * DZ * DY
    shw = [1, 1]
    shw[axis] = -1
    gam = Win.gamma.reshape(shw)
    g -= sbp._along(Win.avg.T, gam * sbp._along(Win.delta, Z, axis) * sbp._along(Win.delta, Y, axis), axis) / h
    if axis == 0:
        g[0, :] -= Z[0, :] * DY[0, :]
        g[-1, :] += Z[-1, :] * DY[-1, :]
    else:
        g[:, 0] -= Z[:, 0] * DY[:, 0]
        g[:, -1] += Z[:, -1] * DY[:, -1]
    return g


def coef_gradient(P, k, w, Y, t=0.0, homogeneous=True):
    """Gradient with respect to C (shape (2, 2, 2, 2, n2, n1)) of the bilinear
    form w^T D^tot(C) Y on block k (w, Y of shape (2, n2, n1)); the boundary
    data enter the displacement SAT through delta = Y - g(t) unless homogeneous."""
    B = P.blocks[k]
    n1, n2, o, h1, h2 = B.n1, B.n2, B.order, B.h1, B.h2
    w = np.asarray(w, dtype=float).reshape(2, n2, n1)
    Y = np.asarray(Y, dtype=float).reshape(2, n2, n1)
    # volume: (w / J)^T DD(c) Y, then c = F J C F
    z = w / B.J
    gc = np.zeros((2, 2, 2, 2, n2, n1))
    D1x, D1y = sbp._ops(n1, h1, o)[1], sbp._ops(n2, h2, o)[1]
    for j in range(2):
        for l in range(2):
            if B.operator == 'wide':
                # w^T D_i (b D_i y) -> (D_i^T w) (D_i y), like the mixed terms
                gc[0, j, 0, l] += sbp._along(D1x.T, z[j], 1) * sbp.apply_d1(Y[l], h1, o, axis=1)
                gc[1, j, 1, l] += sbp._along(D1y.T, z[j], 0) * sbp.apply_d1(Y[l], h2, o, axis=0)
            else:
                gc[0, j, 0, l] += d2fc_coef_grad(z[j], Y[l], h1, o, axis=1)
                gc[1, j, 1, l] += d2fc_coef_grad(z[j], Y[l], h2, o, axis=0)
            gc[0, j, 1, l] += sbp._along(D1x.T, z[j], 1) * sbp.apply_d1(Y[l], h2, o, axis=0)
            gc[1, j, 0, l] += sbp._along(D1y.T, z[j], 0) * sbp.apply_d1(Y[l], h1, o, axis=1)
    gC = np.einsum('Ii...,ijkl...,Kk...->IjKl...', B.F, gc, B.F) * B.J
    gCf = gC.reshape(2, 2, 2, 2, -1)
    JH = (B.J * B.H).ravel()
    wflat = w.reshape(2, -1)
    for f in range(4):
        bc = B.bc[f]
        fo = B._face_ops[f]
        idx, n, Ff, Jh, Hf = fo['idx'], fo['n'], fo['Ff'], fo['Jhat'], fo['Hf']
        if bc['kind'] in (TRACTION, ROBIN):
            # -(w_J / JH) Jhat H_f n_I C_IJKL D_K Y_L at the face
            Du = np.stack([[fo['ED'][kk] @ Y[L].ravel() for kk in range(2)] for L in range(2)])
            DK = np.einsum('Kkf,Lkf->LKf', Ff, Du)
            wh = -(wflat[:, idx] / JH[idx]) * Jh * Hf                       # [J, f]
            gCf[..., idx] += np.einsum('Jf,If,LKf->IJKLf', wh, n, DK)
        elif bc['kind'] == DISPLACEMENT:
            delta = B.face_values(f, Y)
            if not homogeneous:
                delta = delta - P._data(bc, t, len(idx))
            om = Jh * Hf * delta                                            # omega_L
            what = wflat / JH                                               # w / JH, volume
            Dw = np.stack([[fo['ED'][kk] @ what[J] for kk in range(2)] for J in range(2)])   # [J, k, f]
            DKw = np.einsum('Kkf,Jkf->JKf', Ff, Dw)                         # D_K (w_J / JH) at the face
            gCf[..., idx] += np.einsum('If,Lf,JKf->ILKJf', n, om, DKw)
            zf = P.beta * DIM * Jh / (fo['h_1'] * fo['Jf'])
            gCf[..., idx] -= np.einsum('f,If,Kf,Jf,Lf->ILKJf', zf, n, n, what[:, idx], om)
        elif bc['kind'] == INTERFACE:
            raise NotImplementedError('coefficient gradients across interfaces')
    return gC


# --------------------------------------------------------------- the misfit
def _sample_ops(spec, P):
    """Receiver sampling as (block, idx, w) per receiver (moment weights; the
    discrete delta function is cited in Sec. 7.3-7.4)."""
    from .sources import weights_2d
    ops = []
    for (bid, x1, x2) in spec.get('receivers', []):
        B = P.blocks[bid]
        for a, b in zip(x1, x2):
            idx, w = weights_2d(a, b, B.n1, B.n2)
            ops.append((bid, idx, w))
    return ops


def sample(ops, us):
    return np.array([[np.dot(w, us[b][c].ravel()[idx]) for c in range(2)] for (b, idx, w) in ops])


def sample_transpose(ops, r, P):
    out = [np.zeros((2, B.npts)) for B in P.blocks]
    for (b, idx, w), rr in zip(ops, r):
        for c in range(2):
            np.add.at(out[b][c], idx, w * rr[c])
    return [o.reshape(2, B.n2, B.n1) for o, B in zip(out, P.blocks)]


def forward_receivers(P, spec, nsteps, dt, t0=0.0):
    """Receiver traces (nsteps, nrec, 2) of a run from rest."""
    ops = _sample_ops(spec, P)
    us = [np.zeros((2, B.n2, B.n1)) for B in P.blocks]
    vs = [np.zeros_like(u) for u in us]
    t = t0
    out = []
    for _ in range(nsteps):
        us, vs = T.rk4_step(P, us, vs, t, dt)
        t += dt
        out.append(sample(ops, us))
    return np.array(out)


def misfit(P, spec, nsteps, dt, d_obs):
    r = forward_receivers(P, spec, nsteps, dt) - d_obs
    return 0.5 * float(np.sum(r * r))


def misfit_gradient(P, spec, nsteps, dt, d_obs):
    """(J, dJ/drho per block (n2, n1), dJ/dC per block (2, 2, 2, 2, n2, n1))
    by the reverse pass of the discrete RK4 map (single block, small grids)."""
    if len(P.blocks) != 1 or P.interfaces:
        raise NotImplementedError('single block only')
    B = P.blocks[0]
    ops = _sample_ops(spec, P)
    # forward, keeping the state at every step
    us = [np.zeros((2, B.n2, B.n1))]
    vs = [np.zeros_like(us[0])]
    states = []
    t = 0.0
    Jval = 0.0
    res = []
    for n in range(nsteps):
        states.append((us, vs, t))
        us, vs = T.rk4_step(P, us, vs, t, dt)
        t += dt
        r = sample(ops, us) - d_obs[n]
        res.append(r)
        Jval += 0.5 * float(np.sum(r * r))
    # homogeneous operator D^tot as a dense matrix (its transpose drives the adjoint)
    A = P.assemble()                                    # diag(JH) D^tot
    JH2 = np.tile((B.J * B.H).ravel(), 2)
    Dt = A / JH2[:, None]
    DtT = Dt.T
    rho = B.rho.ravel()
    shape = (2, B.n2, B.n1)
    g_rho = np.zeros(B.npts)
    g_C = np.zeros((2, 2, 2, 2, B.n2, B.n1))
    ub = sample_transpose(ops, res[-1], P)[0].reshape(2, -1)
    vb = np.zeros_like(ub)
    bw = (1 / 6, 1 / 3, 1 / 3, 1 / 6)
    cw = (0.0, 0.5, 0.5, 1.0)
    for n in range(nsteps - 1, -1, -1):
        (u0, v0, tn) = states[n]
        u0, v0 = u0[0].reshape(2, -1), v0[0].reshape(2, -1)
        # stages of the step (Sec. 7.1)
        U, V, Aacc = [], [], []
        ku = kv = None
        for i in range(4):
            if i == 0:
                Ui, Vi = u0, v0
            else:
                Ui, Vi = u0 + dt * cw[i] * ku, v0 + dt * cw[i] * kv
            ai = P.rhs([Ui.reshape(shape)], tn + cw[i] * dt)[0].reshape(2, -1)
            U.append(Ui)
            V.append(Vi)
            Aacc.append(ai)
            ku, kv = Vi, ai
        kub = [dt * b * ub for b in bw]
        kvb = [dt * b * vb for b in bw]
        yu, yv = ub.copy(), vb.copy()
        for i in range(3, -1, -1):
            # k_i = (V_i, a(U_i)): adjoint of the stage input
            zr = kvb[i] / rho
            Yu = (DtT @ zr.ravel()).reshape(2, -1)
            Yv = kub[i]
            g_rho += -np.sum(kvb[i] * Aacc[i], axis=0) / rho
            g_C += coef_gradient(P, 0, zr.reshape(shape), U[i].reshape(shape), tn + cw[i] * dt, homogeneous=False)
            if i > 0:
                kub[i - 1] = kub[i - 1] + dt * cw[i] * Yu
                kvb[i - 1] = kvb[i - 1] + dt * cw[i] * Yv
            yu += Yu
            yv += Yv
        ub, vb = yu, yv
        if n > 0:
            ub = ub + sample_transpose(ops, res[n - 1], P)[0].reshape(2, -1)
    return Jval, g_rho.reshape(B.n2, B.n1), g_C
