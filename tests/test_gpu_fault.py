"""Interface jump data V and Theta (Sec. 6, eq. scheme_interface) through the
C ABI, against the oracle.

* One RHS evaluation with jump data on a reversed curvilinear interface
  between random materials (the data enter at the stage time through their
  time function), FP64 and FP32.
* The fault manufactured solution (workloads.spec_fault) advanced to t = 0.5:
  the library's state equals the oracle's, and its error against the exact
  solution is the oracle's fourth-order error.
"""
import sys

import numpy as np
import pytest

from oracle import timestep as T
from oracle.spec import build
from paper_2003_12811_amd import workloads as W
from parity import band_max_rel

pytestmark = pytest.mark.gpu
TOL = {'f64': 1e-11, 'f32': 1e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def solver(spec, dtype='f64'):
    from paper_2003_12811_amd.solver import Solver
    return Solver(spec, dtype=dtype)


def rounded(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == 'f32' else x


def _reversed_spec(n, order, dtype, rng):
    XA = W.grid(W.SineWarp(0.05), n, n, (0, 0.5), (0, 1))

    class Flip(W.Mapping):
        def __call__(self, x1, x2):
            return W.SineWarp(0.05)(x1, 1.0 - x2)
    XB = W.grid(Flip(), n, n, (0.5, 1), (0, 1))
    XB = (np.ascontiguousarray(XB[0][:, ::-1]), np.ascontiguousarray(XB[1][:, ::-1]))
    ra, Ca = W.paper_random_material((n, n), 2)
    rb, Cb = W.paper_random_material((n, n), 3)
    free = [(W.TRACTION, None, W.T_ZERO, None, None)] * 4
    bcA = list(free)
    bcA[0] = (W.DISPLACEMENT, None, W.T_ZERO, None, None)
    V = rounded(rng.normal(size=(2, n)), dtype)
    Th = rounded(rng.normal(size=(2, n)), dtype)
    return dict(order=order,
                blocks=[dict(X1=XA[0], X2=XA[1], rho=ra, C10=Ca, bc=bcA, forcing=None),
                        dict(X1=XB[0], X2=XB[1], rho=rb, C10=Cb, bc=list(free), forcing=None)],
                interfaces=[(0, 1, 1, 1, True)],
                interface_data=[(0, V, Th, W.T_COS, (3.0, 0.2))],
                sources=[], receivers=[])


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
@pytest.mark.parametrize("order", [4, 2])
def test_apply_jump_data_reversed_interface(dtype, order):
    n = 29
    say('apply with jump data, reversed interface', dtype, order)
    rng = np.random.default_rng(21)
    spec = _reversed_spec(n, order, dtype, rng)
    P = build(spec)
    sol = solver(spec, dtype)
    try:
        us = [rounded(rng.normal(size=(2, n, n)), dtype) for _ in range(2)]
        t = 0.37
        got = [x.double().cpu().numpy() for x in sol.apply(us, t=t)]
        ref = P.rhs(us, t)
        err = rel(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in ref]))
        # the data part alone (zero state): isolates V and Theta
        zs = [np.zeros((2, n, n)) for _ in range(2)]
        got0 = [x.double().cpu().numpy() for x in sol.apply(zs, t=t)]
        ref0 = P.rhs(zs, t)
        err0 = rel(np.concatenate([g.ravel() for g in got0]), np.concatenate([r.ravel() for r in ref0]))
        eb, eb0 = band_max_rel(got, ref, order), band_max_rel(got0, ref0, order)
        say('  rel L2 %.3e, data part alone %.3e; band max %.3e, %.3e' % (err, err0, eb, eb0))
        assert np.linalg.norm(np.concatenate([r.ravel() for r in ref0])) > 0
        assert err < TOL[dtype] and err0 < TOL[dtype]
        assert eb < TOL[dtype] and eb0 < TOL[dtype]
    finally:
        sol.close()


def test_advance_fault_mms_fp64():
    n = 33
    spec = W.spec_fault(n=n)
    say('advance fault MMS', n)
    P = build(spec)
    mms = spec['mms']
    nst, dt = T.steps_for(spec['T'], T.dt_cfl(P, spec['cfl']))
    sol = solver(spec, 'f64')
    try:
        u0 = [m['u'] for m in mms]
        sol.set_state(u0, None, 0.0)
        sol.advance(nst, dt)
        ug, vg = sol.state_numpy()
        us, vs, t = [u.copy() for u in u0], [np.zeros_like(u) for u in u0], 0.0
        for _ in range(nst):
            us, vs = T.rk4_step(P, us, vs, t, dt)
            t += dt
        eu = rel(np.concatenate([g.ravel() for g in ug]), np.concatenate([r.ravel() for r in us]))
        ev = rel(np.concatenate([g.ravel() for g in vg]), np.concatenate([r.ravel() for r in vs]))
        w = mms[0]['omega']
        err = np.sqrt(sum(np.sum(B.J * B.H * ((g - m['u'] * np.cos(w * t)) ** 2).sum(0))
                          for B, g, m in zip(P.blocks, ug, mms)))
        say('  rel L2 vs oracle u %.3e v %.3e; error vs exact %.3e' % (eu, ev, err))
        assert eu < 1e-11 and ev < 1e-11
        assert err < 1e-4
    finally:
        sol.close()
