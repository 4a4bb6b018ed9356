"""Sixth-order operators (Sec. 4; the paper's third order, Sec. 7.1) through
the C ABI, against the oracle's sixth-order operators.

* sbpe_apply on a curvilinear block with every boundary kind carrying data,
  forcing and point sources (FP64 1e-11, FP32 1e-5 relative L2, and the same
  bounds in the max norm on the boundary band), on shapes with ragged tiles;
  on 2x2 blocks with interfaces; on a reversed interface.
* sbpe_advance against the oracle's literal RK4: the manufactured solution
  with traction and displacement data (the error to the exact solution is
  also checked), a source with receivers, the one-launch sweeps and the
  two-stream sweeps (forced with one-row tiles), and a batch (bitwise).
* The energy equals the oracle's and does not grow.
* The full 1025^2 single-block workload: one apply and three RK4 steps.
"""
import sys

import numpy as np
import pytest

from oracle import timestep as T
from oracle.spec import build, receivers
from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W
from parity import TOL, band_max_rel, rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def solver(spec, dtype='f64', **kw):
    from paper_2003_12811_amd.solver import Solver
    return Solver(spec, dtype=dtype, **kw)


def rounded(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == 'f32' else x


def cat(xs):
    return np.concatenate([np.asarray(x, dtype=float).ravel() for x in xs])


def mixed_spec(n1, n2, seed=3):
    X1, X2 = W.grid(W.GaussianTopography(0.15, 0.2), n1, n2)
    rho, C10 = W.paper_random_material((n2, n1), seed)
    rng = np.random.default_rng(seed)
    nf = [n2, n2, n1, n1]
    Q = rng.uniform(0, 1, (2, 2, n2))
    U = np.einsum('ikf,jkf->ijf', Q, Q)
    bc = [(W.DISPLACEMENT, rng.normal(size=(2, nf[0])), W.T_COS, (3.0, 0.2), None),
          (W.ROBIN, rng.normal(size=(2, nf[1])), W.T_RICKER, (5.0, 0.1), U),
          (W.TRACTION, rng.normal(size=(2, nf[2])), W.T_COS, (2.0, -0.4), None),
          (W.DISPLACEMENT, None, W.T_ZERO, None, None)]
    F = rng.normal(size=(2, n2, n1))
    blk = dict(X1=X1, X2=X2, rho=rho, C10=C10, bc=bc, forcing=(F, W.T_COS, (1.5, 0.3)))
    return dict(order=6, blocks=[blk], interfaces=[],
                sources=[(0, 0.37, 0.61, 0.3, -1.0, 2.0, 8.0, 0.05), (0, 0.0, 0.96, 1.0, 0.0, 1.0, 6.0, 0.02)],
                receivers=[])


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
@pytest.mark.parametrize("shape", [(97, 83), (19 + 58, 19), (150, 41)])
def test_sixth_apply_single_block_all_bcs(dtype, shape):
    n1, n2 = shape
    say('order 6 apply single block', dtype, n1, n2)
    spec = mixed_spec(n1, n2)
    P = build(spec)
    sol = solver(spec, dtype)
    try:
        rng = np.random.default_rng(11)
        u = rounded(rng.normal(size=(2, n2, n1)), dtype)
        for t, hom in ((0.13, False), (0.0, True)):
            got = sol.apply([u], t=t, homogeneous=hom)[0].double().cpu().numpy()
            if hom:
                B = P.blocks[0]
                ref = (P.total_operator([u], t, homogeneous=True)[0] / B.rho.ravel()).reshape(2, n2, n1)
            else:
                ref = P.rhs([u], t)[0]
            err, eb = rel(got, ref), band_max_rel(got, ref, 6)
            say('  t', t, 'hom', hom, 'rel L2 %.3e band max %.3e' % (err, eb))
            assert err < TOL[dtype] and eb < TOL[dtype]
    finally:
        sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_sixth_apply_multiblock(dtype):
    n = 45
    say('order 6 apply 2x2 blocks', dtype, n)
    spec = W.spec_c3(n=n, order=6)
    P = build(spec)
    sol = solver(spec, dtype)
    try:
        rng = np.random.default_rng(5)
        us = [rounded(rng.normal(size=(2, n, n)), dtype) for _ in range(4)]
        got = [x.double().cpu().numpy() for x in sol.apply(us, t=0.11)]
        ref = P.rhs(us, 0.11)
        err, eb = rel(cat(got), cat(ref)), band_max_rel(got, ref, 6)
        say('  rel L2 %.3e band max %.3e' % (err, eb))
        assert err < TOL[dtype] and eb < TOL[dtype]
    finally:
        sol.close()


def test_sixth_apply_reversed_interface():
    n = 31
    say('order 6 apply reversed interface')
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
    spec = dict(order=6, blocks=[dict(X1=XA[0], X2=XA[1], rho=ra, C10=Ca, bc=bcA, forcing=None),
                                 dict(X1=XB[0], X2=XB[1], rho=rb, C10=Cb, bc=list(free), forcing=None)],
                interfaces=[(0, 1, 1, 1, True)], sources=[], receivers=[])
    P = build(spec)
    sol = solver(spec, 'f64')
    try:
        rng = np.random.default_rng(8)
        us = [rng.normal(size=(2, n, n)) for _ in range(2)]
        got = [x.cpu().numpy() for x in sol.apply(us)]
        ref = P.rhs(us, 0.0)
        err, eb = rel(cat(got), cat(ref)), band_max_rel(got, ref, 6)
        say('  rel L2 %.3e band max %.3e' % (err, eb))
        assert err < 1e-11 and eb < 1e-11
    finally:
        sol.close()


@pytest.mark.parametrize("kinds", [(0, 0, 0, 0), (0, 2, 0, 2)])
def test_sixth_advance_mms(kinds):
    """The manufactured solution (traction and displacement data, forcing) to
    t = 0.5 against the oracle's literal RK4; both are near the exact solution."""
    n = 49
    say('order 6 MMS advance', kinds)
    spec = W.spec_mms(n=n, order=6, kinds=kinds)
    P = build(spec)
    mm = spec['mms']
    sol = solver(spec, 'f64')
    try:
        nst, dt = T.steps_for(spec['T'], sol.dt_cfl(spec['cfl']))
        sol.set_state([mm['u']], None, 0.0)
        sol.advance(nst, dt)
        ug, vg = sol.state_numpy()
        u, v, t = [mm['u'].copy()], [np.zeros_like(mm['u'])], 0.0
        for _ in range(nst):
            u, v = T.rk4_step(P, u, v, t, dt)
            t += dt
        eu, ev = rel(ug[0], u[0]), rel(vg[0], v[0])
        ex = mm['u'] * np.cos(mm['omega'] * t)
        B = P.blocks[0]
        err = np.sqrt(np.sum(B.J * B.H * ((ug[0] - ex) ** 2).sum(0)))
        say('  %d steps: rel L2 to oracle u %.3e v %.3e; error to exact %.3e' % (nst, eu, ev, err))
        assert eu < 1e-11 and ev < 1e-11
        assert err < 1e-5
    finally:
        sol.close()


@pytest.mark.parametrize("dtype,two_stream", [('f64', False), ('f32', False), ('f64', True), ('f32', True)])
def test_sixth_advance_sources_receivers(dtype, two_stream):
    """A curvilinear block with boundary data, forcing, a source and
    receivers: the one-launch sweeps, or (one-row tiles, over 4096 tiles) the
    two-stream sweeps, against the oracle's literal RK4; then the same shot
    in a batch, bitwise."""
    import torch
    n1, n2 = (600, 470) if two_stream else (131, 97)
    nsteps, t0 = 4, 0.04
    say('order 6 advance', dtype, 'two-stream' if two_stream else 'one launch', n1, n2)
    spec = mixed_spec(n1, n2, seed=7)
    spec['receivers'] = [(0, np.array([0.3, 0.52, 0.99]), np.array([0.4, 0.6, 0.99]))]
    X1, X2 = spec['blocks'][0]['X1'], spec['blocks'][0]['X2']
    u0 = rounded(np.stack([np.sin(3 * X1 + 1) * np.cos(2 * X2), np.cos(2 * X1) * np.sin(3 * X2 + 0.5)]), dtype)
    v0 = rounded(np.stack([np.sin(5 * X1 + 1) * np.cos(2 * X2), np.cos(2 * X1) * np.sin(5 * X2 + 0.5)]), dtype)
    rows = 1 if two_stream else 0
    sol, other = solver(spec, dtype, tile_rows=rows), solver(spec, dtype, tile_rows=rows)
    b = S.sbpe_batch_create(0, torch.cuda.current_stream().cuda_stream, S.F64 if dtype == 'f64' else S.F32, 6)
    try:
        plan = S.sbpe_plan_info(sol.ctx)
        assert plan['fused_sweep'] != two_stream, plan
        dt = sol.dt_cfl(0.5)
        sol.set_state([u0], [v0], t0)
        sol.advance(nsteps, dt)
        ug, vg = sol.state_numpy()
        rg = sol.receivers()
        P = build(spec)
        u, v, t, rec = [u0.copy()], [v0.copy()], t0, []
        for _ in range(nsteps):
            u, v = T.rk4_step(P, u, v, t, dt)
            t += dt
            rec.append(receivers(spec, u))
        eu, ev, er = rel(ug[0], u[0]), rel(vg[0], v[0]), rel(rg, np.array(rec))
        say('  rel L2 u %.3e v %.3e receivers %.3e' % (eu, ev, er))
        assert max(eu, ev, er) < TOL[dtype]
        other.set_state([u0], [v0], t0)
        S.sbpe_batch_add(b, other.ctx, nsteps, dt)
        S.sbpe_batch_advance(b, nsteps)
        S.sbpe_batch_synchronize(b)
        S.sbpe_batch_remove(b, other.ctx)
        ub, vb = other.state_numpy()
        assert np.array_equal(ub[0], ug[0]) and np.array_equal(vb[0], vg[0])
    finally:
        S.sbpe_batch_destroy(b)
        sol.close()
        other.close()


def test_sixth_energy():
    n = 61
    say('order 6 energy', n)
    spec = W.spec_c2(n=n, nrec=0, order=6)
    spec['sources'] = []
    P = build(spec)
    sol = solver(spec, 'f64')
    try:
        rng = np.random.default_rng(4)
        u0, v0 = rng.normal(size=(2, n, n)), rng.normal(size=(2, n, n))
        sol.set_state([u0], [v0], 0.0)
        e_lib, e_or = sol.energy(), P.energy([u0], [v0])
        say('  energy lib %.12e oracle %.12e' % (e_lib, e_or))
        assert abs(e_lib / e_or - 1) < 1e-11
        dt = sol.dt_cfl(0.5)
        prev = e_lib
        for _ in range(5):
            sol.advance(10, dt)
            e = sol.energy()
            assert e <= prev * (1 + 1e-12)
            prev = e
    finally:
        sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_sixth_full_size_c2(dtype):
    """The 1025^2 workload at order 6: one apply (band included) and three RK4
    steps from a smooth state inside the Ricker pulse, against the oracle."""
    n, nsteps = 1025, 3
    say('order 6 full size 1025^2', dtype)
    spec = W.spec_c2(n=n, nrec=16, order=6)
    P = build(spec)
    sol = solver(spec, dtype)
    try:
        x1, x2 = W.reference_grid(n, n)
        u = rounded(np.stack([np.sin(7 * x1) * np.cos(5 * x2), np.cos(3 * x1 + 2 * x2)]) +
                    1e-3 * np.random.default_rng(0).normal(size=(2, n, n)), dtype)
        got = sol.apply([u], t=0.1)[0].double().cpu().numpy()
        ref = P.rhs([u], 0.1)[0]
        err, eb = rel(got, ref), band_max_rel(got, ref, 6)
        say('  apply rel L2 %.3e band max %.3e' % (err, eb))
        assert err < TOL[dtype] and eb < TOL[dtype]
        dt = sol.dt_cfl(0.5)
        u0 = rounded(np.stack([np.sin(7 * x1) * np.cos(5 * x2), np.cos(3 * x1 + 2 * x2)]), dtype)
        v0 = rounded(np.stack([np.cos(4 * x1) * np.sin(3 * x2), np.sin(2 * x1 - x2)]), dtype)
        sol.set_state([u0], [v0], 0.09)
        sol.advance(nsteps, dt)
        ug, vg = sol.state_numpy()
        uo, vo, t = [u0.copy()], [v0.copy()], 0.09
        for _ in range(nsteps):
            uo, vo = T.rk4_step(P, uo, vo, t, dt)
            t += dt
        eu, ev = rel(ug[0], uo[0]), rel(vg[0], vo[0])
        say('  advance rel L2 u %.3e v %.3e' % (eu, ev))
        assert eu < TOL[dtype] and ev < TOL[dtype]
    finally:
        sol.close()
