"""Time stepping through the two-stream launch path, against the oracle.

On grids with 4096 interior tiles or more, every RK sweep runs the interior
tiles (one wave per tile, both fields) on the context stream and the assembled
frame operator on a second stream.  The full-size workloads that take this
path are too large for the oracle's literal RK4, so these tests force it at
oracle sizes with one-row tiles, and compare whole states (FP64 1e-11, FP32
1e-5 relative L2):

* one curvilinear block with every boundary type carrying data, a Robin matrix
  U, dissipative Robin terms V u_t on a Robin and a traction face (the remark
  after eq. sat_traction, Sec. 5.1), forcing, a point source and receivers,
  for both orders and both operators (narrow D2^FC of Sec. 4.1, wide D_i c D_i
  of Sec. 7.1), and the same shot advanced in a batch (bitwise);
* 2x2 conforming blocks (the interface SAT of Sec. 6) with material contrast.
"""
import sys

import numpy as np
import pytest

from oracle import timestep as T
from oracle.spec import build, receivers
from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W

pytestmark = pytest.mark.gpu
TOL = {'f64': 1e-11, 'f32': 1e-5}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def rounded(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == 'f32' else x


def _psd(rng, nf, scale):
    Q = rng.uniform(-1, 1, (2, 2, nf))
    return scale * np.einsum('ikf,jkf->ijf', Q, Q)


def _block_spec(n1, n2, order, operator, seed=11):
    X1, X2 = W.grid(W.GaussianTopography(0.15, 0.2), n1, n2)
    rho, C10 = W.paper_random_material((n2, n1), seed)
    rng = np.random.default_rng(seed)
    nf = [n2, n2, n1, n1]
    bc = [(W.DISPLACEMENT, rng.normal(size=(2, nf[0])), W.T_COS, (3.0, 0.2), None),
          (W.ROBIN, rng.normal(size=(2, nf[1])), W.T_RICKER, (5.0, 0.1), _psd(rng, nf[1], 1.0)),
          (W.TRACTION, rng.normal(size=(2, nf[2])), W.T_COS, (2.0, -0.4), None),
          (W.TRACTION, None, W.T_ZERO, None, None)]
    F = rng.normal(size=(2, n2, n1))
    blk = dict(X1=X1, X2=X2, rho=rho, C10=C10, bc=bc, forcing=(F, W.T_COS, (1.5, 0.3)))
    return dict(order=order, operator=operator, blocks=[blk], interfaces=[],
                dissipation=[(0, 1, _psd(rng, nf[1], 2.0)), (0, 3, _psd(rng, nf[3], 2.0))],
                sources=[(0, 0.37, 0.61, 0.3, -1.0, 2.0, 8.0, 0.05)],
                receivers=[(0, np.array([0.3, 0.52, 0.99]), np.array([0.4, 0.6, 0.99]))])


def _smooth(X1, X2, a, dtype):
    return rounded(np.stack([np.sin(a * X1 + 1) * np.cos(2 * X2), np.cos(2 * X1) * np.sin(a * X2 + 0.5)]), dtype)


def _oracle_advance(spec, us, vs, t, dt, nsteps):
    P = build(spec)
    u, v, rec = [x.copy() for x in us], [x.copy() for x in vs], []
    for _ in range(nsteps):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
        rec.append(receivers(spec, u))
    return u, v, np.array(rec)


@pytest.mark.parametrize("dtype,order,operator", [
    ('f64', 4, 'narrow'), ('f32', 4, 'narrow'), ('f64', 2, 'narrow'),
    ('f64', 4, 'wide'), ('f32', 2, 'wide')])
def test_two_stream_advance_single_block(dtype, order, operator):
    import torch
    from paper_2003_12811_amd.solver import Solver
    n1, n2, nsteps, t0 = 600, 470, 4, 0.04
    say('two-stream advance', dtype, order, operator, n1, n2)
    spec = _block_spec(n1, n2, order, operator)
    X1, X2 = spec['blocks'][0]['X1'], spec['blocks'][0]['X2']
    u0, v0 = _smooth(X1, X2, 3.0, dtype), _smooth(X1, X2, 5.0, dtype)
    sol = Solver(spec, dtype=dtype, tile_rows=1)
    other = Solver(spec, dtype=dtype, tile_rows=1)
    b = S.sbpe_batch_create(0, torch.cuda.current_stream().cuda_stream, S.F64 if dtype == 'f64' else S.F32, order)
    try:
        plan = S.sbpe_plan_info(sol.ctx)
        assert plan['interior_workgroups'] >= 4096 and not plan['fused_sweep'], plan
        dt = sol.dt_cfl(0.5)
        sol.set_state([u0], [v0], t0)
        sol.advance(nsteps, dt)
        ug, vg = sol.state_numpy()
        rg = sol.receivers()
        u, v, rec = _oracle_advance(spec, [u0], [v0], t0, dt, nsteps)
        eu, ev, er = rel(ug[0], u[0]), rel(vg[0], v[0]), rel(rg, rec)
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


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_two_stream_advance_multiblock(dtype):
    from paper_2003_12811_amd.solver import Solver
    n, nsteps, t0 = 257, 4, 0.08
    say('two-stream multiblock advance', dtype, n)
    spec = W.spec_c3(n=n)
    us = [_smooth(B['X1'], B['X2'], 3.0 + k, dtype) for k, B in enumerate(spec['blocks'])]
    vs = [_smooth(B['X1'], B['X2'], 6.0 - k, dtype) for k, B in enumerate(spec['blocks'])]
    sol = Solver(spec, dtype=dtype, tile_rows=1)
    try:
        plan = S.sbpe_plan_info(sol.ctx)
        assert plan['interior_workgroups'] >= 4096 and not plan['fused_sweep'], plan
        dt = sol.dt_cfl(0.5)
        sol.set_state(us, vs, t0)
        sol.advance(nsteps, dt)
        ug, vg = sol.state_numpy()
        rg = sol.receivers()
        u, v, rec = _oracle_advance(spec, us, vs, t0, dt, nsteps)
        eu = rel(np.concatenate([x.ravel() for x in ug]), np.concatenate([x.ravel() for x in u]))
        ev = rel(np.concatenate([x.ravel() for x in vg]), np.concatenate([x.ravel() for x in v]))
        er = rel(rg, rec)
        say('  rel L2 u %.3e v %.3e receivers %.3e' % (eu, ev, er))
        assert max(eu, ev, er) < TOL[dtype]
    finally:
        sol.close()
