"""sbpe_advance_noalloc (time-function table in the library's device scratch
array) against sbpe_advance, through the C ABI: two calls in a row on
different contexts, the second with a smaller grid and fewer steps, so the
second call runs over scratch contents left by the first.  Results must be
equal bit for bit (the same kernels on the same tabulated values)."""
import sys

import numpy as np
import pytest

from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _spec(n):
    """Every kind of time-tabulated data: boundary data on a displacement and
    a traction face, forcing, a Ricker source, receivers."""
    spec = W.spec_c2(n=n, nrec=6)
    rng = np.random.default_rng(n)
    blk = spec['blocks'][0]
    bc = list(blk['bc'])
    bc[2] = (W.DISPLACEMENT, rng.normal(size=(2, n)), W.T_COS, (3.0, 0.2), None)
    bc[0] = (W.TRACTION, rng.normal(size=(2, n)), W.T_RICKER, (8.0, 0.05), None)
    blk['bc'] = bc
    blk['forcing'] = (rng.normal(size=(2, n, n)), W.T_COS, (2.0, 0.1))
    return spec


def _pair(n, dtype, nsteps):
    from paper_2003_12811_amd.solver import Solver
    spec = _spec(n)
    ref, new = Solver(spec, dtype), Solver(spec, dtype)
    try:
        dt = ref.dt_cfl(0.5)
        x1, x2 = W.reference_grid(n, n)
        u0 = np.stack([np.sin(5 * x1) * np.cos(3 * x2), np.cos(2 * x1 + x2)])
        v0 = np.stack([np.cos(4 * x1 - x2), np.sin(3 * x1) * x2])
        for s in (ref, new):
            s.set_state([u0], [v0], 0.02)
        S.sbpe_advance(ref.ctx, nsteps, dt)
        S.sbpe_reserve_steps(new.ctx, nsteps)
        S.sbpe_advance_noalloc(new.ctx, nsteps, dt)
        (ur,), (vr,) = ref.state_numpy()
        (un,), (vn,) = new.state_numpy()
        rr, rn = ref.receivers(), new.receivers()
        say('  n=%d %s %d steps: max |du| %.3e |dv| %.3e |drec| %.3e' % (
            n, dtype, nsteps, np.abs(un - ur).max(), np.abs(vn - vr).max(), np.abs(rn - rr).max()))
        assert rr.shape == (nsteps, 6, 2) and np.abs(rr).max() > 0
        assert np.array_equal(un, ur) and np.array_equal(vn, vr) and np.array_equal(rn, rr)
        assert S.sbpe_get_time(new.ctx) == S.sbpe_get_time(ref.ctx)
    finally:
        ref.close()
        new.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_noalloc_advance_equals_advance(dtype):
    say('no-allocation advance', dtype)
    _pair(97, dtype, 30)     # first call
    _pair(61, dtype, 12)     # second call: smaller grid, fewer steps, stale scratch beyond its table


def test_noalloc_advance_limits():
    from paper_2003_12811_amd.solver import Solver
    say('no-allocation advance limits')
    sol = Solver(_spec(33), 'f64')
    try:
        dt = sol.dt_cfl(0.5)
        sol.set_state(None, None, 0.0)
        # receivers without reserved capacity
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_advance_noalloc(sol.ctx, 5, dt)
        assert e.value.code == S.ESTATE
        # more steps than the scratch table holds (9 items per block + 1 source, 3 values each)
        S.sbpe_reserve_steps(sol.ctx, 20000)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_advance_noalloc(sol.ctx, 20000, dt)
        assert e.value.code == S.EINVAL
        assert S.sbpe_get_time(sol.ctx) == 0.0
        (u,), (v,) = sol.state_numpy()
        assert not u.any() and not v.any()
        S.sbpe_advance_noalloc(sol.ctx, 4000, dt)       # 4000 * 10 * 3 <= 131072
        assert abs(S.sbpe_get_time(sol.ctx) - 4000 * dt) < 1e-9
    finally:
        sol.close()
