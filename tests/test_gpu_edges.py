"""Degenerate and invalid calls of the stepping entry points, through the C ABI.

* sbpe_advance with zero steps leaves the bound state bitwise, the time and
  the receiver record unchanged.
* Step counts and sizes that are not valid (negative count; zero, negative,
  NaN or infinite step) fail with SBPE_EINVAL and leave the state bitwise.
* Advancing in pieces (3 + 0 + 5 + 12 steps) reaches the state of one call of
  20 steps (to 1e-13: each call restarts its stage times from the time the
  previous call reached, which rounds differently), and the receiver records
  of the pieces concatenate to the record of the single call.
* The zero state with the data switched off is a fixed point: sbpe_apply
  returns exact zeros (L 0 = 0).
"""
import math
import sys

import numpy as np
import pytest

from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _solver(dtype='f64'):
    from paper_2003_12811_amd.solver import Solver
    return Solver(W.spec_c2(n=97, nrec=8), dtype=dtype)


def _initial(n):
    x1, x2 = W.reference_grid(n, n)
    u0 = np.stack([np.sin(5 * x1) * np.cos(3 * x2), np.cos(2 * x1 + x2)])
    v0 = np.stack([np.cos(3 * x1) * np.sin(4 * x2), np.sin(x1 - 2 * x2)])
    return u0, v0


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_zero_steps_and_invalid_steps_leave_the_state(dtype):
    say('zero and invalid steps', dtype)
    sol = _solver(dtype)
    try:
        u0, v0 = _initial(97)
        dt = sol.dt_cfl(0.5)
        sol.set_state([u0], [v0], 0.05)
        sol.advance(4, dt)
        ua, va = sol.state_numpy()
        ta, ra = sol.time(), sol.receivers()
        sol.advance(0, dt)
        for n, h in ((-1, dt), (3, 0.0), (3, -dt), (3, math.nan), (3, math.inf)):
            with pytest.raises(S.SbpeError) as e:
                sol.advance(n, h)
            assert e.value.code == S.EINVAL
        ub, vb = sol.state_numpy()
        assert np.array_equal(ua[0], ub[0]) and np.array_equal(va[0], vb[0])
        assert sol.time() == ta
        rb = sol.receivers()
        assert rb.shape == ra.shape and np.array_equal(ra, rb)
    finally:
        sol.close()


def test_advance_in_pieces_matches_one_call():
    say('advance in pieces')
    one, parts = _solver(), _solver()
    try:
        u0, v0 = _initial(97)
        dt = one.dt_cfl(0.5)
        one.set_state([u0], [v0], 0.05)
        one.advance(20, dt)
        parts.set_state([u0], [v0], 0.05)
        for n in (3, 0, 5, 12):
            parts.advance(n, dt)
        (u1,), (v1,) = one.state_numpy()
        (u2,), (v2,) = parts.state_numpy()
        r1, r2 = one.receivers(), parts.receivers()
        assert abs(one.time() - parts.time()) < 1e-14
        assert r1.shape == r2.shape == (20, 8, 2)
        for a, b in ((u1, u2), (v1, v2), (r1, r2)):
            err = np.linalg.norm(a - b) / np.linalg.norm(a)
            say('  rel L2 %.3e' % err)
            assert err < 1e-13
    finally:
        one.close()
        parts.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_zero_state_is_a_fixed_point(dtype):
    say('zero state', dtype)
    sol = _solver(dtype)
    try:
        z = np.zeros((2, 97, 97))
        (a,) = sol.apply([z], t=0.1, homogeneous=True)
        a = a.double().cpu().numpy()
        assert np.all(np.isfinite(a)) and not np.any(a)
    finally:
        sol.close()
