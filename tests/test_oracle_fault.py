"""Pins of the oracle's interface jump data (Sec. 6, eq. interface_phys and
eq. scheme_interface).

A manufactured solution that jumps across the interface (different
materials, amplitudes and phases on the two sides) satisfies the interface
problem with V = u^a - u^b and Theta = tau^a + tau^b.  With these data the
discrete solution converges at the scheme's rate; with the data left out (or
entered with a flipped sign) the error does not decrease, so a dropped term or
a wrong sign of V or Theta fails the test.
"""
import numpy as np
import pytest

from oracle import timestep as T
from oracle.spec import build
from paper_2003_12811_amd import workloads as W


def _fault_error(n, order=4, jump_data=True, flip=None):
    spec = W.spec_fault(n=n, order=order, jump_data=jump_data)
    if flip is not None:
        k, V, Th, tk, tp = spec['interface_data'][0]
        spec['interface_data'] = [(k, -V if flip == 'V' else V, -Th if flip == 'Theta' else Th, tk, tp)]
    P = build(spec)
    mms = spec['mms']
    w = mms[0]['omega']
    nst, dt = T.steps_for(spec['T'], T.dt_cfl(P, spec['cfl']))
    us = [m['u'].copy() for m in mms]
    vs = [np.zeros_like(u) for u in us]
    t = 0.0
    for _ in range(nst):
        us, vs = T.rk4_step(P, us, vs, t, dt)
        t += dt
    err = 0.0
    for B, u, m in zip(P.blocks, us, mms):
        err += np.sum(B.J * B.H * ((u - m['u'] * np.cos(w * t)) ** 2).sum(0))
    return np.sqrt(err)


def test_fault_mms_converges_with_jump_data():
    errs = [_fault_error(n) for n in (17, 33, 65)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.2, (errs, rates)
    assert errs[-1] < 1e-4, errs


@pytest.mark.parametrize("variant", ['none', 'V', 'Theta'])
def test_fault_mms_fails_without_correct_jump_data(variant):
    """Leaving the data out, or flipping the sign of V or of Theta, leaves an
    O(1) error that does not shrink under refinement."""
    kw = dict(jump_data=False) if variant == 'none' else dict(flip=variant)
    e1, e2 = _fault_error(17, **kw), _fault_error(33, **kw)
    good = _fault_error(33)
    assert e2 > 0.5 * e1, (e1, e2)
    assert e2 > 100 * good, (e2, good)
