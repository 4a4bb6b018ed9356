"""Pins of the oracle's displacement-SAT data term (Sec. 5.2, eq. dirichlet_ansatz).

The displacement SAT acts on delta = u - g at the face points.  A manufactured
solution whose boundary displacement enters as g converges at the scheme's
rate; with g's sign flipped or with g left out the discrete solution solves a
different problem and keeps an O(1) error that does not shrink under
refinement.  This pins the sign and the scaling of g in both the penalty term
Z delta and the traction-transpose term T^T delta, on a Cartesian block and on
a curved one (where T mixes both reference directions through the metric).
"""
import numpy as np
import pytest

from oracle import timestep as T
from oracle.spec import build
from paper_2003_12811_amd import workloads as W

TR, DI = W.TRACTION, W.DISPLACEMENT


def _mms_error(n, kinds, mapping=None, order=4, **kw):
    spec = W.spec_mms(n=n, order=order, kinds=kinds, mapping=mapping, **kw)
    P = build(spec)
    mm = spec['mms']
    nst, dt = T.steps_for(spec['T'], T.dt_cfl(P, spec['cfl']))
    u, v, t = [mm['u'].copy()], [np.zeros_like(mm['u'])], 0.0
    for _ in range(nst):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
    B = P.blocks[0]
    ex = mm['u'] * np.cos(mm['omega'] * t)
    return np.sqrt(np.sum(B.J * B.H * ((u[0] - ex) ** 2).sum(0)))


CASES = {
    'cartesian_two_faces': dict(kinds=(TR, DI, TR, DI), mapping=None),
    'curved_three_faces': dict(kinds=(DI, TR, DI, DI), mapping=W.SineWarp(0.05)),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_displacement_data_mms_converges(case):
    errs = [_mms_error(n, **CASES[case]) for n in (17, 33, 65)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 3.4, (errs, rates)
    assert errs[-1] < 1e-4, errs


def test_displacement_data_mms_second_order():
    errs = [_mms_error(n, kinds=(TR, DI, TR, DI), order=2) for n in (17, 33, 65)]
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(rates) > 1.7, (errs, rates)


@pytest.mark.parametrize("variant", ['flipped', 'dropped'])
@pytest.mark.parametrize("case", sorted(CASES))
def test_displacement_data_mms_fails_without_correct_data(case, variant):
    """g with the wrong sign, or no g, leaves an O(1) error that does not
    decrease from 17^2 to 33^2."""
    kw = dict(data_sign=-1.0) if variant == 'flipped' else dict(drop_displacement_data=True)
    e1, e2 = _mms_error(17, **CASES[case], **kw), _mms_error(33, **CASES[case], **kw)
    good = _mms_error(33, **CASES[case])
    assert e2 > 0.5 * e1, (e1, e2)
    assert e2 > 100 * good, (e2, good)
