"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle.

Tolerances (relative L2): FP64 1e-11, FP32 1e-5.  FP32 cases feed both sides
the same FP32-rounded inputs (the oracle promotes them to FP64).
"""
import sys

import numpy as np
import pytest

from oracle import elastic as E, timestep as T
from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W

from oracle.spec import build, receivers
from parity import TOL, band_max_rel

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def solver(spec, dtype='f64', **kw):
    from paper_2003_12811_amd.solver import Solver
    return Solver(spec, dtype=dtype, **kw)


def rounded(x, dtype):
    return x.astype(np.float32).astype(np.float64) if dtype == 'f32' else x


def mixed_spec(n1, n2, order=4, seed=3):
    """One curvilinear block, Cosserat random material, every boundary type with data,
    forcing and a point source."""
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
    return dict(order=order, blocks=[blk], interfaces=[],
                sources=[(0, 0.37, 0.61, 0.3, -1.0, 2.0, 8.0, 0.05), (0, 0.0, 0.96, 1.0, 0.0, 1.0, 6.0, 0.02)],
                receivers=[])


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
@pytest.mark.parametrize("order", [4, 2])
@pytest.mark.parametrize("shape", [(97, 83), (13 + 64, 13)])
def test_apply_single_block_all_bcs(dtype, order, shape):
    n1, n2 = shape
    if order == 2:
        n1, n2 = n1 - 3, n2 + 2
    say('apply single block', dtype, order, n1, n2)
    spec = mixed_spec(n1, n2, order)
    P = build(spec)
    sol = solver(spec, dtype)
    rng = np.random.default_rng(11)
    u = rounded(rng.normal(size=(2, n2, n1)), dtype)
    for t, hom in ((0.13, False), (0.0, True)):
        got = sol.apply([u], t=t, homogeneous=hom)[0].double().cpu().numpy()
        if hom:
            L = P.total_operator([u], t, homogeneous=True)[0]
            B = P.blocks[0]
            ref = (L / B.rho.ravel()).reshape(2, n2, n1)
        else:
            ref = P.rhs([u], t)[0]
        err, eb = rel(got, ref), band_max_rel(got, ref, order)
        say('  t', t, 'hom', hom, 'rel L2', err, 'band max', eb)
        assert err < TOL[dtype] and eb < TOL[dtype]
    sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
@pytest.mark.parametrize("n", [45, 77])
def test_apply_multiblock_c3_geometry(dtype, n):
    say('apply 2x2 blocks', dtype, n)
    spec = W.spec_c3(n=n)
    P = build(spec)
    sol = solver(spec, dtype)
    rng = np.random.default_rng(5)
    us = [rounded(rng.normal(size=(2, n, n)), dtype) for _ in range(4)]
    got = [x.double().cpu().numpy() for x in sol.apply(us, t=0.11)]
    ref = P.rhs(us, 0.11)
    err = rel(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in ref]))
    eb = band_max_rel(got, ref, 4)
    say('  rel L2', err, 'band max', eb)
    assert err < TOL[dtype] and eb < TOL[dtype]
    sol.close()


@pytest.mark.parametrize("order", [4, 2])
def test_apply_reversed_interface(order):
    n = 29
    say('apply reversed interface', order)
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
    spec = dict(order=order, blocks=[dict(X1=XA[0], X2=XA[1], rho=ra, C10=Ca, bc=bcA, forcing=None),
                                     dict(X1=XB[0], X2=XB[1], rho=rb, C10=Cb, bc=list(free), forcing=None)],
                interfaces=[(0, 1, 1, 1, True)], sources=[], receivers=[])
    P = build(spec)
    sol = solver(spec, 'f64')
    rng = np.random.default_rng(8)
    us = [rng.normal(size=(2, n, n)) for _ in range(2)]
    got = [x.cpu().numpy() for x in sol.apply(us)]
    ref = P.rhs(us, 0.0)
    err = rel(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in ref]))
    eb = band_max_rel(got, ref, order)
    say('  rel L2', err, 'band max', eb)
    assert err < 1e-11 and eb < 1e-11
    sol.close()


def test_advance_mms_c1_fp64():
    """Config 1 end to end: 65^2, MMS forcing and traction data, CFL 0.5 to t = 0.5."""
    spec = W.spec_c1(65)
    say('advance C1 MMS 65^2 fp64')
    P = build(spec)
    dt_lib = None
    sol = solver(spec, 'f64')
    dt_lib = sol.dt_cfl(0.5)
    dt_or = T.dt_cfl(P, 0.5)
    assert abs(dt_lib / dt_or - 1) < 1e-6
    nst, dt = T.steps_for(0.5, dt_or)
    assert nst == 140
    u0 = spec['mms']['u']
    sol.set_state([u0], None, 0.0)
    sol.advance(nst, dt)
    ug, vg = sol.state_numpy()
    u, v, t = [u0.copy()], [np.zeros_like(u0)], 0.0
    for _ in range(nst):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
    eu, ev = rel(ug[0], u[0]), rel(vg[0], v[0])
    say('  rel L2 u', eu, 'v', ev, 't', sol.time())
    assert eu < 1e-11 and ev < 1e-11
    assert abs(sol.time() - 0.5) < 1e-12
    exact = u0 * np.cos(spec['mms']['omega'] * 0.5)
    B = P.blocks[0]
    err = np.sqrt(np.sum(B.J * B.H * ((ug[0] - exact) ** 2).sum(0)))
    say('  MMS l2 error', err)
    assert err < 2e-5
    sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_advance_source_receivers_c2_small(dtype):
    n, nsteps = 97, 60
    say('advance C2 geometry', n, dtype)
    spec = W.spec_c2(n=n, nrec=8)
    P = build(spec)
    sol = solver(spec, dtype)
    dt = T.dt_cfl(P, 0.5)
    sol.set_state(None, None, 0.0)
    sol.advance(nsteps, dt)
    ug, vg = sol.state_numpy()
    rg = sol.receivers()
    u, v, t = [np.zeros((2, n, n))], [np.zeros((2, n, n))], 0.0
    rec = []
    for _ in range(nsteps):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
        rec.append(receivers(spec, u))
    rec = np.array(rec)
    eu, ev, er = rel(ug[0], u[0]), rel(vg[0], v[0]), rel(rg, rec)
    say('  rel L2 u', eu, 'v', ev, 'receivers', er, 'max|u|', np.abs(u[0]).max())
    assert rg.shape == rec.shape
    assert np.abs(u[0]).max() > 0
    assert max(eu, ev, er) < TOL[dtype]
    sol.close()


def test_energy_and_determinism():
    n = 61
    say('energy and determinism', n)
    spec = W.spec_c2(n=n, nrec=0)
    spec['sources'] = []
    P = build(spec)
    sol = solver(spec, 'f64')
    rng = np.random.default_rng(4)
    u0 = rng.normal(size=(2, n, n))
    v0 = rng.normal(size=(2, n, n))
    sol.set_state([u0], [v0], 0.0)
    e_lib = sol.energy()
    e_or = P.energy([u0], [v0])
    say('  energy lib', e_lib, 'oracle', e_or)
    assert abs(e_lib / e_or - 1) < 1e-11
    dt = T.dt_cfl(P, 0.5)
    prev = e_lib
    for _ in range(5):
        sol.advance(10, dt)
        e = sol.energy()
        assert e <= prev * (1 + 1e-12)
        prev = e
    u1, v1 = sol.state_numpy()
    sol.set_state([u0], [v0], 0.0)
    sol.advance(50, dt)
    u2, v2 = sol.state_numpy()
    assert np.array_equal(u1[0], u2[0]) and np.array_equal(v1[0], v2[0])
    sol.close()


def test_energy_guard_trips_on_oversized_step():
    n = 41
    say('energy guard', n)
    spec = W.spec_c2(n=n, nrec=0)
    spec['sources'] = []
    sol = solver(spec, 'f64')
    rng = np.random.default_rng(1)
    sol.set_state([rng.normal(size=(2, n, n))], None, 0.0)
    S.sbpe_set_energy_guard(sol.ctx, 2, 1e-6)
    dt = sol.dt_cfl(0.5) * 6.0
    with pytest.raises(S.SbpeError) as e:
        sol.advance(40, dt)
    assert e.value.code == S.EUNSTABLE
    sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_full_size_c2_apply(dtype):
    """Config 2 at its full size (1025^2), in the kernels the benchmark times."""
    n = 1025
    say('full size C2 apply', dtype)
    spec = W.spec_c2(n=n, nrec=0)
    P = build(spec)
    sol = solver(spec, dtype)
    x1, x2 = W.reference_grid(n, n)
    u = rounded(np.stack([np.sin(7 * x1) * np.cos(5 * x2), np.cos(3 * x1 + 2 * x2)]) +
                1e-3 * np.random.default_rng(0).normal(size=(2, n, n)), dtype)
    got = sol.apply([u], t=0.1)[0].double().cpu().numpy()
    ref = P.rhs([u], 0.1)[0]
    err, eb = rel(got, ref), band_max_rel(got, ref, 4)
    say('  rel L2', err, 'band max', eb)
    assert err < TOL[dtype] and eb < TOL[dtype]
    sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_full_size_c2_advance(dtype):
    """Config 2 at its full size (1025^2, source, receivers), advanced by the
    one-launch RK sweeps the benchmark times (in the launch shapes its tuning
    picked on the measured machine: 20-row tiles, 2 frame groups per frame
    workgroup in FP64 and 4 in FP32), against the oracle's literal RK4: the
    whole state after 3 steps from a smooth nonzero state."""
    n, nsteps = 1025, 3
    say('full size C2 advance', dtype)
    spec = W.spec_c2(n=n, nrec=16)
    P = build(spec)
    sol = solver(spec, dtype, tile_rows=20)
    sol.set_frame_loop(2 if dtype == 'f64' else 4)
    try:
        plan = S.sbpe_plan_info(sol.ctx)
        assert plan['fused_sweep']
        dt = sol.dt_cfl(0.5)
        x1, x2 = W.reference_grid(n, n)
        u0 = rounded(np.stack([np.sin(7 * x1) * np.cos(5 * x2), np.cos(3 * x1 + 2 * x2)]), dtype)
        v0 = rounded(np.stack([np.cos(4 * x1) * np.sin(3 * x2), np.sin(2 * x1 - x2)]), dtype)
        t0 = 0.09          # inside the Ricker pulse
        sol.set_state([u0], [v0], t0)
        sol.advance(nsteps, dt)
        ug, vg = sol.state_numpy()
        u, v, t = [u0.copy()], [v0.copy()], t0
        for _ in range(nsteps):
            u, v = T.rk4_step(P, u, v, t, dt)
            t += dt
        eu, ev = rel(ug[0], u[0]), rel(vg[0], v[0])
        say('  rel L2 u %.3e v %.3e' % (eu, ev))
        tol = {'f64': 1e-11, 'f32': 1e-5}[dtype]
        assert eu < tol and ev < tol
    finally:
        sol.close()


def test_tile_rows_do_not_change_results():
    """The launch shape (interior tile height, frame groups per frame
    workgroup) does not change a run's bits (the benchmark picks the fastest)."""
    n, nsteps = 97, 20
    spec = W.spec_c2(n=n, nrec=8)
    say('launch shapes', n)
    out = []
    for rows, loop in ((10, 1), (7, 3), (20, 4)):
        sol = solver(spec, 'f64', tile_rows=rows)
        sol.set_frame_loop(loop)
        try:
            dt = T.dt_cfl(build(spec), 0.5) if not out else out[0][3]
            sol.set_state(None, None, 0.0)
            sol.advance(nsteps, dt)
            u, v = sol.state_numpy()
            out.append((u[0], v[0], sol.receivers(), dt))
        finally:
            sol.close()
    for u, v, r, _ in out[1:]:
        assert np.array_equal(u, out[0][0]) and np.array_equal(v, out[0][1]) and np.array_equal(r, out[0][2])


def test_small_grid_default_shape():
    """On a small grid the default launch shape is tiles of order + 1 rows and
    one frame group per frame workgroup; a run in it has the bits of a run in
    the large-grid default shape (10 rows, 2 groups)."""
    n, nsteps = 129, 20
    spec = W.spec_c2(n=n, nrec=8)
    say('small-grid default shape', n)
    out = []
    for rows, loop in ((0, 0), (10, 2)):
        sol = solver(spec, 'f64', tile_rows=rows)
        if loop:
            sol.set_frame_loop(loop)
        try:
            plan = S.sbpe_plan_info(sol.ctx)
            interior = n - 2 * plan['frame_width']
            if not loop:
                # 60 written columns per tile, 5 rows per tile at order 4
                assert plan['interior_workgroups'] == -(-interior // 60) * -(-interior // 5)
            dt = T.dt_cfl(build(spec), 0.5) if not out else out[0][3]
            sol.set_state(None, None, 0.0)
            sol.advance(nsteps, dt)
            u, v = sol.state_numpy()
            out.append((u[0], v[0], sol.receivers(), dt))
        finally:
            sol.close()
    u, v, r, _ = out[1]
    assert np.array_equal(u, out[0][0]) and np.array_equal(v, out[0][1]) and np.array_equal(r, out[0][2])


@pytest.fixture(scope='module')
def c3_full():
    """The 2x2 x 2049^2 workload and its oracle (about a minute of CPU time)."""
    spec = W.spec_c3(n=2049)
    return spec, build(spec)


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_full_size_c3_apply_and_energy(dtype, c3_full):
    """The 2x2 x 2049^2 workload at its full size, element by element against
    the oracle: one right-hand side inside the Ricker pulse (interfaces,
    displacement and traction faces, the point source), in the two-stream
    launch path the benchmark times, and the FP64 energy of a state."""
    spec, P = c3_full
    n = 2049
    say('full size C3 apply and energy', dtype)
    sol = solver(spec, dtype)
    try:
        assert not S.sbpe_plan_info(sol.ctx)['fused_sweep']
        x1, x2 = W.reference_grid(n, n)
        rng = np.random.default_rng(9)
        us, vs = [], []
        for _ in spec['blocks']:
            a, b, c, d = rng.uniform(1, 6, 4)
            us.append(rounded(np.stack([np.sin(a * x1 + b * x2 + c), np.cos(d * x1 - a * x2)]) +
                              1e-3 * rng.normal(size=(2, n, n)), dtype))
            vs.append(rounded(np.stack([np.cos(b * x1 - c * x2), np.sin(c * x1 + d * x2)]), dtype))
        t = 0.1
        got = [x.double().cpu().numpy() for x in sol.apply(us, t=t)]
        ref = P.rhs(us, t)
        err = rel(np.concatenate([g.ravel() for g in got]), np.concatenate([r.ravel() for r in ref]))
        eb = band_max_rel(got, ref, 4)
        say('  apply rel L2 %.3e  band max %.3e' % (err, eb))
        assert err < TOL[dtype] and eb < TOL[dtype]
        sol.set_state(us, vs, 0.0)
        e_lib, e_or = sol.energy(), P.energy(us, vs)
        say('  energy lib %.12e oracle %.12e rel %.2e' % (e_lib, e_or, abs(e_lib / e_or - 1)))
        assert abs(e_lib / e_or - 1) < TOL[dtype]
    finally:
        sol.close()


@pytest.mark.parametrize("dtype", ['f64', 'f32'])
def test_full_size_c3_self_adjoint(dtype):
    """The 2x2 x 2049^2 workload at its full size, through the launch path the
    benchmark times there (tiles and frame on two streams, interfaces through
    the frame operator's partner columns), checked by properties that hold at
    any size: H rho~ L is symmetric (w . H L u = u . H L w, the self-adjointness
    of Sec. 5-6) and negative semidefinite (u . H L u <= 0)."""
    from oracle import sbp
    n = 2049
    say('full size C3 self-adjointness', dtype)
    spec = W.spec_c3(n=n)
    sol = solver(spec, dtype)
    try:
        assert not S.sbpe_plan_info(sol.ctx)['fused_sweep']
        x1, x2 = W.reference_grid(n, n)
        rng = np.random.default_rng(3)

        def field():
            out = []
            for _ in spec['blocks']:
                a, b, c, d = rng.uniform(1, 6, 4)
                f = np.stack([np.sin(a * x1 + b * x2 + c), np.cos(d * x1 - a * x2)])
                out.append(rounded(f + 1e-2 * rng.normal(size=f.shape), dtype))
            return out
        us, ws = field(), field()
        lu = [x.double().cpu().numpy() for x in sol.apply(us, homogeneous=True)]
        lw = [x.double().cpu().numpy() for x in sol.apply(ws, homogeneous=True)]
        s_wu = s_uw = s_uu = scale = 0.0
        for k, blk in enumerate(spec['blocks']):
            _, J, _ = S.sbpe_get_block_fields(sol.ctx, k)
            h = 1.0 / (n - 1)
            Hr = np.outer(sbp.norm(n, h, 4), sbp.norm(n, h, 4)) * J * blk['rho']   # H rho~
            s_wu += float(np.sum(Hr * (ws[k] * lu[k]).sum(0)))
            s_uw += float(np.sum(Hr * (us[k] * lw[k]).sum(0)))
            s_uu += float(np.sum(Hr * (us[k] * lu[k]).sum(0)))
            scale += float(np.sum(Hr * np.abs(ws[k] * lu[k]).sum(0)))
        asym = abs(s_wu - s_uw) / scale
        say('  w.HLu %.6e  u.HLw %.6e  relative asymmetry %.2e  u.HLu %.4e' % (s_wu, s_uw, asym, s_uu))
        assert asym < {'f64': 1e-12, 'f32': 1e-5}[dtype]
        assert s_uu < 0
    finally:
        sol.close()
