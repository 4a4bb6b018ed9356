"""CPU checks of the HIP library's host side (no GPU needed).

* libsbpe.so loads and exports every function declared in include/sbpe.h;
* the library's own 1-D operators (closure table derived in C++, interior
  stencil written out in the kernels) agree with the oracle's D1 and D2^FC;
* setup in a host-only context: transformed stiffness c = F J C F, J, Jhat
  and the Christoffel time step agree with the oracle;
* argument validation and error codes.
"""
import os
import re

import numpy as np
import pytest

from oracle import elastic as E, material as M, sbp, timestep as T
from oracle.geometry import metrics
from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, 'include', 'sbpe.h')).read()
    names = set(re.findall(r'\b(sbpe_[a-z0-9_]+)\s*\(', hdr))
    assert len(names) >= 25
    hdr3 = open(os.path.join(ROOT, 'include', 'sbpe3.h')).read()
    names3 = set(re.findall(r'\b(sbpe3_[a-z0-9_]+)\s*\(', hdr3))
    assert len(names3) >= 12
    names |= names3
    L = S.lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("order", [2, 4, 6])
@pytest.mark.parametrize("n", [19, 20, 41])
def test_library_line_operators_match_oracle(order, n):
    rng = np.random.default_rng(n + order)
    b = 1.0 + rng.uniform(0, 1, n)
    u = rng.normal(size=n)
    h = 1.0 / (n - 1)
    ref = sbp.d2fc(b, h, order) @ u
    got = S.sbpe_host_d2fc_line(order, b, u)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
    ref1 = sbp.d1(n, h, order) @ u
    assert np.allclose(S.sbpe_host_d1_line(order, u), ref1, rtol=1e-12, atol=1e-12 * np.abs(ref1).max())


def _host_ctx(order=4, dtype=S.F64):
    return S.sbpe_create(-1, None, dtype, order, 1.0)


@pytest.mark.parametrize("order", [2, 4, 6])
def test_setup_matches_oracle(order):
    n1, n2 = (19, 16) if order < 6 else (23, 20)
    X1, X2 = W.grid(W.GaussianTopography(0.15, 0.2), n1, n2)
    rho, C10 = W.paper_random_material((n2, n1), 4)
    ctx = _host_ctx(order)
    try:
        b = S.sbpe_add_block(ctx, X1, X2, rho, C10)
        S.sbpe_finalize(ctx)
        c10, J, jhat = S.sbpe_get_block_fields(ctx, b)
        B = E.Block(X1, X2, rho, M.full_from_c10(C10), order=order)
        assert np.allclose(J, B.J, rtol=1e-13)
        assert np.allclose(c10, M.c10_from_full(B.c), rtol=1e-12, atol=1e-12 * np.abs(c10).max())
        g = metrics(X1, X2, order)
        for f in range(4):
            assert np.allclose(jhat[f], g['faces'][f]['Jhat'], rtol=1e-13)
        dt = S.sbpe_dt_cfl(ctx, 0.5)
        assert abs(dt / T.dt_cfl(E.Problem([B]), 0.5) - 1) < 1e-6
    finally:
        S.sbpe_destroy(ctx)


def test_voigt_conversion_matches_oracle():
    rng = np.random.default_rng(0)
    V = rng.uniform(0, 1, (6, 3, 4))
    got = S.sbpe_voigt_to_c10(V)
    ref = M.c10_from_full(M.full_from_voigt(V))
    assert np.array_equal(got, ref)
    assert np.array_equal(got, W.voigt_to_c10(V))


def test_error_codes():
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    rho, C10 = W.paper_random_material((n, n), 0)
    ctx = _host_ctx()
    try:
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_add_block(ctx, X1[:, ::-1], X2, rho, C10)
            S.sbpe_finalize(ctx)
        assert e.value.code == S.ENONPOS_J
    finally:
        S.sbpe_destroy(ctx)
    ctx = _host_ctx()
    try:
        bad = C10.copy()
        bad[0] = -5.0
        S.sbpe_add_block(ctx, X1, X2, rho, bad)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_finalize(ctx)
        assert e.value.code == S.ENOT_PSD
    finally:
        S.sbpe_destroy(ctx)
    ctx = _host_ctx()
    try:
        S.sbpe_add_block(ctx, X1, X2, rho, C10)
        X1b, X2b = W.grid(W.Identity(), n + 2, n)
        rb, Cb = W.paper_random_material((n, n + 2), 1)
        S.sbpe_add_block(ctx, X1b, X2b, rb, Cb)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_connect(ctx, 0, S.FACE_X2HI, 1, S.FACE_X2LO)
        assert e.value.code == S.EIFACE
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_bc(ctx, 0, 7, S.BC_TRACTION)
        assert e.value.code == S.EINVAL
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_bc(ctx, 0, 0, S.BC_ROBIN, None)
        assert e.value.code == S.EINVAL
        S.sbpe_finalize(ctx)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_advance(ctx, 1, 1e-3)
        assert e.value.code == S.ESTATE
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_add_block(ctx, X1, X2, rho, C10)
        assert e.value.code == S.ESTATE
    finally:
        S.sbpe_destroy(ctx)
    with pytest.raises(S.SbpeError):
        S.sbpe_create(-1, None, 7, 4, 1.0)
    with pytest.raises(S.SbpeError):
        S.sbpe_create(-1, None, S.F64, 8, 1.0)
    with pytest.raises(S.SbpeError):
        S.sbpe_create(-1, None, S.F64, 4, 0.5)
    # order 6: no wide-stencil operator; blocks of at least 19 points per direction
    ctx = _host_ctx(6)
    try:
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_operator(ctx, S.OP_WIDE)
        assert e.value.code == S.EINVAL
        Xs1, Xs2 = W.grid(W.Identity(), 18, 25)
        rs, Cs = W.paper_random_material((25, 18), 2)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_add_block(ctx, Xs1, Xs2, rs, Cs)
        assert e.value.code == S.EINVAL
    finally:
        S.sbpe_destroy(ctx)


def test_set_operator_states():
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    rho, C10 = W.paper_random_material((n, n), 0)
    ctx = _host_ctx()
    try:
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_operator(ctx, 5)
        assert e.value.code == S.EINVAL
        S.sbpe_set_operator(ctx, S.OP_WIDE)
        S.sbpe_set_operator(ctx, S.OP_NARROW)
        S.sbpe_set_operator(ctx, S.OP_WIDE)
        S.sbpe_add_block(ctx, X1, X2, rho, C10)
        S.sbpe_finalize(ctx)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_operator(ctx, S.OP_NARROW)
        assert e.value.code == S.ESTATE
    finally:
        S.sbpe_destroy(ctx)


def test_block_size_limits():
    """Below the operator's minimum and above 2^28 points a block is refused
    before its arrays are read (the raw call gets one-element arrays)."""
    import ctypes
    lib = S.lib()
    one = np.ones(1)
    ptr = one.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    bid = ctypes.c_int(-1)
    for order, sizes in ((4, [(12, 40), (40, 12), (16385, 16385), (1 << 20, 257)]), (2, [(5, 30)])):
        ctx = _host_ctx(order)
        try:
            for n1, n2 in sizes:
                st = lib.sbpe_add_block(ctx, n1, n2, ptr, ptr, ptr, ptr, ctypes.byref(bid))
                assert st == S.EINVAL, (order, n1, n2, st)
        finally:
            S.sbpe_destroy(ctx)


def test_tile_rows_states():
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    rho, C10 = W.paper_random_material((n, n), 0)
    ctx = _host_ctx()
    try:
        for bad in (-1, 257):
            with pytest.raises(S.SbpeError) as e:
                S.sbpe_set_tile_rows(ctx, bad)
            assert e.value.code == S.EINVAL
        S.sbpe_set_tile_rows(ctx, 20)
        S.sbpe_set_tile_rows(ctx, 0)
        for bad in (0, 65):
            with pytest.raises(S.SbpeError) as e:
                S.sbpe_set_frame_loop(ctx, bad)
            assert e.value.code == S.EINVAL
        S.sbpe_set_frame_loop(ctx, 4)
        S.sbpe_add_block(ctx, X1, X2, rho, C10)
        S.sbpe_finalize(ctx)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_tile_rows(ctx, 12)
        assert e.value.code == S.ESTATE
    finally:
        S.sbpe_destroy(ctx)


def test_dissipation_states():
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    rho, C10 = W.paper_random_material((n, n), 0)
    ctx = _host_ctx()
    try:
        S.sbpe_add_block(ctx, X1, X2, rho, C10)
        S.sbpe_set_bc(ctx, 0, 0, S.BC_DISPLACEMENT)
        V = np.zeros((2, 2, n))
        V[0, 0] = V[1, 1] = 1.0
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_bc_dissipation(ctx, 0, 0, V)
        assert e.value.code == S.ESTATE
        bad = V.copy()
        bad[0, 1] = 3.0      # not symmetric
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_set_bc_dissipation(ctx, 0, 1, bad)
        assert e.value.code == S.EINVAL
        S.sbpe_set_bc_dissipation(ctx, 0, 1, V)
        # the face may not change kind afterwards
        S.sbpe_set_bc(ctx, 0, 1, S.BC_DISPLACEMENT)
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_finalize(ctx)
        assert e.value.code == S.EINVAL
    finally:
        S.sbpe_destroy(ctx)


def _finalize_status(M4):
    """sbpe_finalize on a small host-only block whose stiffness, as the 4x4
    matrix over the pairs (11, 12, 21, 22), is M4 at every point."""
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    iu = np.triu_indices(4)
    C10 = np.asarray(M4)[iu][:, None, None] * np.ones((1, n, n))
    ctx = _host_ctx()
    try:
        S.sbpe_add_block(ctx, X1, X2, np.ones((n, n)), C10)
        S.sbpe_finalize(ctx)
        return 0
    except S.SbpeError as e:
        return e.code
    finally:
        S.sbpe_destroy(ctx)


def test_stiffness_psd_check_against_eigenvalues():
    """The finalize check accepts exactly the semidefinite stiffnesses (up to a
    relative 1e-10), judged here by numpy's eigenvalues: full-rank and
    minor-symmetric (rank 3) media, and matrices with one eigenvalue moved to
    -1e-13 (accepted) or -1e-6 (rejected) of the scale."""
    rng = np.random.default_rng(11)
    for trial in range(20):
        Q, _ = np.linalg.qr(rng.normal(size=(4, 4)))
        lam = rng.uniform(0.5, 3.0, 4)
        if trial % 4 == 1:
            lam[rng.integers(4)] = 0.0                  # semidefinite
        if trial % 4 == 2:
            lam[rng.integers(4)] = -1e-13 * lam.max()   # within the tolerance
        if trial % 4 == 3:
            lam[rng.integers(4)] = -1e-6 * lam.max()    # clearly indefinite
        A = (Q * lam) @ Q.T
        A = 0.5 * (A + A.T)
        want_ok = np.linalg.eigvalsh(A).min() >= -1e-10 * max(1.0, np.abs(A).max())
        assert (_finalize_status(A) == 0) == want_ok, (trial, np.linalg.eigvalsh(A))
    # minor-symmetric media from Voigt (rank 3) are accepted
    V = np.array(W.VOIGT_C1)
    A = M.full_from_c10(W.voigt_to_c10(V)).reshape(4, 4)
    assert _finalize_status(A) == 0


def test_allocator_states():
    """Callbacks come in pairs and are set before the context allocates;
    host-only contexts never call them."""
    n = 15
    X1, X2 = W.grid(W.Identity(), n, n)
    rho, C10 = W.paper_random_material((n, n), 0)
    calls = []
    ctx = _host_ctx()
    try:
        import ctypes
        lib = S.lib()
        a = S.ALLOC_FN(lambda nb, u: calls.append(nb) or None)
        r = S.RELEASE_FN(lambda p, u: calls.append(p))
        assert lib.sbpe_set_allocator(ctx, a, S.RELEASE_FN(), None) == S.EINVAL
        assert lib.sbpe_set_allocator(ctx, S.ALLOC_FN(), r, None) == S.EINVAL
        S.sbpe_set_allocator(ctx, lambda nb: calls.append(nb) or 0, lambda p: calls.append(p))
        assert lib.sbpe_set_allocator(ctx, S.ALLOC_FN(), S.RELEASE_FN(), None) == S.OK
        S.sbpe_add_block(ctx, X1, X2, rho, C10)
        S.sbpe_finalize(ctx)
        assert lib.sbpe_set_allocator(ctx, a, r, None) == S.ESTATE
    finally:
        S.sbpe_destroy(ctx)
    assert calls == []


def test_homogeneous_spec_keeps_the_operator_and_drops_the_data():
    # the adjoint's data-free context: same blocks, material, boundary kinds,
    # Robin matrices, interfaces and operator; no boundary data, forcing,
    # sources, receivers or interface jump data
    from paper_2003_12811_amd import adjoint as ADJ
    spec = W.spec_mms(n=17)
    spec['sources'] = [(0, 0.5, 0.5, 0.0, 1.0, 1.0, 10.0, 0.1)]
    spec['receivers'] = [(0, np.array([0.3]), np.array([0.7]))]
    spec['interface_data'] = [(0, None, None, 0, None)]
    spec['operator'] = 'wide'
    h = ADJ.homogeneous_spec(spec)
    assert 'sources' not in h and 'receivers' not in h and 'interface_data' not in h
    assert h['operator'] == 'wide' and h['order'] == spec['order'] and h['interfaces'] == spec['interfaces']
    for b, hb in zip(spec['blocks'], h['blocks']):
        assert hb.get('forcing') is None and b.get('forcing') is not None
        assert hb['X1'] is b['X1'] and hb['rho'] is b['rho'] and hb['C10'] is b['C10']
        for (kind, g, tfn, tp, U), (hk, hg, htf, htp, hU) in zip(b['bc'], hb['bc']):
            assert hk == kind and hU is U and hg is None and htf is None and htp is None
    # the input is left as it was
    assert spec['blocks'][0]['bc'][1][1] is not None and 'sources' in spec
