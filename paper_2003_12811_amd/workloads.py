"""Seeded synthetic inputs: grids, material fields, manufactured solutions.

This module holds input generation only (mappings, random material fields,
analytic manufactured-solution data).  It contains none of the discretisation:
no SBP operators, no SATs, no time stepping.  Tests, the smoke check and the
benchmark feed the same arrays to the HIP library and to the CPU oracle.

Recipes (all in reference coordinates x in [0, 1]^2, physical X = X(x)):

* ``identity``             X = x.
* ``gaussian_topography``  X1 = x1, X2 = x2 + A exp(-((x1 - 0.5)/w)^2) (1 - x2),
                           A = 0.1, w = 0.1: a Gaussian bump on the face x2 = 0.
* ``sine_warp``            X = x + eps sin(pi x1) sin(pi x2) (1, 1), eps = 0.05, one
                           smooth global map that is split into conforming blocks.
* ``smooth_random_material``  rho and the six Voigt entries (c11, c12, c16, c22,
  c26, c66) are mean * (1 + 0.3/8 sum_{m<8} a_m cos(2 pi (kx_m X1 + ky_m X2) + phi_m))
  with integer kx, ky in [-4, 4], a ~ U(-1, 1), phi ~ U(0, 2 pi) drawn from
  numpy.random.default_rng(seed) field by field in the order rho, c11, c12,
  c16, c22, c26, c66; the 3x3 Voigt matrix is then clipped to eigenvalues
  >= 0.2 and rho to >= 0.2 at every point.
* ``paper_random_material``  rho = 1 + U(0, 1) and every independent
  component of a major-symmetric (not minor-symmetric) tensor drawn from
  U(0, 1), plus 4 on the C_IJIJ entries: the recipe of the paper's
  self-adjointness experiment (Sec. 7.2).
* ``mms_c1``  u_L = sin(2 pi X1 + L) cos(2 pi X2) cos(2 sqrt(2) pi t), L = 1, 2,
  with constant stiffness; forcing rho u_tt - C_IJKL d_I d_K u_L and traction
  data n_I C_IJKL d_K u_L are returned as space parts multiplying cos(omega t).
"""
import numpy as np

VOIGT_C1 = (4.0, 1.0, 0.5, 3.0, 0.3, 1.5)        # c11, c12, c16, c22, c26, c66


# ------------------------------------------------------------------ mappings
class Mapping:
    """X(x) and its analytic Jacobian dX_I/dx_i."""

    def __call__(self, x1, x2):
        raise NotImplementedError

    def jac(self, x1, x2):
        raise NotImplementedError


class Identity(Mapping):
    def __call__(self, x1, x2):
        return x1 + 0.0 * x2, x2 + 0.0 * x1

    def jac(self, x1, x2):
        o, z = np.ones_like(x1 + x2), np.zeros_like(x1 + x2)
        return np.array([[o, z], [z, o]])        # [i][I]


class GaussianTopography(Mapping):
    def __init__(self, amp=0.1, width=0.1):
        self.A, self.w = amp, width

    def __call__(self, x1, x2):
        g = self.A * np.exp(-((x1 - 0.5) / self.w) ** 2)
        return x1 + 0.0 * x2, x2 + g * (1.0 - x2)

    def jac(self, x1, x2):
        g = self.A * np.exp(-((x1 - 0.5) / self.w) ** 2)
        dg = g * (-2.0 * (x1 - 0.5) / self.w ** 2)
        o, z = np.ones_like(x1 + x2), np.zeros_like(x1 + x2)
        return np.array([[o, dg * (1.0 - x2)], [z, 1.0 - g + 0.0 * x1]])


class SineWarp(Mapping):
    def __init__(self, eps=0.05):
        self.e = eps

    def __call__(self, x1, x2):
        s = self.e * np.sin(np.pi * x1) * np.sin(np.pi * x2)
        return x1 + s, x2 + s

    def jac(self, x1, x2):
        d1 = self.e * np.pi * np.cos(np.pi * x1) * np.sin(np.pi * x2)
        d2 = self.e * np.pi * np.sin(np.pi * x1) * np.cos(np.pi * x2)
        return np.array([[1.0 + d1, d1], [d2, 1.0 + d2]])


MAPPINGS = {'identity': Identity, 'gaussian_topography': GaussianTopography,
            'sine_warp': SineWarp}


def reference_grid(n1, n2, x1lim=(0.0, 1.0), x2lim=(0.0, 1.0)):
    x1 = np.linspace(x1lim[0], x1lim[1], n1)
    x2 = np.linspace(x2lim[0], x2lim[1], n2)
    return np.meshgrid(x1, x2)            # arrays (n2, n1), x1 fastest


def grid(mapping, n1, n2, x1lim=(0.0, 1.0), x2lim=(0.0, 1.0)):
    """Physical grid coordinates (X1, X2), arrays of shape (n2, n1)."""
    x1, x2 = reference_grid(n1, n2, x1lim, x2lim)
    X1, X2 = mapping(x1, x2)
    return np.ascontiguousarray(X1), np.ascontiguousarray(X2)


def outward_normal(mapping, face, n1, n2, x1lim=(0.0, 1.0), x2lim=(0.0, 1.0)):
    """Exact unit outward physical normal on a face of a (sub)block, shape (2, nf)."""
    x1, x2 = reference_grid(n1, n2, x1lim, x2lim)
    sel = [(slice(None), 0), (slice(None), -1), (0, slice(None)), (-1, slice(None))][face]
    A = mapping.jac(x1[sel], x2[sel])                   # A[i][I] = dX_I/dx_i
    a = 0 if face < 2 else 1
    t = 1 - a
    tang = np.array([A[t][0], A[t][1]])
    n = np.array([tang[1], -tang[0]])                  # rotate the tangent by -90 deg
    # orient outward: compare with the covariant normal direction a_a
    nor = np.array([A[a][0], A[a][1]])
    sgn = -1.0 if face in (0, 2) else 1.0
    s = np.sign(np.sum(n * nor, axis=0)) * sgn
    n = n * s
    return n / np.sqrt(n[0] ** 2 + n[1] ** 2)


# --------------------------------------------------------- material fields
def voigt_to_c10(V):
    """Voigt (6, ...) -> the 10 major-symmetric components in the library order
    C1111, C1112, C1121, C1122, C1212, C1221, C1222, C2121, C2122, C2222."""
    c11, c12, c16, c22, c26, c66 = V
    return np.stack([c11, c16, c16, c12, c66, c66, c26, c66, c26, c22])


def smooth_random_material(X1, X2, seed, rho_mean=1.0, voigt_mean=VOIGT_C1,
                           nmodes=8, kmax=4, rel_amp=0.3, min_eig=0.2, device=None):
    """device (a torch device, e.g. 'cuda') evaluates the Fourier sums with
    torch there: same draws and formula, different rounding of cos."""
    rng = np.random.default_rng(seed)
    fields = []
    if device is not None:
        import torch
        tX1 = torch.as_tensor(np.ascontiguousarray(X1), device=device)
        tX2 = torch.as_tensor(np.ascontiguousarray(X2), device=device)
        tt = torch.empty_like(tX1)
    for mean in (rho_mean,) + tuple(voigt_mean):
        kx = rng.integers(-kmax, kmax + 1, nmodes)
        ky = rng.integers(-kmax, kmax + 1, nmodes)
        ph = rng.uniform(0.0, 2.0 * np.pi, nmodes)
        a = rng.uniform(-1.0, 1.0, nmodes)
        if device is not None:
            ts = torch.zeros_like(tX1)
            for m in range(nmodes):
                torch.mul(tX1, 2.0 * np.pi * float(kx[m]), out=tt)
                tt.add_(tX2, alpha=2.0 * np.pi * float(ky[m])).add_(float(ph[m])).cos_()
                ts.add_(tt, alpha=float(a[m]))
            s = ts.cpu().numpy()
        else:
            s = np.zeros_like(X1)
            for m in range(nmodes):
                s += a[m] * np.cos(2.0 * np.pi * (kx[m] * X1 + ky[m] * X2) + ph[m])
        fields.append(mean * (1.0 + rel_amp * s / nmodes))
    rho = np.maximum(fields[0], min_eig)
    V = np.stack(fields[1:])
    # eigen-clip the Voigt matrix where M - min_eig I is not positive definite
    # (leading principal minors), leaving every other point unchanged
    c11, c12, c16, c22, c26, c66 = V - min_eig * np.array([1, 0, 0, 1, 0, 1.0]).reshape(6, *([1] * X1.ndim))
    d1 = c11
    d2 = c11 * c22 - c12 * c12
    d3 = c11 * (c22 * c66 - c26 * c26) - c12 * (c12 * c66 - c26 * c16) + c16 * (c12 * c26 - c22 * c16)
    bad = ~((d1 > 0) & (d2 > 0) & (d3 > 0))
    if bad.any():
        Vb = V[:, bad]
        b11, b12, b16, b22, b26, b66 = Vb
        M = np.stack([np.stack([b11, b12, b16], -1), np.stack([b12, b22, b26], -1),
                      np.stack([b16, b26, b66], -1)], -2)
        lam, Q = np.linalg.eigh(M)
        lam = np.maximum(lam, min_eig)
        M = np.einsum('...ik,...k,...jk->...ij', Q, lam, Q)
        V[:, bad] = np.stack([M[..., 0, 0], M[..., 0, 1], M[..., 0, 2], M[..., 1, 1], M[..., 1, 2], M[..., 2, 2]])
    return np.ascontiguousarray(rho), np.ascontiguousarray(V)


def paper_random_material(shape, seed):
    """rho (shape) and C10 (10, *shape), Cosserat (major symmetry only)."""
    rng = np.random.default_rng(seed)
    rho = 1.0 + rng.uniform(0.0, 1.0, shape)
    C10 = rng.uniform(0.0, 1.0, (10,) + tuple(shape))
    for m in (0, 4, 7, 9):                  # C1111, C1212, C2121, C2222 (the C_IJIJ entries)
        C10[m] += 4.0
    return rho, C10


def c10_to_full(C10):
    order = [(0, 0), (0, 1), (0, 2), (0, 3), (1, 1), (1, 2), (1, 3), (2, 2), (2, 3), (3, 3)]
    pairs = [(0, 0), (0, 1), (1, 0), (1, 1)]
    C = np.zeros((2, 2, 2, 2) + C10.shape[1:])
    for m, (p, q) in enumerate(order):
        C[pairs[p] + pairs[q]] = C10[m]
        C[pairs[q] + pairs[p]] = C10[m]
    return C


# ------------------------------------------------- manufactured solution
OMEGA_C1 = 2.0 * np.sqrt(2.0) * np.pi


def mms_c1(X1, X2, C10, rho=1.0):
    """Space parts of u, forcing and tractions for the C1 manufactured solution.

    Constant stiffness C10 (10,), constant rho.  Returns dict with
    ``u`` (2, n2, n1), ``f`` (2, n2, n1) and ``grad`` (2 [L], 2 [K], n2, n1) so
    that u(t) = u cos(omega t), f(t) = f cos(omega t); the traction data on a
    face with unit normal n is n_I C_IJKL grad[L, K] (see ``traction_data``).
    """
    C = c10_to_full(np.asarray(C10, dtype=float))
    tp = 2.0 * np.pi
    u = np.stack([np.sin(tp * X1 + L) * np.cos(tp * X2) for L in (1, 2)])
    grad = np.stack([np.stack([tp * np.cos(tp * X1 + L) * np.cos(tp * X2),
                               -tp * np.sin(tp * X1 + L) * np.sin(tp * X2)]) for L in (1, 2)])
    hess = np.empty((2, 2, 2) + X1.shape)        # [L, I, K]
    for Li, L in enumerate((1, 2)):
        s = np.sin(tp * X1 + L) * np.cos(tp * X2)
        m = np.cos(tp * X1 + L) * np.sin(tp * X2)
        hess[Li, 0, 0] = -tp ** 2 * s
        hess[Li, 1, 1] = -tp ** 2 * s
        hess[Li, 0, 1] = -tp ** 2 * m
        hess[Li, 1, 0] = -tp ** 2 * m
    div = np.einsum('IJKL,LIK...->J...', C, hess)
    f = -rho * OMEGA_C1 ** 2 * u - div
    return dict(u=u, f=f, grad=grad, C=C, omega=OMEGA_C1)


def mms_wave(X1, X2, C10, rho=1.0, amp=1.0, phase=0.0, omega=OMEGA_C1):
    """The C1 manufactured solution with an amplitude and a phase,
    u_L = amp sin(2 pi X1 + L + phase) cos(2 pi X2) cos(omega t), for constant
    C10 (10,) and rho; same fields as ``mms_c1``."""
    C = c10_to_full(np.asarray(C10, dtype=float))
    tp = 2.0 * np.pi
    ph = [L + phase for L in (1, 2)]
    u = np.stack([amp * np.sin(tp * X1 + q) * np.cos(tp * X2) for q in ph])
    grad = np.stack([np.stack([amp * tp * np.cos(tp * X1 + q) * np.cos(tp * X2),
                               -amp * tp * np.sin(tp * X1 + q) * np.sin(tp * X2)]) for q in ph])
    hess = np.empty((2, 2, 2) + X1.shape)        # [L, I, K]
    for Li, q in enumerate(ph):
        sv = amp * np.sin(tp * X1 + q) * np.cos(tp * X2)
        m = amp * np.cos(tp * X1 + q) * np.sin(tp * X2)
        hess[Li, 0, 0] = -tp ** 2 * sv
        hess[Li, 1, 1] = -tp ** 2 * sv
        hess[Li, 0, 1] = -tp ** 2 * m
        hess[Li, 1, 0] = -tp ** 2 * m
    div = np.einsum('IJKL,LIK...->J...', C, hess)
    f = -rho * omega ** 2 * u - div
    return dict(u=u, f=f, grad=grad, C=C, omega=omega)


def traction_data(mms, face_idx, normal):
    """n_I C_IJKL d_K u_L at the face points (flat indices), shape (2, nf)."""
    g = mms['grad'].reshape(2, 2, -1)[..., face_idx]
    return np.einsum('If,IJKL,LKf->Jf', normal, mms['C'], g)


# ------------------------------------------------------------ problem specs
# A spec is a plain dict consumed by both the library front end
# (paper_2003_12811_amd.solver) and the tests' oracle builder:
#   order, blocks: [dict(X1, X2, rho, C10, bc=[(kind, g, time_fn, time_params, U)] * 4,
#                        forcing=None | (F, time_fn, time_params))],
#   interfaces: [(block_a, face_a, block_b, face_b, reversed)],
#   sources: [(block, x1, x2, f1, f2, amp, peak_hz, t0)], receivers: [(block, x1[], x2[])]
# Boundary kinds / time functions use the numbering of include/sbpe.h.
TRACTION, ROBIN, DISPLACEMENT = 0, 1, 2
T_ZERO, T_ONE, T_COS, T_RICKER = 0, 1, 2, 3


def _free_faces():
    return [(TRACTION, None, T_ZERO, None, None) for _ in range(4)]


def face_flat_index(face, n1, n2):
    if face < 2:
        return np.arange(n2) * n1 + (0 if face == 0 else n1 - 1)
    return (0 if face == 2 else n2 - 1) * n1 + np.arange(n1)


def spec_c1(n=65, order=4):
    """Plain method: 65^2 Cartesian block, constant anisotropic C, MMS, traction SATs."""
    X1, X2 = grid(Identity(), n, n)
    C10c = voigt_to_c10(np.array(VOIGT_C1))
    mm = mms_c1(X1, X2, C10c)
    C10 = C10c[:, None, None] * np.ones((1, n, n))
    bc = []
    for f in range(4):
        g = traction_data(mm, face_flat_index(f, n, n), outward_normal(Identity(), f, n, n))
        bc.append((TRACTION, g, T_COS, (mm['omega'], 0.0), None))
    blk = dict(X1=X1, X2=X2, rho=np.ones((n, n)), C10=C10, bc=bc,
               forcing=(mm['f'], T_COS, (mm['omega'], 0.0)))
    return dict(order=order, blocks=[blk], interfaces=[], sources=[], receivers=[],
                mms=mm, T=0.5, cfl=0.5)


def spec_mms(n=65, order=4, kinds=(TRACTION, DISPLACEMENT, TRACTION, DISPLACEMENT), mapping=None,
             data_sign=1.0, drop_displacement_data=False):
    """The C1 manufactured solution on a block with a chosen boundary kind per
    face: traction faces carry the exact traction n_I C_IJKL d_K u_L, and
    displacement faces the exact boundary displacement g = u (Sec. 5.2,
    eq. dirichlet_ansatz), both times cos(omega t).  mapping (default the
    identity) may curve the block; the material stays constant in physical
    space.  data_sign multiplies the displacement data and
    drop_displacement_data leaves it out: both give a problem whose discrete
    solution does not converge to the manufactured one."""
    m = Identity() if mapping is None else mapping
    X1, X2 = grid(m, n, n)
    C10c = voigt_to_c10(np.array(VOIGT_C1))
    mm = mms_c1(X1, X2, C10c)
    C10 = C10c[:, None, None] * np.ones((1, n, n))
    bc = []
    for f, kind in enumerate(kinds):
        idx = face_flat_index(f, n, n)
        if kind == DISPLACEMENT:
            if drop_displacement_data:
                bc.append((DISPLACEMENT, None, T_ZERO, None, None))
                continue
            g = data_sign * mm['u'].reshape(2, -1)[:, idx]
        else:
            g = traction_data(mm, idx, outward_normal(m, f, n, n))
        bc.append((kind, np.ascontiguousarray(g), T_COS, (mm['omega'], 0.0), None))
    blk = dict(X1=X1, X2=X2, rho=np.ones((n, n)), C10=C10, bc=bc,
               forcing=(mm['f'], T_COS, (mm['omega'], 0.0)))
    return dict(order=order, blocks=[blk], interfaces=[], sources=[], receivers=[],
                mms=mm, T=0.5, cfl=0.5)


def spec_fault(n=33, order=4, jump_data=True):
    """Two Cartesian blocks [0, 1/2] x [0, 1] and [1/2, 1] x [0, 1] of n^2
    points each, joined along x1 = 1/2, with different constant materials and a
    manufactured solution that jumps across the interface; the jumps in
    displacement and traction enter as interface data (Sec. 6,
    eq. interface_phys), the outer faces carry the exact tractions.
    jump_data=False drops the interface data (the solution then does not
    satisfy the discrete problem)."""
    voigt = np.array(VOIGT_C1)
    parts = [dict(lim=(0.0, 0.5), scale=1.0, rho=1.0, amp=1.0, phase=0.0),
             dict(lim=(0.5, 1.0), scale=2.5, rho=1.5, amp=0.6, phase=0.9)]
    blocks, mms = [], []
    for k, P in enumerate(parts):
        X1, X2 = grid(Identity(), n, n, P['lim'])
        C10c = voigt_to_c10(P['scale'] * voigt)
        mm = mms_wave(X1, X2, C10c, rho=P['rho'], amp=P['amp'], phase=P['phase'])
        bc = []
        for f in range(4):
            if f == 1 - k:          # the interface face
                bc.append((TRACTION, None, T_ZERO, None, None))
                continue
            g = traction_data(mm, face_flat_index(f, n, n), outward_normal(Identity(), f, n, n, P['lim']))
            bc.append((TRACTION, g, T_COS, (mm['omega'], 0.0), None))
        blocks.append(dict(X1=X1, X2=X2, rho=P['rho'] * np.ones((n, n)), C10=C10c[:, None, None] * np.ones((1, n, n)),
                           bc=bc, forcing=(mm['f'], T_COS, (mm['omega'], 0.0))))
        mms.append(mm)
    # face 1 (x1 = 1/2) of block 0 meets face 0 of block 1, same point order
    ia, ib = face_flat_index(1, n, n), face_flat_index(0, n, n)
    V = mms[0]['u'].reshape(2, -1)[:, ia] - mms[1]['u'].reshape(2, -1)[:, ib]
    Th = (traction_data(mms[0], ia, outward_normal(Identity(), 1, n, n, parts[0]['lim']))
          + traction_data(mms[1], ib, outward_normal(Identity(), 0, n, n, parts[1]['lim'])))
    spec = dict(order=order, blocks=blocks, interfaces=[(0, 1, 1, 0, False)], sources=[], receivers=[],
                mms=mms, T=0.5, cfl=0.5)
    if jump_data:
        spec['interface_data'] = [(0, V, Th, T_COS, (mms[0]['omega'], 0.0))]
    return spec


def spec_c2(n=1025, seed=0, order=4, nrec=16):
    """Curvilinear block with Gaussian topography, random smooth SPD material,
    displacement on the bumped face x2 = 0, traction elsewhere, Ricker point force."""
    X1, X2 = grid(GaussianTopography(), n, n)
    rho, V = smooth_random_material(X1, X2, seed)
    bc = _free_faces()
    bc[2] = (DISPLACEMENT, None, T_ZERO, None, None)
    blk = dict(X1=X1, X2=X2, rho=rho, C10=voigt_to_c10(V), bc=bc, forcing=None)
    xr = np.linspace(0.05, 0.95, nrec) if nrec else np.zeros(0)
    return dict(order=order, blocks=[blk], interfaces=[],
                sources=[(0, 0.5, 0.75, 0.0, -1.0, 1.0, 10.0, 0.1)],
                receivers=[(0, xr, np.ones_like(xr))] if nrec else [],
                steps=2000, cfl=0.5)


def spec_c3(n=2049, seed=0, order=4, nrec=16):
    """2x2 conforming curvilinear blocks of one smooth map, material contrast 3
    in a checkerboard, traction on the top and left outer faces, displacement on
    the bottom and right ones, 16 receivers on the top face."""
    m = SineWarp()
    blocks = []
    for by in range(2):
        for bx in range(2):
            lim1 = (0.5 * bx, 0.5 * bx + 0.5)
            lim2 = (0.5 * by, 0.5 * by + 0.5)
            X1, X2 = grid(m, n, n, lim1, lim2)
            rho, V = smooth_random_material(X1, X2, seed)
            fac = 3.0 if (bx + by) % 2 else 1.0
            bc = _free_faces()
            if bx == 1:
                bc[1] = (DISPLACEMENT, None, T_ZERO, None, None)
            if by == 0:
                bc[2] = (DISPLACEMENT, None, T_ZERO, None, None)
            blocks.append(dict(X1=X1, X2=X2, rho=fac * rho, C10=fac * voigt_to_c10(V), bc=bc, forcing=None))
    itfs = [(0, 1, 1, 0, False), (2, 1, 3, 0, False), (0, 3, 2, 2, False), (1, 3, 3, 2, False)]
    half = nrec // 2
    xr = (np.arange(half) + 0.5) / half
    recs = [(2, xr, np.ones(half)), (3, xr, np.ones(half))] if nrec else []
    return dict(order=order, blocks=blocks, interfaces=itfs,
                sources=[(2, 0.6, 0.3, 0.0, -1.0, 1.0, 10.0, 0.1)],
                receivers=recs, steps=1000, cfl=0.5)


def spec_shot(n, seed, order=4, nrec=64, device=None):
    """One served shot: Gaussian-topography block of n^2 points, its own random
    material (seed), Ricker source at a random interior point, receivers on x2 = 1."""
    rng = np.random.default_rng(10_000 + seed)
    X1, X2 = grid(GaussianTopography(), n, n)
    rho, V = smooth_random_material(X1, X2, seed, device=device)
    bc = _free_faces()
    bc[2] = (DISPLACEMENT, None, T_ZERO, None, None)
    xs = rng.uniform(0.1, 0.9, 2)
    xr = np.linspace(0.02, 0.98, nrec)
    return dict(order=order,
                blocks=[dict(X1=X1, X2=X2, rho=rho, C10=voigt_to_c10(V), bc=bc, forcing=None)],
                interfaces=[], sources=[(0, xs[0], xs[1], 0.0, -1.0, 1.0, 10.0, 0.1)],
                receivers=[(0, xr, np.ones(nrec))], steps=1500, cfl=0.5)


def blob(X1, X2, center=(0.5, 0.5), width=0.1):
    """Gaussian blob exp(-|X - center|^2 / (2 width^2)) on the physical grid."""
    return np.exp(-((X1 - center[0]) ** 2 + (X2 - center[1]) ** 2) / (2.0 * width ** 2))


def spec_c5(n=513, seed=0, order=4, nrec=100, perturbed=False):
    """Differentiation workload: Gaussian-topography block of n^2 points with its
    random smooth material (seed), displacement bottom and traction elsewhere,
    a 10 Hz vertical Ricker force at (0.5, 0.75) and nrec receivers on x2 = 1.
    perturbed=True multiplies rho and every stiffness field by (1 + 0.05 blob),
    the model of the observed data."""
    X1, X2 = grid(GaussianTopography(), n, n)
    rho, V = smooth_random_material(X1, X2, seed)
    C10 = voigt_to_c10(V)
    if perturbed:
        s = 1.0 + 0.05 * blob(X1, X2)
        rho, C10 = rho * s, C10 * s
    bc = _free_faces()
    bc[2] = (DISPLACEMENT, None, T_ZERO, None, None)
    xr = np.linspace(0.02, 0.98, nrec)
    return dict(order=order,
                blocks=[dict(X1=X1, X2=X2, rho=rho, C10=C10, bc=bc, forcing=None)],
                interfaces=[], sources=[(0, 0.5, 0.75, 0.0, -1.0, 1.0, 10.0, 0.1)],
                receivers=[(0, xr, np.ones(nrec))], steps=2000, cfl=0.5)


def smooth_direction(X1, X2, seed, nmodes=4, kmax=3):
    """A random smooth perturbation direction (rho (n2, n1), Voigt (6, n2, n1))
    for finite-difference checks: low Fourier modes per field."""
    rng = np.random.default_rng(50_000 + seed)
    out = []
    for _ in range(7):
        kx = rng.integers(-kmax, kmax + 1, nmodes)
        ky = rng.integers(-kmax, kmax + 1, nmodes)
        ph = rng.uniform(0.0, 2.0 * np.pi, nmodes)
        a = rng.normal(size=nmodes)
        s = np.zeros_like(X1)
        for m in range(nmodes):
            s += a[m] * np.cos(2.0 * np.pi * (kx[m] * X1 + ky[m] * X2) + ph[m])
        out.append(s / nmodes)
    return out[0], np.stack(out[1:])


# ---------------------------------------------------------------- 3-D inputs
def grid3(n1, n2, n3, eps=0.04):
    """Curvilinear map of the unit cube: arrays (n3, n2, n1), x1 fastest."""
    x3, x2, x1 = np.meshgrid(np.linspace(0, 1, n3), np.linspace(0, 1, n2), np.linspace(0, 1, n1), indexing='ij')
    bump = eps * np.sin(np.pi * x1) * np.sin(np.pi * x2) * np.sin(np.pi * x3)
    return x1 + bump, x2 + 0.6 * bump + eps * x3 * x1, x3 - 0.8 * bump


def random_material3(shape, seed, minor=False):
    """rho (shape) and C [81][shape]: a random positive definite 9 x 9 matrix
    (major symmetric; with minor=True from a 6 x 6 Voigt matrix, so also minor
    symmetric) times a smooth positive variation."""
    rng = np.random.default_rng(seed)
    if minor:
        Q = rng.normal(size=(6, 6))
        V = Q @ Q.T / 6 + np.eye(6)
        vi = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
        M = np.zeros((9, 9))
        for a, (i, j) in enumerate(vi):
            for b, (k, l) in enumerate(vi):
                for (p, q) in {(i, j), (j, i)}:
                    for (r, s) in {(k, l), (l, k)}:
                        M[3 * p + q, 3 * r + s] = V[a, b]
    else:
        Q = rng.normal(size=(9, 9))
        M = Q @ Q.T / 9 + np.eye(9)
    k = np.arange(int(np.prod(shape))).reshape(shape)
    var = 1.0 + 0.2 * np.sin(0.37 * k)
    rho = 1.0 + 0.3 * np.cos(0.11 * k)
    return rho, M.reshape(81, *([1] * len(shape))) * var
