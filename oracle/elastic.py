"""Discrete elastic operator and SATs in physical form (oracle, test infrastructure only).

Semidiscrete scheme (Sec. 5, eq. semidiscrete_general):

    rho u_tt = D^Omega(C) u + f + SAT,      D^Omega(C) = J^{-1} DD_ik(c_ijkl)

* DD_ik(b) = D_ii^FC(b) for i = k, D_i b D_k for i != k (Sec. 4.6, eq. def_cd);
  the elastic operator is DD_ik(c_ijkl) u_l (Sec. 4.7) and the physical one is
  scaled by J^{-1} (Theorem 1).  Block(operator='wide') replaces D_ii^FC(b) by
  D_i b D_i, the wide-stencil operator compared in Sec. 7.1 with the same SATs.
* Discrete traction T_JL = n_I C_IJKL D_K with D_K = F_Kk D_k
  (eq. discr_traction_op, eq. chain_discrete).
* Robin / traction SAT (Sec. 5.1, eq. sat_traction):
  SAT_J = -(JH)^{-1} sum_f e_f Jhat H_f ( e_f^T (T_JL u_L + U_JL u_L) - g_J ).
* Dissipative Robin term (the remark after eq. sat_traction): T u + U u + V u_t = g
  with V symmetric PSD, imposed by adding -(JH)^{-1} sum_f e_f Jhat H_f V v to the
  Robin SAT (Problem.dissipation; v = u_t enters the RHS only through it).
* Displacement SAT (Sec. 5.2, eq. dirichlet_ansatz, Theorem 2):
  SAT_J = (JH)^{-1} sum_f (T_LJ - Z_LJ)^T e_f Jhat H_f (e_f^T u_L - g_L),
  Z_JL = beta d Jhat / (h_1 J) n_I C_IJKL n_K.
* Interface SAT (Sec. 6, eq. scheme_interface) with
  Z_JL = beta d Jhat / 4 ( nCn^u / (h_1^u J^u) + nCn^v / (h_1^v J^v) ).
  When the two sides have different first norm weights, each side's term uses
  its own h_1 (the Z = Z^u + Z^v split of the stability proof in Sec. 6).

Faces are treated one at a time (Sec. 4.3, eq. set_of_faces): on each face the
normal, Jhat and the face quadrature H_f take that face's values, including at
its end points, so corner points receive the SATs of both faces.  h_1 is the
first weight of the 1-D norm in the face-normal direction.  d = 2.

Parity status: pinned (tests/test_oracle_2d.py: brute-force symmetry of
A = diag(JH, JH) D^tot and negative semidefiniteness for every boundary type and
for a two-block interface, translation null space for traction-only blocks,
constant-coefficient textbook reduction, isotropic reduction;
tests/test_oracle_time.py: manufactured-solution convergence, energy;
tests/test_oracle_dissipation.py: the energy rate equals the dissipation of the
V terms, and an impedance face reflects the textbook fraction of a plane wave;
tests/test_oracle_wide.py: the wide operator's squared-stencil rows, its PSD
difference from the narrow one, symmetry, convergence and the accuracy and
spectral-radius comparisons of Sec. 7.1).
"""
import numpy as np
import scipy.sparse as sps

from . import sbp
from .geometry import metrics, face_index, FACES
from .material import transform

TRACTION, ROBIN, DISPLACEMENT, INTERFACE = 0, 1, 2, 3
DIM = 2


class Block:
    """One curvilinear block: grid, density, stiffness, boundary conditions."""

    def __init__(self, X1, X2, rho, C, order=4, beta=1.0, operator='narrow'):
        if operator not in ('narrow', 'wide'):
            raise ValueError(operator)
        self.order = order
        self.beta = beta
        # 'narrow': D_ii^FC(c) (Sec. 4.1); 'wide': D_i c D_i with the first
        # derivative applied twice (the wide-stencil operator the narrow one is
        # compared with in Sec. 7.1; fully compatible in the sense of Sec. 4.7)
        self.operator = operator
        self.X1 = np.asarray(X1, dtype=float)
        self.X2 = np.asarray(X2, dtype=float)
        self.n2, self.n1 = self.X1.shape
        self.npts = self.n1 * self.n2
        self.geo = metrics(self.X1, self.X2, order)
        self.J = self.geo['J']
        self.F = self.geo['F']
        self.h1, self.h2 = self.geo['h']
        self.rho = np.asarray(rho, dtype=float) * np.ones_like(self.J)
        self.C = np.asarray(C, dtype=float) * np.ones((2, 2, 2, 2) + self.J.shape)
        self.c = transform(self.C, self.F, self.J)
        self.H1 = sbp.norm(self.n1, self.h1, order)
        self.H2 = sbp.norm(self.n2, self.h2, order)
        self.H = np.outer(self.H2, self.H1)
        self.bc = [dict(kind=TRACTION, g=None, tfun=None, U=None) for _ in range(4)]
        self._face_ops = [self._build_face_ops(f) for f in range(4)]

    # --------------------------------------------------------- face helpers
    def _build_face_ops(self, f):
        """Sparse E_f^T D_k (k = 0, 1) and per-face metric data."""
        g = self.geo['faces'][f]
        idx = g['idx']
        nf = len(idx)
        n1, n2, o = self.n1, self.n2, self.order
        D1x = sbp.d1(n1, self.h1, o)
        D1y = sbp.d1(n2, self.h2, o)
        a, s = FACES[f]
        if a == 0:
            i0 = 0 if s == 0 else n1 - 1
            sel = sps.csr_matrix(([1.0], ([0], [i0])), shape=(1, n1))
            ED0 = sps.kron(sps.identity(n2), D1x[i0:i0 + 1, :])      # normal
            ED1 = sps.kron(D1y, sel)                                 # tangential
            Hf = self.H2
            h_1 = self.H1[0]
        else:
            j0 = 0 if s == 0 else n2 - 1
            sel = sps.csr_matrix(([1.0], ([0], [j0])), shape=(1, n2))
            ED0 = sps.kron(sel, D1x)                                 # tangential
            ED1 = sps.kron(D1y[j0:j0 + 1, :], sps.identity(n1))     # normal
            Hf = self.H1
            h_1 = self.H2[0]
        E = sps.csr_matrix((np.ones(nf), (np.arange(nf), idx)), shape=(nf, self.npts))
        Cf = self.C.reshape(2, 2, 2, 2, -1)[..., idx]
        Ff = self.F.reshape(2, 2, -1)[..., idx]
        return dict(idx=idx, E=E, ED=[ED0.tocsr(), ED1.tocsr()], Hf=Hf, h_1=h_1,
                    Jhat=g['Jhat'], n=g['n'], Cf=Cf, Ff=Ff,
                    Jf=self.J.ravel()[idx], JH=(self.J * self.H).ravel()[idx])

    def traction(self, f, u):
        """e_f^T T_JL u_L on face f: n_I C_IJKL F_Kk D_k u_L, shape (2, nf)."""
        fo = self._face_ops[f]
        n, Cf, Ff = fo['n'], fo['Cf'], fo['Ff']
        Du = np.stack([[fo['ED'][k] @ u[L].ravel() for k in range(2)] for L in range(2)])  # [L,k]
        DK = np.einsum('Kkf,Lkf->LKf', Ff, Du)
        return np.einsum('If,IJKLf,LKf->Jf', n, Cf, DK)

    def traction_transpose(self, f, y):
        """sum_L (e_f^T T_LJ)^T y_L for face vectors y (2, nf) -> volume (2, npts)."""
        fo = self._face_ops[f]
        n, Cf, Ff = fo['n'], fo['Cf'], fo['Ff']
        # coefficient of ED[k] for the map y_L -> component J: sum_IK n_I C_ILKJ F_Kk
        coef = np.einsum('If,ILKJf,Kkf->LJkf', n, Cf, Ff)
        out = np.zeros((2, self.npts))
        for J in range(2):
            for L in range(2):
                for k in range(2):
                    out[J] += fo['ED'][k].T @ (coef[L, J, k] * y[L])
        return out

    def nCn(self, f):
        fo = self._face_ops[f]
        return np.einsum('If,IJKLf,Kf->JLf', fo['n'], fo['Cf'], fo['n'])

    def face_values(self, f, u):
        idx = self._face_ops[f]['idx']
        return np.stack([u[L].ravel()[idx] for L in range(2)])

    def spread(self, f, y):
        """e_f Jhat H_f y for a face vector y (2, nf) -> volume (2, npts)."""
        fo = self._face_ops[f]
        out = np.zeros((2, self.npts))
        w = fo['Jhat'] * fo['Hf']
        for J in range(2):
            out[J] = fo['E'].T @ (w * y[J])
        return out

    def lift(self, f, y):
        """(JH)^{-1} e_f Jhat H_f y -> volume (2, npts)."""
        return self.spread(f, y) / (self.J * self.H).ravel()

    # ------------------------------------------------------------- volume
    def volume(self, u):
        """DD_ik(c_ijkl) u_l in the reference domain (Sec. 4.7), shape (2, n2, n1)."""
        c, o, h1, h2 = self.c, self.order, self.h1, self.h2
        r = np.zeros((2, self.n2, self.n1))
        for j in range(2):
            for l in range(2):
                if self.operator == 'wide':
                    r[j] += sbp.apply_d1(c[0, j, 0, l] * sbp.apply_d1(u[l], h1, o, axis=1), h1, o, axis=1)
                    r[j] += sbp.apply_d1(c[1, j, 1, l] * sbp.apply_d1(u[l], h2, o, axis=0), h2, o, axis=0)
                else:
                    r[j] += sbp.apply_d2fc(u[l], c[0, j, 0, l], h1, o, axis=1)
                    r[j] += sbp.apply_d2fc(u[l], c[1, j, 1, l], h2, o, axis=0)
                r[j] += sbp.apply_d1(c[0, j, 1, l] * sbp.apply_d1(u[l], h2, o, axis=0), h1, o, axis=1)
                r[j] += sbp.apply_d1(c[1, j, 0, l] * sbp.apply_d1(u[l], h1, o, axis=1), h2, o, axis=0)
        return r


class Interface:
    """Conforming interface: face fa of block a meets face fb of block b.

    ``reversed`` is True when the two faces are traversed in opposite
    directions.  V and Theta are optional jump data (2, nf) for displacement
    and traction (Sec. 6, eq. interface_phys): u^a - u^b = V tfun(t) and
    tau^a + tau^b = Theta tfun(t), in side a's point order (tfun None: 1).
    """

    def __init__(self, a, fa, b, fb, reversed=False, V=None, Theta=None, tfun=None):
        self.a, self.fa, self.b, self.fb = a, fa, b, fb
        self.reversed = reversed
        self.V = V
        self.Theta = Theta
        self.tfun = tfun


class Problem:
    """A set of blocks with boundary conditions, interfaces, forcing and sources."""

    def __init__(self, blocks, interfaces=(), beta=1.0):
        self.blocks = list(blocks)
        self.interfaces = list(interfaces)
        self.beta = beta
        self.forcing = [None] * len(self.blocks)     # (F_space (2,n2,n1), tfun)
        self.sources = []                            # dicts, see sources.point_source
        for itf in self.interfaces:
            A, B = self.blocks[itf.a], self.blocks[itf.b]
            if len(A._face_ops[itf.fa]['idx']) != len(B._face_ops[itf.fb]['idx']):
                raise ValueError("non-conforming interface")
            A.bc[itf.fa] = dict(kind=INTERFACE, itf=itf, side=0)
            B.bc[itf.fb] = dict(kind=INTERFACE, itf=itf, side=1)

    def set_bc(self, blk, face, kind, g=None, tfun=None, U=None, V=None):
        """V (traction and Robin faces): the dissipative term V_JL du_L/dt of the
        generalised Robin condition (the remark after eq. sat_traction, Sec. 5.1),
        shape (2, 2, nf), symmetric positive semidefinite per face point."""
        self.blocks[blk].bc[face] = dict(kind=kind, g=g, tfun=tfun, U=U, V=V)

    # ------------------------------------------------------------ the SATs
    def _data(self, bc, t, nf):
        if bc.get('g') is None or bc.get('tfun') is None:
            return np.zeros((2, nf))
        return bc['g'] * bc['tfun'](t)

    def sat(self, k, us, t, homogeneous):
        B = self.blocks[k]
        u = us[k]
        out = np.zeros((2, B.npts))
        for f in range(4):
            bc = B.bc[f]
            fo = B._face_ops[f]
            nf = len(fo['idx'])
            if bc['kind'] in (TRACTION, ROBIN):
                y = B.traction(f, u)
                if bc['kind'] == ROBIN and bc.get('U') is not None:
                    y = y + np.einsum('JLf,Lf->Jf', bc['U'], B.face_values(f, u))
                if not homogeneous:
                    y = y - self._data(bc, t, nf)
                out -= B.lift(f, y)
            elif bc['kind'] == DISPLACEMENT:
                delta = B.face_values(f, u)
                if not homogeneous:
                    delta = delta - self._data(bc, t, nf)
                w = fo['Jhat'] * fo['Hf'] * delta                      # Jhat H_f (u - g)
                Z = self.beta * DIM * fo['Jhat'] / (fo['h_1'] * fo['Jf']) * B.nCn(f)
                term = B.traction_transpose(f, w)
                for J in range(2):
                    term[J] -= fo['E'].T @ np.einsum('Lf,Lf->f', Z[:, J], w)
                out += term / (B.J * B.H).ravel()
            else:
                out += self._interface_sat(k, f, bc, us, t, homogeneous)
        return out

    def _partner(self, bc):
        itf = bc['itf']
        if bc['side'] == 0:
            return itf.b, itf.fb, 1.0
        return itf.a, itf.fa, -1.0

    def _interface_sat(self, k, f, bc, us, t, homogeneous):
        itf = bc['itf']
        B = self.blocks[k]
        pk, pf, sgn = self._partner(bc)
        P = self.blocks[pk]
        fo, po = B._face_ops[f], P._face_ops[pf]
        perm = slice(None, None, -1) if itf.reversed else slice(None)
        u_f = B.face_values(f, us[k])
        v_f = P.face_values(pf, us[pk])[:, perm]
        Tu = B.traction(f, us[k])
        Tv = P.traction(pf, us[pk])[:, perm]
        jump = u_f - v_f
        th = np.zeros_like(jump)
        own = slice(None) if sgn > 0 else perm      # V, Theta are stored in side a's order
        if not homogeneous:
            tv = 1.0 if itf.tfun is None else itf.tfun(t)
            if itf.V is not None:
                jump = jump - sgn * tv * itf.V[:, own]
            if itf.Theta is not None:
                th = tv * itf.Theta[:, own]
        Jhat = fo['Jhat']
        Z = self.beta * DIM * Jhat / 4.0 * (
            B.nCn(f) / (fo['h_1'] * fo['Jf'])
            + P.nCn(pf)[..., perm] / (po['h_1'] * po['Jf'][perm]))
        w = Jhat * fo['Hf'] * jump
        out = np.zeros((2, B.npts))
        for J in range(2):
            out[J] -= fo['E'].T @ np.einsum('Lf,Lf->f', Z[:, J], w)
        out += 0.5 * B.traction_transpose(f, w)
        out -= 0.5 * B.spread(f, Tu + Tv - th)
        return out / (B.J * B.H).ravel()

    # ----------------------------------------------------------- the RHS
    def total_operator(self, us, t=0.0, homogeneous=True):
        """D^tot u = D^Omega u + SAT (physical form), per block, shape (2, npts)."""
        out = []
        for k, B in enumerate(self.blocks):
            vol = (B.volume(us[k]) / B.J).reshape(2, -1)
            out.append(vol + self.sat(k, us, t, homogeneous))
        return out

    def dissipation(self, k, vs):
        """SAT of the dissipative Robin term on block k: the Robin SAT with
        T u + U u - g replaced by V u_t, i.e. -(JH)^{-1} sum_f e_f Jhat H_f V v."""
        B = self.blocks[k]
        out = np.zeros((2, B.npts))
        for f in range(4):
            bc = B.bc[f]
            if bc['kind'] in (TRACTION, ROBIN) and bc.get('V') is not None:
                out -= B.lift(f, np.einsum('JLf,Lf->Jf', bc['V'], B.face_values(f, vs[k])))
        return out

    def rhs(self, us, t, vs=None):
        """Acceleration u_tt = rho^{-1} (D^Omega u + f + SAT) for every block;
        the velocities vs enter the dissipative Robin terms (omitted when None)."""
        L = self.total_operator(us, t, homogeneous=False)
        out = []
        for k, B in enumerate(self.blocks):
            r = L[k]
            if vs is not None:
                r = r + self.dissipation(k, vs)
            if self.forcing[k] is not None:
                Fs, tf = self.forcing[k]
                r = r + Fs.reshape(2, -1) * tf(t)
            for s in self.sources:
                if s['block'] == k:
                    amp = s['tfun'](t)
                    for p, w in zip(s['idx'], s['w']):
                        r[:, p] += s['dir'] * amp * w / (B.J.ravel()[p] * B.H.ravel()[p])
            out.append((r / B.rho.ravel()).reshape(2, B.n2, B.n1))
        return out

    # ------------------------------------------------------- diagnostics
    def inner(self, k, a, b):
        """Physical discrete inner product sum J H a_J b_J on block k."""
        B = self.blocks[k]
        return float(np.sum((B.J * B.H).ravel() * (a.reshape(2, -1) * b.reshape(2, -1)).sum(0)))

    def energy(self, us, vs):
        """eps = 1/2 (v^T P H v - u^T A u), A = diag(JH) D^tot (Sec. 7.2)."""
        L = self.total_operator(us, homogeneous=True)
        e = 0.0
        for k, B in enumerate(self.blocks):
            kin = np.sum((B.rho * B.J * B.H).ravel() * (vs[k].reshape(2, -1) ** 2).sum(0))
            pot = self.inner(k, us[k], L[k])
            e += 0.5 * (kin - pot)
        return e

    def assemble(self):
        """Brute-force A = diag(JH, JH) D^tot by applying D^tot to unit vectors."""
        sizes = [2 * B.npts for B in self.blocks]
        offs = np.concatenate([[0], np.cumsum(sizes)])
        ntot = offs[-1]
        A = np.zeros((ntot, ntot))
        Hall = np.concatenate([np.tile((B.J * B.H).ravel(), 2) for B in self.blocks])
        for col in range(ntot):
            e = np.zeros(ntot)
            e[col] = 1.0
            us = [e[offs[k]:offs[k + 1]].reshape(2, B.n2, B.n1) for k, B in enumerate(self.blocks)]
            L = self.total_operator(us)
            A[:, col] = Hall * np.concatenate([x.ravel() for x in L])
        return A
