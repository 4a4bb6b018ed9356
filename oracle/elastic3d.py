"""The scheme on a single curvilinear 3-D block (oracle, test infrastructure only).

The same semidiscrete scheme as oracle/elastic.py with d = 3 (the paper
states every operator for a general dimension; its experiments are 2-D):

* Grid X(x) of the reference cube, arrays of shape (n3, n2, n1) with x1 the
  fast index, x_a = i_a h_a, h_a = 1/(n_a - 1).
* Metric (Sec. 3.2, 3.3): A[i][I] = dX_I/dx_i with the first-derivative SBP
  operator along axis i, J = det A, F = A^{-1} (F[I][i] = dx_i/dX_I).
* Face scale factor (Sec. 3.2.2, eq. surfint_J): Jhat = |a_t1 x a_t2| with
  a_t = dX/dx_t the two tangential covariant basis vectors of the face;
  outward unit normal from Nanson's formula Jhat n_I = J F_Ia nu_a (eq. nanson).
* Volume: DD_ik(c_ijkl) u_l = sum_i D_ii^FC(c_ijil) u_l + sum_{i != k}
  D_i(c_ijkl D_k u_l) with c_ijkl = F_Ii J C_IjKl F_Kk (Sec. 4.6-4.7, eq.
  transf_density_stiffness); the physical operator is J^{-1} DD (Theorem 1).
* Traction T_JL = n_I C_IJKL F_Kk D_k (eq. discr_traction_op, eq. chain_discrete).
* Traction SAT (Sec. 5.1): -(JH)^{-1} e_f Jhat H_f (e_f^T T u - g).
* Displacement SAT (Sec. 5.2, eq. dirichlet_ansatz): (JH)^{-1} (T_LJ -
  Z_LJ)^T e_f Jhat H_f (e_f^T u_L - g_L), Z_JL = beta d Jhat/(h_1 J)
  n_I C_IJKL n_K with d = 3 (Sec. 4.5, eq. borrowing_nd_H_global).
* H = H_1 (x) H_2 (x) H_3, face quadrature H_f the product of the two
  tangential norms, h_1 the first norm weight in the face-normal direction.

Parity status: pinned (tests/test_oracle_3d.py: brute-force symmetry and
negative semidefiniteness of diag(JH) D^tot for traction and displacement
faces on a curved block, constant fields in the traction-only null space, the
extruded plane-strain reduction to the pinned 2-D operator, affine metric
identities, manufactured-solution convergence).
"""
import numpy as np
import scipy.sparse as sps

from . import sbp
from .material import transform

TRACTION, DISPLACEMENT = 0, 2
DIM = 3
# faces: (axis a of x1/x2/x3, side 0 = lower / 1 = upper), in the order x1=0, x1=1, x2=0, x2=1, x3=0, x3=1
FACES3 = [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0), (2, 1)]


def _along(Dm, U, axis):
    """Apply the sparse 1-D operator Dm along array axis `axis` of U (3-D)."""
    V = np.moveaxis(U, axis, 0)
    sh = V.shape
    out = np.asarray(Dm @ V.reshape(sh[0], -1)).reshape((Dm.shape[0],) + sh[1:])
    return np.moveaxis(out, 0, axis)


def _axis(i):
    """Array axis of reference direction i (arrays are (n3, n2, n1))."""
    return 2 - i


def apply_d1(U, h, order, i):
    n = U.shape[_axis(i)]
    return _along(sbp.d1(n, h, order), U, _axis(i))


def apply_d2fc(U, Bc, h, order, i):
    """D2^FC(b) along every grid line of reference direction i (line-wise b),
    in the literal SBP form H^{-1}(-D1^T H b D1 u - R(b) u + boundary terms)
    of Sec. 4.1, as oracle/sbp.apply_d2fc does in 2-D."""
    ax = _axis(i)
    n = U.shape[ax]
    Hd, D, W = sbp._ops(n, h, order)
    sh = [1, 1, 1]
    sh[ax] = n
    Hb = Hd.reshape(sh)
    DU = _along(D, U, ax)
    wide = _along(D.T, Hb * Bc * DU, ax)
    shw = [1, 1, 1]
    shw[ax] = -1
    gam = W.gamma.reshape(shw)
    rem = _along(W.delta.T, gam * _along(W.avg, Bc, ax) * _along(W.delta, U, ax), ax) / h
    out = -wide - rem
    first = [slice(None)] * 3
    last = [slice(None)] * 3
    first[ax], last[ax] = 0, n - 1
    first, last = tuple(first), tuple(last)
    out[first] -= Bc[first] * DU[first]
    out[last] += Bc[last] * DU[last]
    return out / Hb


def face_index3(f, n1, n2, n3):
    """Flat indices of the points of face f, as an array shaped like the face
    (tangential directions in increasing order, the lower one fast)."""
    a, s = FACES3[f]
    I = np.arange(n1 * n2 * n3).reshape(n3, n2, n1)
    c = 0 if s == 0 else [n1, n2, n3][a] - 1
    sl = [slice(None)] * 3
    sl[_axis(a)] = c
    return I[tuple(sl)]


class Block3D:
    def __init__(self, X1, X2, X3, rho, C, order=4, beta=1.0):
        self.order, self.beta = order, beta
        X = [np.asarray(x, dtype=float) for x in (X1, X2, X3)]
        self.n3, self.n2, self.n1 = X[0].shape
        self.n = (self.n1, self.n2, self.n3)
        self.h = tuple(1.0 / (m - 1) for m in self.n)
        self.npts = self.n1 * self.n2 * self.n3
        # A[i][I] = dX_I / dx_i
        A = np.empty((3, 3) + X[0].shape)
        for i in range(3):
            for I in range(3):
                A[i, I] = apply_d1(X[I], self.h[i], order, i)
        Am = np.moveaxis(A, (0, 1), (-2, -1))
        J = np.linalg.det(Am)
        if np.any(J <= 0):
            raise ValueError("non-positive discrete Jacobian")
        Fm = np.linalg.inv(Am)               # Fm[..., I, i] = dx_i / dX_I
        self.A, self.J = A, J
        self.F = np.moveaxis(Fm, (-2, -1), (0, 1))
        self.rho = np.asarray(rho, dtype=float) * np.ones_like(J)
        C = np.asarray(C, dtype=float)
        if C.ndim == 4:                       # one constant tensor for every point
            C = C[..., None, None, None]
        self.C = C * np.ones((3, 3, 3, 3) + J.shape)
        self.c = transform(self.C, self.F, self.J)
        Hs = [sbp.norm(m, hh, order) for m, hh in zip(self.n, self.h)]
        self.Hn = Hs
        self.H = Hs[2][:, None, None] * Hs[1][None, :, None] * Hs[0][None, None, :]
        self.bc = [dict(kind=TRACTION, g=None, tfun=None) for _ in range(6)]
        self.faces = [self._face(f) for f in range(6)]

    def _face(self, f):
        a, s = FACES3[f]
        t1, t2 = [t for t in range(3) if t != a]
        idx = face_index3(f, *self.n)
        fl = idx.ravel()
        at1 = np.stack([self.A[t1, I].ravel()[fl] for I in range(3)])
        at2 = np.stack([self.A[t2, I].ravel()[fl] for I in range(3)])
        Jhat = np.linalg.norm(np.cross(at1, at2, axis=0), axis=0)
        nu = -1.0 if s == 0 else 1.0
        Jf = self.J.ravel()[fl]
        nrm = np.stack([Jf * self.F[I, a].ravel()[fl] * nu / Jhat for I in range(3)])
        Hf = np.outer(self.Hn[t2], self.Hn[t1]).ravel()     # face arrays: t1 fast
        E = sps.csr_matrix((np.ones(len(fl)), (np.arange(len(fl)), fl)), shape=(len(fl), self.npts))
        # E_f D_k for the three reference directions (sparse, nf x npts)
        ED = []
        for k in range(3):
            Dk = sbp.d1(self.n[k], self.h[k], self.order)
            mats = [sps.identity(self.n[0]), sps.identity(self.n[1]), sps.identity(self.n[2])]
            mats[k] = Dk
            Dfull = sps.kron(mats[2], sps.kron(mats[1], mats[0])).tocsr()
            ED.append((E @ Dfull).tocsr())
        Cf = self.C.reshape(3, 3, 3, 3, -1)[..., fl]
        Ff = self.F.reshape(3, 3, -1)[..., fl]
        return dict(idx=fl, shape=idx.shape, axis=a, nu=nu, E=E, ED=ED, Hf=Hf, h_1=self.Hn[a][0],
                    Jhat=Jhat, n=nrm, Cf=Cf, Ff=Ff, Jf=Jf)

    def traction(self, f, u):
        """e_f^T T_JL u_L = n_I C_IJKL F_Kk D_k u_L on face f, shape (3, nf)."""
        fo = self.faces[f]
        Du = np.stack([[fo['ED'][k] @ u[L].ravel() for k in range(3)] for L in range(3)])   # [L, k]
        DK = np.einsum('Kkf,Lkf->LKf', fo['Ff'], Du)
        return np.einsum('If,IJKLf,LKf->Jf', fo['n'], fo['Cf'], DK)

    def traction_transpose(self, f, y):
        """sum_L (e_f^T T_LJ)^T y_L for a face vector y (3, nf) -> volume (3, npts)."""
        fo = self.faces[f]
        coef = np.einsum('If,ILKJf,Kkf->LJkf', fo['n'], fo['Cf'], fo['Ff'])
        out = np.zeros((3, self.npts))
        for J in range(3):
            for L in range(3):
                for k in range(3):
                    out[J] += fo['ED'][k].T @ (coef[L, J, k] * y[L])
        return out

    def nCn(self, f):
        fo = self.faces[f]
        return np.einsum('If,IJKLf,Kf->JLf', fo['n'], fo['Cf'], fo['n'])

    def face_values(self, f, u):
        return np.stack([u[L].ravel()[self.faces[f]['idx']] for L in range(3)])

    def lift(self, f, y):
        """(JH)^{-1} e_f Jhat H_f y -> volume (3, npts)."""
        fo = self.faces[f]
        w = fo['Jhat'] * fo['Hf']
        out = np.stack([fo['E'].T @ (w * y[J]) for J in range(3)])
        return out / (self.J * self.H).ravel()

    def volume(self, u):
        """DD_ik(c_ijkl) u_l in the reference domain, shape (3, n3, n2, n1)."""
        c, o, h = self.c, self.order, self.h
        r = np.zeros((3,) + self.J.shape)
        for j in range(3):
            for l in range(3):
                for i in range(3):
                    r[j] += apply_d2fc(u[l], c[i, j, i, l], h[i], o, i)
                    for k in range(3):
                        if k != i:
                            r[j] += apply_d1(c[i, j, k, l] * apply_d1(u[l], h[k], o, k), h[i], o, i)
        return r


class Problem3D:
    """One block with boundary conditions and separable forcing."""

    def __init__(self, block, beta=1.0):
        self.block = block
        self.beta = beta
        self.forcing = None      # (F_space (3, n3, n2, n1), tfun)

    def set_bc(self, face, kind, g=None, tfun=None):
        if kind not in (TRACTION, DISPLACEMENT):
            raise ValueError(kind)
        self.block.bc[face] = dict(kind=kind, g=g, tfun=tfun)

    def sat(self, u, t, homogeneous):
        B = self.block
        out = np.zeros((3, B.npts))
        for f in range(6):
            bc, fo = B.bc[f], B.faces[f]
            nf = len(fo['idx'])
            g = np.zeros((3, nf))
            if not homogeneous and bc['g'] is not None and bc['tfun'] is not None:
                g = np.asarray(bc['g']).reshape(3, nf) * bc['tfun'](t)
            if bc['kind'] == TRACTION:
                out -= B.lift(f, B.traction(f, u) - g)
            else:
                w = fo['Jhat'] * fo['Hf'] * (B.face_values(f, u) - g)
                Z = self.beta * DIM * fo['Jhat'] / (fo['h_1'] * fo['Jf']) * B.nCn(f)
                term = B.traction_transpose(f, w)
                for J in range(3):
                    term[J] -= fo['E'].T @ np.einsum('Lf,Lf->f', Z[:, J], w)
                out += term / (B.J * B.H).ravel()
        return out

    def total_operator(self, u, t=0.0, homogeneous=True):
        """D^tot u = J^{-1} DD u + SAT (physical form), shape (3, npts)."""
        B = self.block
        return (B.volume(u) / B.J).reshape(3, -1) + self.sat(u, t, homogeneous)

    def rhs(self, us, t, vs=None):
        """u_tt = rho^{-1} (D^tot u + f), as a one-element list (the time
        stepper of oracle/timestep.py works on lists of blocks)."""
        B = self.block
        r = self.total_operator(us[0], t, homogeneous=False)
        if self.forcing is not None:
            Fs, tf = self.forcing
            r = r + Fs.reshape(3, -1) * tf(t)
        return [(r / B.rho.ravel()).reshape((3,) + B.J.shape)]

    def energy(self, u, v):
        """1/2 (v^T P H v - u^T A u), A = diag(JH) D^tot (Sec. 7.2)."""
        B = self.block
        L = self.total_operator(u)
        w = (B.J * B.H).ravel()
        kin = np.sum((B.rho.ravel() * w) * (v.reshape(3, -1) ** 2).sum(0))
        pot = np.sum(w * (u.reshape(3, -1) * L).sum(0))
        return 0.5 * (kin - pot)

    def assemble(self):
        """Brute-force A = diag(JH) D^tot (3 npts square) from unit vectors."""
        B = self.block
        n = 3 * B.npts
        A = np.zeros((n, n))
        Hall = np.tile((B.J * B.H).ravel(), 3)
        for col in range(n):
            e = np.zeros(n)
            e[col] = 1.0
            A[:, col] = Hall * self.total_operator(e.reshape((3,) + B.J.shape)).ravel()
        return A


def vmax2(block, ndir=2000):
    """max over unit directions xi of lambda_max(xi_i c_ijkl xi_k) / rho~ over
    the block (Fibonacci sphere of directions; the dt rule of Sec. 7)."""
    k = np.arange(ndir) + 0.5
    z = 1.0 - 2.0 * k / ndir
    r = np.sqrt(1.0 - z * z)
    ph = np.pi * (1.0 + 5 ** 0.5) * k
    xi = np.stack([r * np.cos(ph), r * np.sin(ph), z])
    c = block.c.reshape(3, 3, 3, 3, -1)
    rt = (block.rho * block.J).ravel()
    best = 0.0
    for d in range(ndir):
        G = np.einsum('i,ijklp,k->pjl', xi[:, d], c, xi[:, d])
        best = max(best, float(np.max(np.linalg.eigvalsh(G)[:, -1] / rt)))
    return best


def dt_cfl(block, cfl):
    return cfl * min(block.h) / np.sqrt(vmax2(block))
