"""Gradient of a receiver misfit with respect to rho and C by the discrete adjoint.

    J(rho, C) = 1/2 sum_{n=1..N} sum_r |S_r u_n - d_{n,r}|^2

for a forward run of N classical RK4 steps (Sec. 7.1) from rest.  The
gradient is the exact derivative of the discrete map (up to rounding):

* Forward: ``sbpe_advance`` with a checkpoint of (u, v, t) every
  ``checkpoint_every`` steps; J from the recorded receiver traces.
* Reverse, segment by segment from the last checkpoint: the segment's states
  are recomputed with the stage form of RK4 (``sbpe_apply`` with the data at
  the stage times, ``sbpe_lincomb`` for the stage combinations), then each
  step is reversed: with b = (1/6, 1/3, 1/3, 1/6), c = (0, 1/2, 1/2, 1), the
  stage-slope adjoints k_i = dt b_i y^ are propagated from the last stage to
  the first through (u, v) -> (L^T v, u).  Because H L is symmetric (the energy
  analysis of Sec. 5), in the variables y^ = y / (H rho~) the transpose is the
  forward operator itself, so ``sbpe_apply`` (homogeneous) advances the
  adjoint state.  Each stage adds its parameter term with
  ``sbpe_grad_accumulate``; the receiver residuals enter through
  ``sbpe_receiver_adjoint``.
* ``sbpe_grad_to_physical`` maps the gradients with respect to the stored
  c = F J C F and rho~ = J rho to C (C10 layout) and rho.

``MisfitGradient`` wraps one forward/adjoint pair for a fixed time step (the
step must not depend on the parameters being differentiated), and
``SeismicMisfit`` exposes it as a ``torch.autograd.Function``.
"""
import numpy as np

from . import sbpe as S
from .solver import Solver

B_RK = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
C_RK = (0.0, 0.5, 0.5, 1.0)


class MisfitGradient:
    """Forward run, misfit and adjoint gradient of one single-block problem.

    spec: a problem specification (see workloads.py) with receivers; its
    block's 'rho' and 'C10' are the parameters.  d_obs: observed traces
    (nsteps, nrec, 2) or None (then J = 1/2 sum |S u|^2).
    """

    def __init__(self, spec, nsteps, dt, d_obs=None, dtype='f64', device=0, checkpoint_every=100):
        import torch
        if len(spec['blocks']) != 1:
            raise ValueError('single-block problems only')
        self.torch = torch
        self.spec, self.nsteps, self.dt = spec, nsteps, dt
        self.K = max(1, int(checkpoint_every))
        self.sol = Solver(spec, dtype, device=device)
        self.dev = self.sol.device
        self.tdt = self.sol.tdtype
        self.shape = self.sol.u[0].shape
        self.count = self.sol.u[0].numel()
        self.nrec = self.sol.nrec
        self.d_obs = None if d_obs is None else np.asarray(d_obs, dtype=float)

    def close(self):
        self.sol.close()

    # ------------------------------------------------------------ helpers
    def _new(self):
        return self.torch.empty(self.shape, dtype=self.tdt, device=self.dev)

    def _lin(self, coefs, xs, out):
        S.sbpe_lincomb(self.sol.ctx, coefs, [x.data_ptr() for x in xs], out.data_ptr(), self.count)

    def _apply(self, x, t, homogeneous, out):
        S.sbpe_apply(self.sol.ctx, [x.data_ptr()], [out.data_ptr()], t, homogeneous)

    def _stages(self, u, v, t):
        """Stage displacements U_i, velocities V_i and values a_i of one step."""
        h = self.dt
        U, V, A = [u], [v], []
        for i in range(4):
            a = self._new()
            self._apply(U[i], t + C_RK[i] * h, False, a)
            A.append(a)
            if i < 3:
                Un, Vn = self._new(), self._new()
                self._lin([1.0, C_RK[i + 1] * h], [u, V[i]], Un)
                self._lin([1.0, C_RK[i + 1] * h], [v, A[i]], Vn)
                U.append(Un)
                V.append(Vn)
        return U, V, A

    def _step(self, u, v, t):
        h = self.dt
        U, V, A = self._stages(u, v, t)
        un, vn = self._new(), self._new()
        self._lin([1.0, h * B_RK[0], h * B_RK[1], h * B_RK[2]], [u, V[0], V[1], V[2]], un)
        self._lin([1.0, h * B_RK[3]], [un, V[3]], un)
        self._lin([1.0, h * B_RK[0], h * B_RK[1], h * B_RK[2]], [v, A[0], A[1], A[2]], vn)
        self._lin([1.0, h * B_RK[3]], [vn, A[3]], vn)
        return un, vn

    # ------------------------------------------------------------ forward
    def forward(self):
        """Run from rest with checkpoints; returns J (and keeps the traces)."""
        torch = self.torch
        sol = self.sol
        sol.set_state(None, None, 0.0)
        self.checkpoints = []
        done = 0
        while done < self.nsteps:
            self.checkpoints.append((sol.u[0].clone(), sol.v[0].clone(), sol.time(), done))
            k = min(self.K, self.nsteps - done)
            sol.advance(k, self.dt)
            done += k
        torch.cuda.synchronize(self.dev)
        self.traces = sol.receivers()
        res = self.traces if self.d_obs is None else self.traces - self.d_obs
        self.residuals = res
        return 0.5 * float(np.sum(res * res))

    # ------------------------------------------------------------ reverse
    def gradient(self):
        """(dJ/drho (n2, n1), dJ/dC10 (10, n2, n1)) after ``forward``."""
        torch = self.torch
        ctx = self.sol.ctx
        h = self.dt
        n2, n1 = self.shape[1:]
        gc = torch.zeros((10, n2, n1), dtype=torch.float64, device=self.dev)
        grt = torch.zeros((n2, n1), dtype=torch.float64, device=self.dev)
        res = torch.as_tensor(np.ascontiguousarray(self.residuals), dtype=torch.float64, device=self.dev)
        rstride = self.nrec * 2 * 8
        uh, vh = self._new().zero_(), self._new().zero_()
        N = self.nsteps
        if self.nrec:
            S.sbpe_receiver_adjoint(ctx, res.data_ptr() + (N - 1) * rstride, [uh.data_ptr()], 1.0)
        for (cu, cv, ct, c0) in reversed(self.checkpoints):
            # recompute the segment's states
            k = min(self.K, N - c0)
            states = [(cu, cv, ct)]
            u, v, t = cu, cv, ct
            for s in range(k - 1):
                u, v = self._step(u, v, t)
                t = ct + (s + 1) * h
                states.append((u, v, t))
            for s in range(k - 1, -1, -1):
                n = c0 + s                      # reversing the step from y_n to y_{n+1}
                u, v, t = states[s]
                U, V, A = self._stages(u, v, t)
                ku = []
                kv = []
                for i in range(4):
                    a, b = self._new(), self._new()
                    self._lin([h * B_RK[i]], [uh], a)
                    self._lin([h * B_RK[i]], [vh], b)
                    ku.append(a)
                    kv.append(b)
                yu, yv = uh, vh               # y^_{n+1} carried into y^_n
                for i in range(3, -1, -1):
                    Yu = self._new()
                    self._apply(kv[i], 0.0, True, Yu)
                    Yv = ku[i]
                    S.sbpe_grad_accumulate(ctx, [kv[i].data_ptr()], [U[i].data_ptr()], [A[i].data_ptr()], 1.0,
                                           t + C_RK[i] * h, False, [gc.data_ptr()], [grt.data_ptr()])
                    if i > 0:
                        self._lin([1.0, h * C_RK[i]], [ku[i - 1], Yu], ku[i - 1])
                        self._lin([1.0, h * C_RK[i]], [kv[i - 1], Yv], kv[i - 1])
                    self._lin([1.0, 1.0], [yu, Yu], yu)
                    self._lin([1.0, 1.0], [yv, Yv], yv)
                uh, vh = yu, yv
                if n > 0 and self.nrec:
                    S.sbpe_receiver_adjoint(ctx, res.data_ptr() + (n - 1) * rstride, [uh.data_ptr()], 1.0)
            states = None
        g10, grho = S.sbpe_grad_to_physical(ctx, 0, gc.data_ptr(), grt.data_ptr())
        return grho, g10


def c10_grad_to_voigt(g10):
    """dJ/d(c11, c12, c16, c22, c26, c66) from dJ/dC10 for materials with minor
    symmetry (C10 = c11, c16, c16, c12, c66, c66, c26, c66, c26, c22)."""
    g = np.asarray(g10)
    return np.stack([g[0], g[3], g[1] + g[2], g[9], g[6] + g[8], g[4] + g[5] + g[7]])


def _torch_function():
    import torch

    class SeismicMisfit(torch.autograd.Function):
        """J(rho, C10) for a fixed problem layout; backward by the discrete adjoint.

        forward(rho, C10, spec, nsteps, dt, d_obs, checkpoint_every) with rho (n2, n1)
        and C10 (10, n2, n1) float64 CPU tensors; returns a 0-d tensor.
        """

        @staticmethod
        def forward(ctx, rho, C10, spec, nsteps, dt, d_obs=None, checkpoint_every=100):
            sp = dict(spec)
            blk = dict(sp['blocks'][0])
            blk['rho'] = rho.detach().cpu().numpy()
            blk['C10'] = C10.detach().cpu().numpy()
            sp['blocks'] = [blk]
            mg = MisfitGradient(sp, nsteps, dt, d_obs=d_obs, checkpoint_every=checkpoint_every)
            try:
                J = mg.forward()
                g_rho, g_c10 = mg.gradient()
            finally:
                mg.close()
            ctx.save_for_backward(torch.from_numpy(g_rho), torch.from_numpy(g_c10))
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            g_rho, g_c10 = ctx.saved_tensors
            return gJ * g_rho, gJ * g_c10, None, None, None, None, None

    return SeismicMisfit


_FN = None


def seismic_misfit(rho, C10, spec, nsteps, dt, d_obs=None, checkpoint_every=100):
    """torch-differentiable misfit J(rho, C10) (see ``MisfitGradient``)."""
    global _FN
    if _FN is None:
        _FN = _torch_function()
    return _FN.apply(rho, C10, spec, nsteps, dt, d_obs, checkpoint_every)
