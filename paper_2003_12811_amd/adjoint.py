"""Gradient of a receiver misfit with respect to rho and C by the discrete adjoint.

    J(rho, C) = 1/2 sum_{n=1..N} sum_r |S_r u_n - d_{n,r}|^2

for a forward run of N classical RK4 steps (Sec. 7.1) from rest.  The
gradient is the exact derivative of the discrete map (up to rounding):

* Forward: ``sbpe_advance`` with a checkpoint of (u, v, t) every
  ``checkpoint_every`` steps; J from the recorded receiver traces.
* Reverse, segment by segment from the last checkpoint: the segment's states
  are recomputed with ``sbpe_advance``, each step's stages with the stage form
  of RK4 (``sbpe_apply`` with the data at the stage times, ``sbpe_lincomb``
  for the stage combinations), then each step is reversed: with b = (1/6, 1/3, 1/3, 1/6), c = (0, 1/2, 1/2, 1), the
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
``SeismicMisfit`` exposes it as a ``torch.autograd.Function``: its forward
runs the forward pass (with checkpoints) only, its backward the adjoint.
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

    def _apply(self, x, t, homogeneous, out):
        S.sbpe_apply(self.sol.ctx, [x.data_ptr()], [out.data_ptr()], t, homogeneous)

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
        """(dJ/drho (n2, n1), dJ/dC10 (10, n2, n1)) after ``forward``.

        Per step, with stage slopes k_i = (V_i, A_i) and their adjoints
        (ku_i, kv_i), from the last stage to the first:
            ku_i = dt b_i uh + dt c_{i+1} Yu_{i+1},  kv_i = dt b_i vh + dt c_{i+1} ku_{i+1},
            Yu_i = L kv_i (scaled variables),
        then uh <- uh + sum_i Yu_i and vh <- vh + sum_i ku_i.  The states of a
        checkpoint segment are recomputed with ``sbpe_advance``; every work
        buffer is allocated once.  The buffers are laid out so that every
        pair of combinations is one ``sbpe_lincomb`` over both halves:
        stage i holds Z_i = (U_i, V_i, A_i) and M_i = (Yu_i, ku_i, kv_i), the
        adjoint state W = (uh, vh), so that
            (U_{i+1}, V_{i+1}) = (u, v) + dt c_{i+1} (V_i, A_i)  = Z_0[0:2] + dt c_{i+1} Z_i[1:3],
            (ku_i, kv_i) = dt b_i W + dt c_{i+1} M_{i+1}[0:2],
            W <- W + sum_i M_i[0:2].
        """
        torch = self.torch
        sol = self.sol
        ctx = sol.ctx
        h = self.dt
        n2, n1 = self.shape[1:]
        gc = torch.zeros((10, n2, n1), dtype=torch.float64, device=self.dev)
        grt = torch.zeros((n2, n1), dtype=torch.float64, device=self.dev)
        res = torch.as_tensor(np.ascontiguousarray(self.residuals), dtype=torch.float64, device=self.dev)
        rstride = self.nrec * 2 * 8
        N = self.nsteps
        triple = lambda: torch.empty((3,) + tuple(self.shape), dtype=self.tdt, device=self.dev)
        W = torch.zeros((2,) + tuple(self.shape), dtype=self.tdt, device=self.dev)
        Wn = torch.empty_like(W)
        Z = [triple() for _ in range(4)]
        M = [triple() for _ in range(4)]
        seg_u = [self._new() for _ in range(self.K)]
        seg_v = [self._new() for _ in range(self.K)]
        n2c = 2 * self.count
        lin = lambda coefs, xs, out: S.sbpe_lincomb(ctx, coefs, [x.data_ptr() for x in xs], out.data_ptr(), n2c)
        if self.nrec:
            S.sbpe_receiver_adjoint(ctx, res.data_ptr() + (N - 1) * rstride, [W[0].data_ptr()], 1.0)
        for (cu, cv, ct, c0) in reversed(self.checkpoints):
            k = min(self.K, N - c0)
            # the segment's states
            sol.set_state([cu], [cv], ct)
            seg_u[0].copy_(cu)
            seg_v[0].copy_(cv)
            for s_ in range(1, k):
                sol.advance(1, h)
                seg_u[s_].copy_(sol.u[0])
                seg_v[s_].copy_(sol.v[0])
            for s_ in range(k - 1, -1, -1):
                n = c0 + s_                     # reversing the step from y_n to y_{n+1}
                t = ct + s_ * h
                Z[0][0].copy_(seg_u[s_])
                Z[0][1].copy_(seg_v[s_])
                # stages of the step
                for i in range(4):
                    self._apply(Z[i][0], t + C_RK[i] * h, False, Z[i][2])
                    if i < 3:
                        lin([1.0, C_RK[i + 1] * h], [Z[0], Z[i][1]], Z[i + 1])
                # stage adjoints, last stage first
                for i in range(3, -1, -1):
                    if i == 3:
                        lin([h * B_RK[3]], [W], M[3][1])
                    else:
                        lin([h * B_RK[i], h * C_RK[i + 1]], [W, M[i + 1]], M[i][1])
                    self._apply(M[i][2], 0.0, True, M[i][0])
                    S.sbpe_grad_accumulate(ctx, [M[i][2].data_ptr()], [Z[i][0].data_ptr()], [Z[i][2].data_ptr()],
                                           1.0, t + C_RK[i] * h, False, [gc.data_ptr()], [grt.data_ptr()])
                lin([1.0, 1.0, 1.0, 1.0, 1.0], [W, M[3], M[2], M[1], M[0]], Wn)
                W, Wn = Wn, W
                if n > 0 and self.nrec:
                    S.sbpe_receiver_adjoint(ctx, res.data_ptr() + (n - 1) * rstride, [W[0].data_ptr()], 1.0)
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
            except Exception:
                mg.close()
                raise
            # the adjoint pass runs only when a gradient is asked for; the
            # forward run's checkpoints and residuals stay on the device until then
            ctx.mg = mg if (ctx.needs_input_grad[0] or ctx.needs_input_grad[1]) else None
            if ctx.mg is None:
                mg.close()
            return torch.tensor(J, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gJ):
            mg, ctx.mg = ctx.mg, None
            if mg is None:
                return None, None, None, None, None, None, None
            try:
                g_rho, g_c10 = mg.gradient()
            finally:
                mg.close()
            return (gJ * torch.from_numpy(g_rho), gJ * torch.from_numpy(g_c10), None, None, None, None, None)

    return SeismicMisfit


_FN = None


def seismic_misfit(rho, C10, spec, nsteps, dt, d_obs=None, checkpoint_every=100):
    """torch-differentiable misfit J(rho, C10) (see ``MisfitGradient``)."""
    global _FN
    if _FN is None:
        _FN = _torch_function()
    return _FN.apply(rho, C10, spec, nsteps, dt, d_obs, checkpoint_every)
