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

    def _lin(self, coefs, xs, out):
        S.sbpe_lincomb(self.sol.ctx, coefs, [x.data_ptr() for x in xs], out.data_ptr(), self.count)

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
        buffer is allocated once.
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
        new = self._new
        uh, vh, yu, yv = new().zero_(), new().zero_(), new(), new()
        U = [None] + [new() for _ in range(3)]
        V = [None] + [new() for _ in range(3)]
        A = [new() for _ in range(4)]
        ku = [new() for _ in range(4)]
        kv = [new() for _ in range(4)]
        Yu = [new() for _ in range(4)]
        seg_u = [new() for _ in range(self.K)]
        seg_v = [new() for _ in range(self.K)]
        lin = self._lin
        if self.nrec:
            S.sbpe_receiver_adjoint(ctx, res.data_ptr() + (N - 1) * rstride, [uh.data_ptr()], 1.0)
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
                u, v, t = seg_u[s_], seg_v[s_], ct + s_ * h
                # stages of the step
                U[0], V[0] = u, v
                for i in range(4):
                    self._apply(U[i], t + C_RK[i] * h, False, A[i])
                    if i < 3:
                        lin([1.0, C_RK[i + 1] * h], [u, V[i]], U[i + 1])
                        lin([1.0, C_RK[i + 1] * h], [v, A[i]], V[i + 1])
                # stage adjoints, last stage first
                for i in range(3, -1, -1):
                    if i == 3:
                        lin([h * B_RK[3]], [uh], ku[3])
                        lin([h * B_RK[3]], [vh], kv[3])
                    else:
                        lin([h * B_RK[i], h * C_RK[i + 1]], [uh, Yu[i + 1]], ku[i])
                        lin([h * B_RK[i], h * C_RK[i + 1]], [vh, ku[i + 1]], kv[i])
                    self._apply(kv[i], 0.0, True, Yu[i])
                    S.sbpe_grad_accumulate(ctx, [kv[i].data_ptr()], [U[i].data_ptr()], [A[i].data_ptr()], 1.0,
                                           t + C_RK[i] * h, False, [gc.data_ptr()], [grt.data_ptr()])
                lin([1.0, 1.0, 1.0, 1.0], [uh, Yu[3], Yu[2], Yu[1]], yu)
                lin([1.0, 1.0], [yu, Yu[0]], yu)
                lin([1.0, 1.0, 1.0, 1.0], [vh, ku[3], ku[2], ku[1]], yv)
                lin([1.0, 1.0], [yv, ku[0]], yv)
                uh, yu = yu, uh
                vh, yv = yv, vh
                if n > 0 and self.nrec:
                    S.sbpe_receiver_adjoint(ctx, res.data_ptr() + (n - 1) * rstride, [uh.data_ptr()], 1.0)
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
