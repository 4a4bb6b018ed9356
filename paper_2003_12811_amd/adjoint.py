"""Gradient of a receiver misfit with respect to rho and C by the discrete adjoint.

    J(rho, C) = 1/2 sum_{n=1..N} sum_r |S_r u_n - d_{n,r}|^2

for a forward run of N classical RK4 steps (Sec. 7.1) from rest.  The
gradient is the exact derivative of the discrete map (up to rounding):

* Forward: ``sbpe_advance`` with a checkpoint of (u, v, t) every
  ``checkpoint_every`` steps; J from the recorded receiver traces.  When the
  stage fields of every step fit in device memory (``keep_stages``), the
  forward run advances one step at a time and keeps each step's stage
  displacements U_i and slopes A_i instead (nine fields per step: 76 GB for
  2000 steps at 513^2 in FP64, well inside one GPU's HBM), so the reverse
  pass recomputes nothing.
* Reverse, segment by segment from the last checkpoint: the segment's steps
  are recomputed with ``sbpe_advance`` one step at a time, keeping each
  step's stage displacements U_i and stage values A_i (``sbpe_rk4_stages``
  rebuilds them from the step's end states and the slopes its sweeps
  leave).  Then each step is reversed.  With b = (1/6, 1/3, 1/3, 1/6) and c = (0, 1/2, 1/2, 1), the
  stage-slope adjoints of classical RK4 are k^_{5-j} = dt b_{5-j} Y^_j, with
  Y^_j the stages of one RK4 step of y' = A^T y from the adjoint state y^,
  which that step advances.  Because H L is symmetric (the energy analysis of
  Sec. 5), in the variables y^ = y / (H rho~) L^T = L, so A^T = s A s with
  s (u, v) = (v, u): the adjoint step is one forward step of the homogeneous
  problem on the swapped state (v^, u^), which ``sbpe_advance`` on a data-free
  context performs with its two sweeps.  The stage displacements of that step
  (rebuilt from ``sbpe_stage_slopes``) are the velocity parts of the stage
  adjoints, which ``sbpe_grad_accumulate_rk4`` pairs with the forward U_i and
  A_i of the step; the receiver residuals enter through
  ``sbpe_receiver_adjoint``.
* ``sbpe_grad_to_physical`` maps the gradients with respect to the stored
  c = F J C F and rho~ = J rho to C (C10 layout) and rho.

``MisfitGradient`` wraps one forward/adjoint pair for a fixed time step (the
step must not depend on the parameters being differentiated), and
``SeismicMisfit`` exposes it as a ``torch.autograd.Function``: its forward
runs the forward pass (with checkpoints) only, its backward the adjoint.
"""
import ctypes

import numpy as np

from . import sbpe as S
from .solver import Solver

B_RK = (1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0)
C_RK = (0.0, 0.5, 0.5, 1.0)


def homogeneous_spec(spec):
    """The problem of `spec` with every data term removed (boundary data,
    forcing, sources, receivers, interface jump data): the same operator."""
    sp = {k: v for k, v in spec.items() if k not in ('sources', 'receivers', 'interface_data')}
    blocks = []
    for b in spec['blocks']:
        nb = {k: v for k, v in b.items() if k != 'forcing'}
        nb['bc'] = [(kind, None, None, None, U) for (kind, g, tfn, tp, U) in b['bc']]
        blocks.append(nb)
    sp['blocks'] = blocks
    return sp


class MisfitGradient:
    """Forward run, misfit and adjoint gradient of one single-block problem.

    spec: a problem specification (see workloads.py) with receivers; its
    block's 'rho' and 'C10' are the parameters.  d_obs: observed traces
    (nsteps, nrec, 2) or None (then J = 1/2 sum |S u|^2).
    """

    # share of the free device memory the kept stage fields may take
    KEEP_FRACTION = 0.5

    def __init__(self, spec, nsteps, dt, d_obs=None, dtype='f64', device=0, checkpoint_every=100,
                 keep_stages='auto'):
        """keep_stages: True (keep every step's stage fields in the forward
        run; raises MemoryError if they would take more than KEEP_FRACTION of
        the free device memory), False (checkpoints, the reverse pass reruns
        each segment) or 'auto' (keep them when they fit)."""
        import torch
        if len(spec['blocks']) != 1:
            raise ValueError('single-block problems only')
        if keep_stages not in (True, False, 'auto'):
            raise ValueError('keep_stages must be True, False or "auto"')
        self.torch = torch
        self.spec, self.nsteps, self.dt = spec, nsteps, dt
        self.K = max(1, int(checkpoint_every))
        self.keep_stages = keep_stages
        self.stages = None
        self.dtype = dtype
        self.sol = Solver(spec, dtype, device=device)
        self.dev = self.sol.device
        self.tdt = self.sol.tdtype
        self.shape = self.sol.u[0].shape
        self.count = self.sol.u[0].numel()
        self.nrec = self.sol.nrec
        self.d_obs = None if d_obs is None else np.asarray(d_obs, dtype=float)

    def close(self):
        self.stages = None
        self.sol.close()

    # ------------------------------------------------------------ helpers
    def _apply(self, x, t, homogeneous, out):
        S.sbpe_apply(self.sol.ctx, [x.data_ptr()], [out.data_ptr()], t, homogeneous)

    # ------------------------------------------------------------ forward
    def stage_bytes(self):
        """Device bytes of the stage fields kept by a forward run with
        keep_stages (nine state-sized fields per step)."""
        return self.nsteps * 9 * self.count * self.sol.u[0].element_size()

    def _keep(self):
        if self.keep_stages is False:
            return False
        free, _ = self.torch.cuda.mem_get_info(self.dev)
        fits = self.stage_bytes() <= self.KEEP_FRACTION * free
        if self.keep_stages is True and not fits:
            raise MemoryError('kept stage fields need %d bytes, %d free' % (self.stage_bytes(), free))
        return fits

    def forward(self, for_gradient=True):
        """Run from rest; returns J (and keeps the traces).  With
        for_gradient and kept stages, every step's nine stage fields are
        recorded for the reverse pass; otherwise (u, v, t) is checkpointed
        every checkpoint_every steps."""
        torch = self.torch
        sol = self.sol
        sol.set_state(None, None, 0.0)
        self.checkpoints = []
        self.stages = None
        if for_gradient and self._keep():
            self._forward_keep()
        else:
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

    def _forward_keep(self):
        """One step at a time from rest: the step's start state is copied
        into its record, the step is taken, and ``sbpe_rk4_stages`` fills in
        the stage displacements U_2..U_4 and slopes A_1..A_4 from the end
        state and the sweeps' slopes a1, a2."""
        torch = self.torch
        sol, ctx, h, cnt = self.sol, self.sol.ctx, self.dt, self.count
        N = self.nsteps
        st = torch.empty((N, 9) + tuple(self.shape), dtype=self.tdt, device=self.dev)
        X = torch.zeros((2,) + tuple(self.shape), dtype=self.tdt, device=self.dev)
        S.sbpe_bind_state(ctx, [X[0].data_ptr()], [X[1].data_ptr()], 0.0)
        sol.reserve(N)
        a1f, a2f = S.sbpe_stage_slopes(ctx, 0)
        L, A, chk = S.lib(), S.ptr_array, S.check
        one = np.ones(1)
        one_p = one.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        X_p = A([X.data_ptr()])
        x0, x1 = X[0].data_ptr(), X[1].data_ptr()
        step_bytes = st[0].numel() * st.element_size()
        field_bytes = st[0, 0].numel() * st.element_size()
        base = st.data_ptr()
        for n in range(N):
            e0 = base + n * step_bytes
            e_out = A([e0 + i * field_bytes for i in range(2, 9)])
            chk(ctx, L.sbpe_lincomb(ctx, 1, one_p, X_p, e0, 2 * cnt))
            chk(ctx, L.sbpe_advance(ctx, 1, h))
            chk(ctx, L.sbpe_rk4_stages(ctx, e0, e0 + field_bytes, x0, x1, a1f, a2f, h, e_out, cnt))
        self.stages = st
        self._keep_state = X

    # ------------------------------------------------------------ reverse
    def gradient(self):
        """(dJ/drho (n2, n1), dJ/dC10 (10, n2, n1)) after ``forward``.

        Forward stages of step n from (u, v) at time t: the segment is rerun
        with ``sbpe_advance`` one step at a time, and ``sbpe_rk4_stages``
        rebuilds each step's stage displacements U_1..U_4 and slopes
        A_1..A_4 from its end states and the slopes a1, a2 the sweeps leave
        (``sbpe_stage_slopes``); a step's nine fields (U_1, v, U_2, U_3, U_4,
        A_1..A_4) are kept until it is reversed.  Adjoint state: (u^, v^) is
        held swapped, as the bound state (u', v') = (v^, u^) of a data-free
        context.  Reversing step n:
            keep (u', v'),  one homogeneous RK4 step of (u', v'),
            U'_2, U'_3, U'_4 from ``sbpe_rk4_stages`` of that step,
            gradient += the four stage terms with z_i = U'_{5-i}, alpha_i = dt b_i,
        then the receiver residuals of step n - 1 are added to u^.  Memory:
        nine fields per step of a segment (checkpoint_every steps) and two
        contexts.
        """
        torch = self.torch
        sol = self.sol
        ctx = sol.ctx
        h = self.dt
        n2, n1 = self.shape[1:]
        shape = tuple(self.shape)
        gc = torch.zeros((10, n2, n1), dtype=torch.float64, device=self.dev)
        grt = torch.zeros((n2, n1), dtype=torch.float64, device=self.dev)
        res = torch.as_tensor(np.ascontiguousarray(self.residuals), dtype=torch.float64, device=self.dev)
        rstride = self.nrec * 2 * 8
        N = self.nsteps
        cnt = self.count
        kept = self.stages is not None
        new = lambda *lead: torch.empty(lead + shape, dtype=self.tdt, device=self.dev)
        if kept:
            # the forward run's records: one segment of all N steps
            seg = self.stages
            segments = [(None, None, 0.0, 0)]
            K = N
        else:
            seg = new(self.K, 9)                    # U1, v, U2, U3, U4, A1, A2, A3, A4 of each step
            segments = list(reversed(self.checkpoints))
            K = self.K
        X = new(2)                                  # forward state (u, v)
        Y = new(2)                                  # adjoint state (u', v') = (v^, u^)
        P = new(5)                                  # U'_1 = u', v', U'_2, U'_3, U'_4
        a1f, a2f = S.sbpe_stage_slopes(ctx, 0)
        adj = Solver(homogeneous_spec(self.spec), self.dtype, device=self.dev.index)
        try:
            actx = adj.ctx
            Y.zero_()
            S.sbpe_bind_state(actx, [Y[0].data_ptr()], [Y[1].data_ptr()], 0.0)
            a1p, a2p = S.sbpe_stage_slopes(actx, 0)
            # the per-step calls go straight to the library with their
            # arguments converted once: a step's kernels take tens of
            # microseconds, the argument marshalling of the wrappers as long
            L, A = S.lib(), S.ptr_array
            one = np.ones(1)
            one_p = one.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            alphas = np.array([h * b for b in B_RK])
            alphas_p = alphas.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            X_p, Y_p = A([X.data_ptr()]), A([Y.data_ptr()])
            step_bytes = seg[0].numel() * seg.element_size()
            field_bytes = seg[0, 0].numel() * seg.element_size()
            base = seg.data_ptr()

            def rec(s_):
                """pointers of step s_'s record: U1, v, the seven stage outputs,
                the four stage displacements and the four slopes"""
                e = base + s_ * step_bytes
                f = [e + i * field_bytes for i in range(9)]
                return f[0], f[1], A(f[2:9]), A([f[i] for i in (0, 2, 3, 4)]), A([f[i] for i in (5, 6, 7, 8)])

            adj_out = A([P[i].data_ptr() for i in (2, 3, 4)] + [None] * 4)
            z_p = A([P[i].data_ptr() for i in (4, 3, 2, 0)])
            gc_p, grt_p, y1_p = A([gc.data_ptr()]), A([grt.data_ptr()]), A([Y[1].data_ptr()])
            pP, p0, p1 = P.data_ptr(), P[0].data_ptr(), P[1].data_ptr()
            x0, x1 = X[0].data_ptr(), X[1].data_ptr()
            r0 = res.data_ptr()
            chk = S.check
            if self.nrec:
                chk(ctx, L.sbpe_receiver_adjoint(ctx, r0 + (N - 1) * rstride, y1_p, 1.0))
            for (cu, cv, ct, c0) in segments:
                k = min(K, N - c0)
                if not kept:
                    # the segment's forward stages
                    X[0].copy_(cu)
                    X[1].copy_(cv)
                    S.sbpe_bind_state(ctx, [x0], [x1], ct)
                    for s_ in range(k):
                        e0, e1, e_out = rec(s_)[:3]
                        chk(ctx, L.sbpe_lincomb(ctx, 1, one_p, X_p, e0, 2 * cnt))
                        chk(ctx, L.sbpe_advance(ctx, 1, h))
                        chk(ctx, L.sbpe_rk4_stages(ctx, e0, e1, x0, x1, a1f, a2f, h, e_out, cnt))
                # reversed steps, last first
                for s_ in range(k - 1, -1, -1):
                    n = c0 + s_                     # reversing the step from y_n to y_{n+1}
                    t = ct + s_ * h
                    y_p, a_p = rec(s_)[3:]
                    chk(ctx, L.sbpe_lincomb(ctx, 1, one_p, Y_p, pP, 2 * cnt))
                    chk(actx, L.sbpe_advance(actx, 1, h))
                    chk(ctx, L.sbpe_rk4_stages(ctx, p0, p1, None, None, a1p, a2p, h, adj_out, cnt))
                    chk(ctx, L.sbpe_grad_accumulate_rk4(ctx, z_p, y_p, a_p, alphas_p, t, h, 0, gc_p, grt_p))
                    if n > 0 and self.nrec:
                        chk(ctx, L.sbpe_receiver_adjoint(ctx, r0 + (n - 1) * rstride, y1_p, 1.0))
            g10, grho = S.sbpe_grad_to_physical(ctx, 0, gc.data_ptr(), grt.data_ptr())
        finally:
            adj.close()
            # the forward context's own state buffers again
            S.sbpe_bind_state(ctx, [sol.u[0].data_ptr()], [sol.v[0].data_ptr()], N * h)
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
            grad = ctx.needs_input_grad[0] or ctx.needs_input_grad[1]
            try:
                J = mg.forward(for_gradient=grad)
            except Exception:
                mg.close()
                raise
            # the adjoint pass runs only when a gradient is asked for; the
            # forward run's checkpoints and residuals stay on the device until then
            ctx.mg = mg if grad else None
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
