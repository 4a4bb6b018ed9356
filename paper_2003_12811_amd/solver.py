"""Front end that drives the HIP library from a problem spec (see workloads.py).

PyTorch supplies device memory (state tensors) and the HIP stream; every
numerical step runs in libsbpe.so through the C ABI.
"""
import numpy as np

from . import sbpe as S


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError('no GPU visible: the HIP library needs an MI355X (gfx950)')
    return torch


class TorchMemory:
    """Device memory of a context from PyTorch's caching allocator: each
    allocation is a uint8 tensor kept alive until the library releases it."""

    def __init__(self, torch, device):
        self.torch, self.device, self.live = torch, device, {}

    def alloc(self, nbytes):
        t = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=self.device)
        p = t.data_ptr()
        self.live[p] = t
        return p

    def release(self, ptr):
        self.live.pop(ptr, None)

    def nbytes(self):
        return sum(t.numel() for t in self.live.values())


class Solver:
    """One context of the library built from a spec.  memory='torch' (the
    default) takes the context's device memory from PyTorch's allocator,
    memory='hip' lets the library call hipMalloc."""

    def __init__(self, spec, dtype='f64', device=0, beta=1.0, stream=None, tile_rows=0, memory='torch'):
        torch = _torch()
        self.torch = torch
        self.spec = spec
        self.tdtype = torch.float64 if dtype == 'f64' else torch.float32
        self.device = torch.device('cuda', device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.memory = TorchMemory(torch, self.device) if memory == 'torch' else None
        self.ctx = S.sbpe_create(device, stream.cuda_stream, S.F64 if dtype == 'f64' else S.F32,
                                 spec['order'], beta)
        try:
            if self.memory is not None:
                self._callbacks = S.sbpe_set_allocator(self.ctx, self.memory.alloc, self.memory.release)
            if tile_rows:
                S.sbpe_set_tile_rows(self.ctx, tile_rows)
            self._setup(spec)
        except Exception:
            S.sbpe_destroy(self.ctx)
            self.ctx = None
            raise
        self.shapes = [b['X1'].shape for b in spec['blocks']]
        self.nrec = sum(len(r[1]) for r in spec.get('receivers', []))
        self.u = [torch.zeros((2,) + s, dtype=self.tdtype, device=self.device) for s in self.shapes]
        self.v = [torch.zeros_like(x) for x in self.u]
        self.bound = False

    def _setup(self, spec):
        ctx = self.ctx
        op = spec.get('operator', 'narrow')
        if op != 'narrow':
            S.sbpe_set_operator(ctx, {'wide': S.OP_WIDE}[op])
        for b in spec['blocks']:
            bid = S.sbpe_add_block(ctx, b['X1'], b['X2'], b['rho'], b['C10'])
            for f, (kind, g, tfn, tp, U) in enumerate(b['bc']):
                if kind != S.BC_TRACTION:
                    S.sbpe_set_bc(ctx, bid, f, kind, U)
                if g is not None:
                    S.sbpe_set_bc_data(ctx, bid, f, g, tfn, tp)
            if b.get('forcing') is not None:
                F, tfn, tp = b['forcing']
                S.sbpe_set_forcing(ctx, bid, F, tfn, tp)
        # dissipative Robin terms V u_t: (block, face, V [2][2][nf])
        for (bid, f, V) in spec.get('dissipation', []):
            S.sbpe_set_bc_dissipation(ctx, bid, f, V)
        itfs = spec.get('interfaces', [])
        for (a, fa, bb, fb, rev) in itfs:
            S.sbpe_connect(ctx, a, fa, bb, fb, rev)
        # jump data, given on side a of each interface: V = u_a - u_b, Theta = tau_a + tau_b
        for (k, V, Th, tfn, tp) in spec.get('interface_data', []):
            S.sbpe_set_interface_data(ctx, itfs[k][0], itfs[k][1], V, Th, tfn, tp)
        for (bid, x1, x2, f1, f2, amp, fp, t0) in spec.get('sources', []):
            S.sbpe_add_source(ctx, bid, x1, x2, f1, f2, amp, fp, t0)
        for (bid, x1, x2) in spec.get('receivers', []):
            S.sbpe_add_receivers(ctx, bid, x1, x2)
        S.sbpe_finalize(ctx)

    # ------------------------------------------------------------ calls
    def set_frame_loop(self, groups):
        """Frame groups per frame workgroup of a one-launch sweep (launch shape only)."""
        S.sbpe_set_frame_loop(self.ctx, groups)

    def dt_cfl(self, cfl):
        return S.sbpe_dt_cfl(self.ctx, cfl)

    def set_state(self, u=None, v=None, t=0.0):
        """Copy host (NumPy) or device initial data into the state and bind it."""
        torch = self.torch
        for k in range(len(self.shapes)):
            for dst, src in ((self.u[k], u), (self.v[k], v)):
                if src is None:
                    dst.zero_()
                else:
                    dst.copy_(torch.as_tensor(np.asarray(src[k]) if not torch.is_tensor(src[k]) else src[k]))
        S.sbpe_bind_state(self.ctx, [x.data_ptr() for x in self.u], [x.data_ptr() for x in self.v], t)
        self.bound = True

    def advance(self, nsteps, dt):
        S.sbpe_advance(self.ctx, nsteps, dt)

    def reserve(self, nsteps):
        """Size the time-function table and the receiver record for advance
        calls of up to nsteps steps, so that they allocate nothing."""
        S.sbpe_reserve_steps(self.ctx, nsteps)

    def apply(self, us, t=0.0, homogeneous=False, out=None):
        """a = rho~^{-1}(L u + data(t)) for device tensors us (one per block)."""
        torch = self.torch
        us = [torch.as_tensor(x, dtype=self.tdtype, device=self.device).contiguous() for x in us]
        if out is None:
            out = [torch.empty_like(x) for x in us]
        S.sbpe_apply(self.ctx, [x.data_ptr() for x in us], [x.data_ptr() for x in out], t, homogeneous)
        self._keep = us
        return out

    def energy(self):
        return S.sbpe_energy(self.ctx)

    def time(self):
        return S.sbpe_get_time(self.ctx)

    def receivers(self):
        return S.sbpe_read_receivers(self.ctx, self.nrec)

    def synchronize(self):
        S.sbpe_synchronize(self.ctx)

    def state_numpy(self):
        self.synchronize()
        return ([x.double().cpu().numpy() for x in self.u], [x.double().cpu().numpy() for x in self.v])

    def close(self):
        if self.ctx is not None:
            S.sbpe_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
