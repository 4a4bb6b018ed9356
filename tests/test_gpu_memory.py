"""Device memory from the caller (sbpe_set_allocator): a context whose memory
comes from PyTorch's caching allocator computes bit for bit what a context
with its own hipMalloc'ed memory computes, reports exactly the bytes it took,
and gives every byte back when it is destroyed."""
import numpy as np
import pytest

from paper_2003_12811_amd import sbpe as S
from paper_2003_12811_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_torch_memory_matches_hip_memory():
    import torch
    from paper_2003_12811_amd.solver import Solver
    spec = W.spec_c2(n=201, nrec=8)
    out = {}
    for mem in ('torch', 'hip'):
        sol = Solver(spec, 'f64', memory=mem)
        dt = sol.dt_cfl(0.5)
        sol.set_state(None, None, 0.0)
        sol.advance(30, dt)              # grows the receiver record and the time table
        sol.advance(45, dt)
        u, v = sol.state_numpy()
        out[mem] = (u[0], v[0], sol.receivers())
        held, peak = S.sbpe_device_bytes(sol.ctx)
        if mem == 'torch':
            assert held == sol.memory.nbytes() and held > 0
            live = sol.memory
        sol.close()
    assert live.live == {}
    for a, b in zip(out['torch'], out['hip']):
        assert np.array_equal(a, b)
    torch.cuda.synchronize()


def test_allocation_failure_is_reported():
    import torch
    from paper_2003_12811_amd.solver import TorchMemory
    spec = W.spec_c2(n=129, nrec=4)
    mem = TorchMemory(torch, torch.device('cuda', 0))
    budget = [200000]

    def alloc(nb):                       # refuses once the budget is spent
        if nb > budget[0]:
            return 0
        budget[0] -= nb
        return mem.alloc(nb)

    ctx = S.sbpe_create(0, torch.cuda.current_stream().cuda_stream, S.F64, 4, 1.0)
    try:
        cbs = S.sbpe_set_allocator(ctx, alloc, mem.release)
        b = spec['blocks'][0]
        S.sbpe_add_block(ctx, b['X1'], b['X2'], b['rho'], b['C10'])
        with pytest.raises(S.SbpeError) as e:
            S.sbpe_finalize(ctx)
        assert e.value.code == S.ENOMEM
    finally:
        S.sbpe_destroy(ctx)
    assert mem.live == {}
    del cbs
