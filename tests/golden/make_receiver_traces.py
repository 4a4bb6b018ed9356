"""Write the oracle's receiver traces of the single-block workload at a reduced
size, the stored expected values of tests/test_gpu_runs.py.

Only the oracle runs here (plain NumPy/SciPy FP64 literal RK4, Sec. 7.1); the
inputs come from the seeded workload recipe.  The block is 129^2 (1/8 of the
1025^2 spacing) and the run spans the same time as 2000 steps at 1025^2:
the Ricker pulse (10 Hz, t0 = 0.1) is emitted and reaches the surface
receivers.  The time step is fixed here (not recomputed by either side) so
that library and oracle step identically.

    python tests/golden/make_receiver_traces.py     # writes c2_n129_receivers.npz
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

N = 129
NSTEPS = 250
DT = 1.1381706896233274e-03     # 8 x the CFL-0.5 step of the 1025^2 workload, below this block's limit
OUT = os.path.join(HERE, 'c2_n129_receivers.npz')


def main():
    from paper_2003_12811_amd import workloads as W
    from oracle import spec as OS, timestep as T
    spec = W.spec_c2(n=N)
    P = OS.build(spec)
    assert DT <= T.dt_cfl(P, 0.5), 'time step beyond the CFL 0.5 estimate'
    u = [np.zeros((2, N, N))]
    v = [np.zeros((2, N, N))]
    t, rec = 0.0, []
    t0 = time.time()
    for _ in range(NSTEPS):
        u, v = T.rk4_step(P, u, v, t, DT)
        t += DT
        rec.append(OS.receivers(spec, u))
    rec = np.array(rec)
    np.savez(OUT, receivers=rec, n=N, nsteps=NSTEPS, dt=DT)
    print('wrote %s: %s, max |u| %.3e, %.1f s' % (OUT, rec.shape, np.abs(rec).max(), time.time() - t0))


if __name__ == '__main__':
    main()
