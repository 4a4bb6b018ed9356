#!/usr/bin/env python3
"""Throughput of the RK4-advanced SBP-SAT anisotropic elastic solver on one MI355X.

Workload of the headline line (the largest configuration that fits one GPU,
at the paper's precision): 2 x 2 conforming curvilinear blocks of 2049 x 2049
points (16.8 M points) of one smooth global map, smooth random SPD stiffness
and density with a contrast of 3 between neighbouring blocks, interface SATs
between the blocks, traction on the top and left outer faces, displacement on
the bottom and right ones, a 10 Hz Ricker point force and 16 surface
receivers; 4th-order operators, classical RK4 at CFL 0.5, FP64.  A step is
one full RK4 step (four right-hand-side evaluations fused into two sweeps
over the grid, sources, receivers).  Inputs are resident in HBM and every
per-call table is sized before timing starts.  The launch shape (tile height,
frame groups per frame workgroup) is picked by timing candidates first; it
does not change the results.  The headline's timed steps run with HIP events
around every launch on the launch's own stream, which give the launch
durations of the roofline (at 1.7 ms per step they cost well under 1 %).

Prints one JSON line on stdout; progress goes to stderr.  Beside the headline:
the 1025^2 single-block workload in FP64 and FP32 with the plain operator
apply, the headline workload in FP32, the 1025^2 workload with the
wide-stencil operator, a served stream of shots (continuous batching against
sequential plain solves, p50/p99 latency), the misfit gradient, and the
oracle timed on the host.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# algorithmic words per updated point of each kernel launch (each field read or
# written once per sweep):
#   first sweep : u, v in (4) + 11 coefficient fields + a1, a2 out (4)
#   second sweep: a1, a2 in (4) + 11 coefficients + u, v in (4) + u, v out (4)
#   apply       : u in (2) + 11 coefficients + a out (2)
WORDS = {'interior_rk1': 19, 'interior_rk2': 23, 'interior_apply': 15}
# the same launches counted in the unit of one right-hand-side apply (2 words
# in, 11 coefficient words, 2 words out = 15 words per point): each RK sweep
# applies the operator to two fields
APPLY_WORDS = 15
APPLIES = {'interior_rk1': 2, 'interior_rk2': 2, 'interior_apply': 1}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)
# per workload; ignored once the kernel source or the tile height differs
TRAFFIC_PROFILES = {'c2_1025': os.path.join(ROOT, 'profiles', 'hbm_traffic_c2_1025.md'),
                    'c2_2049': os.path.join(ROOT, 'profiles', 'hbm_traffic_c2_2049.md'),
                    'c3_2049': os.path.join(ROOT, 'profiles', 'hbm_traffic_c3_2049.md')}


def roofline(kind, ms, points, wbytes, traffic_key=None, tile_rows=None, profile=None):
    """HBM roofline of one launch kind.  `achieved` counts the launch's work
    in right-hand-side applies of 15 words per point; `achieved_own_bytes`
    counts the words the fused launch itself must move (fewer: a sweep shares
    the coefficient reads of its two applies)."""
    byts = APPLIES[kind] * APPLY_WORDS * wbytes * points
    own = WORDS[kind] * wbytes * points
    gbs = byts / (ms * 1e-3) / 1e9
    gbs_own = own / (ms * 1e-3) / 1e9
    traffic = None
    if traffic_key is not None and profile is not None:
        from paper_2003_12811_amd import profiling
        t = profiling.read_traffic(TRAFFIC_PROFILES[profile], tile_rows=tile_rows or 10)
        traffic = t.get(traffic_key) if t else None
    return {"bound": "hbm", "kernel": kind, "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
            "avg_ms": round(ms, 5), "bytes_per_launch": byts,
            "achieved_own_bytes": round(gbs_own, 1), "frac_own_bytes": round(gbs_own / PEAK_HBM_GBS, 4),
            "own_bytes_per_launch": own,
            "traffic_over_own_bytes": round(traffic / own, 4) if traffic else None}


TILE_CANDIDATES = (10, 14, 16, 18, 20, 24)
FRAME_LOOP_CANDIDATES = (1, 2, 3, 4)


def tune_launch(spec, dtype, tiles=TILE_CANDIDATES, loops=FRAME_LOOP_CANDIDATES, steps=60):
    """Launch shape (interior tile height, frame groups per frame workgroup)
    with the shortest step on this workload, timed before the benchmark; the
    results do not depend on it.  The default shape (10, 1) is kept unless
    another is more than 1 % faster."""
    import torch
    from paper_2003_12811_amd.solver import Solver
    times = {}
    for rows in tiles:
        sol = Solver(spec, dtype, tile_rows=rows)
        dt = sol.dt_cfl(spec.get('cfl', 0.5))
        sol.set_state(None, None, 0.0)
        sol.reserve(len(loops) * (10 + steps))
        for fl in loops:
            sol.set_frame_loop(fl)
            sol.advance(10, dt)
            sol.synchronize()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol.advance(steps, dt)
            sol.synchronize()
            torch.cuda.synchronize()
            times[(rows, fl)] = 1e3 * (time.perf_counter() - t0) / steps
        sol.close()
    best = (tiles[0], loops[0])
    for key, ms in times.items():
        if ms < 0.99 * times[best]:
            best = key
    table = {'%dx%d' % k: round(v, 4) for k, v in times.items()}
    log('  launch shapes (tile rows x frame groups) %s -> %dx%d' % (table, best[0], best[1]))
    return best, table


def run_gpu(spec, dtype, steps, warmup, apply_reps=0, shape=(0, 0), events_in_timed=False):
    """Advance the workload: warmup steps, then `steps` timed steps.  With
    events_in_timed the timed steps carry HIP events around every launch and
    give the launch durations too; otherwise the same number of steps is run
    again with events (at 1025^2 the events lengthen a step by 12-19 %)."""
    import torch
    from paper_2003_12811_amd import sbpe as S
    from paper_2003_12811_amd.solver import Solver
    sol = Solver(spec, dtype, tile_rows=shape[0])
    if shape[1]:
        sol.set_frame_loop(shape[1])
    dt = sol.dt_cfl(spec.get('cfl', 0.5))
    sol.set_state(None, None, 0.0)
    # every table the advance calls use is sized here, outside the timed region
    sol.reserve(warmup + 2 * steps)
    plan = S.sbpe_plan_info(sol.ctx)
    npts = sum(b['X1'].size for b in spec['blocks'])
    sol.advance(warmup, dt)
    sol.synchronize()
    torch.cuda.synchronize()
    if events_in_timed:
        S.sbpe_set_kernel_timing(sol.ctx, 1)
        S.sbpe_get_kernel_timing(sol.ctx)
    t0 = time.perf_counter()
    sol.advance(steps, dt)
    sol.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    if events_in_timed:
        kt = S.sbpe_get_kernel_timing(sol.ctx)
        ev_ms = 1e3 * wall / steps
    else:
        S.sbpe_set_kernel_timing(sol.ctx, 1)
        S.sbpe_get_kernel_timing(sol.ctx)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        sol.advance(steps, dt)
        sol.synchronize()
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        kt = S.sbpe_get_kernel_timing(sol.ctx)
        ev_ms = 1e3 * (t3 - t2) / steps
    res = dict(dtype=dtype, points=npts, steps=steps, wall_s=wall, ms_per_step=1e3 * wall / steps,
               ms_per_step_with_events=ev_ms,
               updates_per_s=npts * steps / wall, dt=dt, kernels=kt, plan=plan)
    if apply_reps:
        u = [torch.zeros((2,) + b['X1'].shape, dtype=sol.tdtype, device=sol.device) for b in spec['blocks']]
        for x in u:
            x.normal_()
        out = [torch.empty_like(x) for x in u]
        sol.apply(u, 0.0, False, out)
        S.sbpe_get_kernel_timing(sol.ctx)
        for _ in range(apply_reps):
            sol.apply(u, 0.0, False, out)
        res['apply_kernels'] = S.sbpe_get_kernel_timing(sol.ctx)
    S.sbpe_set_kernel_timing(sol.ctx, 0)
    sol.close()
    return res


def gradient_timing(n=513, nsteps=2000, ckpt=100):
    """Wall times of the differentiation workload (FP64): the forward run
    alone (J only, checkpoints), the forward run that keeps every step's
    stage fields for the adjoint, and the reverse pass (the gradient)."""
    import torch
    from paper_2003_12811_amd import adjoint as ADJ
    from paper_2003_12811_amd import workloads as W
    from paper_2003_12811_amd.solver import Solver
    spec, spec_obs = W.spec_c5(n=n), W.spec_c5(n=n, perturbed=True)
    s = Solver(spec, 'f64')
    dt = s.dt_cfl(0.5)
    s.close()
    obs = ADJ.MisfitGradient(spec_obs, nsteps, dt)
    obs.forward(for_gradient=False)
    d_obs = obs.traces.copy()
    obs.close()
    mg = ADJ.MisfitGradient(spec, nsteps, dt, d_obs=d_obs, checkpoint_every=ckpt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J0 = mg.forward(for_gradient=False)
    t1 = time.perf_counter()
    J = mg.forward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kept = mg.stages is not None
    g_rho, g_c10 = mg.gradient()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    mg.close()
    fwd, fwd_keep, rev = t1 - t0, t2 - t1, t3 - t2
    return {"workload": "%dx%d block, %d RK4 steps, 100 receivers, misfit against the +5%% blob model, FP64, %s"
                        % (n, n, nsteps, "every step's stage fields kept (%.0f GB)" % (mg.stage_bytes() / 1e9)
                           if kept else "checkpoints every %d steps" % ckpt),
            "J": J, "J_rel_diff_forward_forms": abs(J - J0) / J0,
            "forward_s": fwd, "forward_keep_s": fwd_keep, "gradient_s": rev,
            "gradient_over_forward": rev / fwd, "value_and_gradient_over_forward": (fwd_keep + rev) / fwd,
            "forward_updates_per_s": n * n * nsteps / fwd}


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device='cuda')
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log('copy probe: 3 copies of %d MiB' % mib)
    del src, dst


def copy_bandwidth(mib=1024, reps=10):
    """Device-to-device copy bandwidth (bytes read + written / time) of a
    plain torch copy of mib MiB, timed with events on the current stream."""
    import torch
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device='cuda')
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


def swept_points(plan):
    """Points whose update the timed 'interior' launch performs: a one-launch
    sweep also updates the frame points."""
    return plan['interior_points'] + (plan['frame_points'] if plan['fused_sweep'] else 0)


def dominant(res):
    best, kind = -1.0, None
    for k, (ms, cnt) in res['kernels'].items():
        if k.startswith('interior') and ms * cnt > best:
            best, kind = ms * cnt, k
    return kind


def c1_latency(reps=5):
    """Time to solution of the plain-method workload: the 65^2 Cartesian block
    with constant anisotropic C, manufactured solution and traction SATs,
    advanced from t = 0 to t = 0.5 at CFL 0.5 in FP64 (setup, then the solve
    from resident inputs; median of reps solves after one warm-up solve)."""
    import numpy as np
    import torch
    from paper_2003_12811_amd import workloads as W
    from paper_2003_12811_amd.solver import Solver
    spec = W.spec_c1(n=65)
    t0 = time.perf_counter()
    sol = Solver(spec, 'f64')
    setup_s = time.perf_counter() - t0
    nsteps = int(np.ceil(spec['T'] / sol.dt_cfl(spec['cfl']) - 1e-12))
    dt = spec['T'] / nsteps
    u0 = spec['mms']['u']
    sol.reserve(nsteps)
    times = []
    for k in range(reps + 1):
        sol.set_state([u0], None, 0.0)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sol.advance(nsteps, dt)
        sol.synchronize()
        times.append(time.perf_counter() - t1)
    ug, _ = sol.state_numpy()
    sol.close()
    exact = u0 * np.cos(spec['mms']['omega'] * spec['T'])
    solve = sorted(times[1:])[len(times[1:]) // 2]
    return {"workload": "65x65 Cartesian block, constant anisotropic C, manufactured solution, traction SATs "
                        "with analytic data and forcing, 4th order, RK4 at CFL 0.5 to t = 0.5, FP64",
            "steps": nsteps, "setup_s": round(setup_s, 4), "solve_ms": round(1e3 * solve, 3),
            "ms_per_step": round(1e3 * solve / nsteps, 4),
            "rel_l2_error_vs_exact": float(np.linalg.norm(ug[0] - exact) / np.linalg.norm(exact))}


def bench_3d(n=97, steps=20, dtype='f64'):
    """One curvilinear 3-D block of n^3 points (random major-symmetric
    stiffness, displacement on x3 = 0 and traction elsewhere, a body force),
    4th order, RK4 at CFL 0.5: time per step of the 3-D point kernel."""
    import numpy as np
    import torch
    from paper_2003_12811_amd import sbpe as S
    from paper_2003_12811_amd import workloads as W
    X = W.grid3(n, n, n)
    rho, C = W.random_material3(X[0].shape, 0)
    ctx = S.sbpe3_create(0, torch.cuda.current_stream().cuda_stream, S.F64 if dtype == 'f64' else S.F32, 4)
    try:
        S.sbpe3_set_block(ctx, *X, rho, C)
        S.sbpe3_set_bc(ctx, 4, S.BC_DISPLACEMENT)
        F = np.zeros((3,) + X[0].shape)
        F[2] = np.exp(-((X[0] - 0.5) ** 2 + (X[1] - 0.5) ** 2 + (X[2] - 0.7) ** 2) / 0.01)
        S.sbpe3_set_forcing(ctx, F, S.TIME_RICKER, (10.0, 0.1))
        S.sbpe3_finalize(ctx)
        dt = S.sbpe3_dt_cfl(ctx, 0.5)
        tdt = torch.float64 if dtype == 'f64' else torch.float32
        u = torch.zeros((3,) + X[0].shape, dtype=tdt, device='cuda')
        v = torch.zeros_like(u)
        S.sbpe3_bind_state(ctx, u.data_ptr(), v.data_ptr(), 0.0)
        S.sbpe3_advance(ctx, 3, dt)
        S.sbpe3_synchronize(ctx)
        t0 = time.perf_counter()
        S.sbpe3_advance(ctx, steps, dt)
        S.sbpe3_synchronize(ctx)
        ms = 1e3 * (time.perf_counter() - t0) / steps
    finally:
        S.sbpe3_destroy(ctx)
    pts = n ** 3
    wb = 8 if dtype == 'f64' else 4
    # own words per point and step: first sweep u, v (6) + 46 coefficients + a1, a2 (6);
    # second sweep a1, a2 (6) + 46 + u, v in (6) and out (6)
    own = (58 + 64) * wb * pts
    return {"workload": "one curvilinear 3-D block of %d^3 points, random major-symmetric stiffness, displacement "
                        "on x3 = 0 and traction elsewhere, body force, 4th order, RK4 at CFL 0.5, %s" % (n, dtype.upper()),
            "ms_per_step": round(ms, 4), "value": pts / (ms * 1e-3),
            "own_bytes_per_step": own, "achieved_own_gbs": round(own / (ms * 1e-3) / 1e9, 1),
            "frac_own_bytes": round(own / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}


def cpu_baseline(n, steps, dt):
    """Oracle RK4 steps on the host (single thread), in a child process."""
    env = dict(os.environ, OMP_NUM_THREADS='1', OPENBLAS_NUM_THREADS='1', MKL_NUM_THREADS='1')
    cmd = [sys.executable, os.path.abspath(__file__), '--cpu-baseline-child', '--cpu-n', str(n),
           '--cpu-steps', str(steps), '--cpu-dt', repr(dt)]
    r = subprocess.run(cmd, capture_output=True, text=True, env=env, timeout=900)
    if r.returncode != 0:
        log(r.stderr[-2000:])
        return None
    out = json.loads(r.stdout.strip().splitlines()[-1])
    # the host it ran on
    try:
        with open('/proc/cpuinfo') as f:
            models = [ln.split(':', 1)[1].strip() for ln in f if ln.startswith('model name')]
        out['cpu_model'] = models[0] if models else None
    except OSError:
        out['cpu_model'] = None
    out['host_cpus'] = os.cpu_count()
    return out


def cpu_baseline_child(n, steps, dt):
    """The oracle on the headline recipe with blocks of n^2 points (the full
    2049^2 blocks take about a minute per RK4 step in the oracle): points x
    steps / wall time of `steps` literal RK4 steps after one warm-up step.  The
    time step (the headline run's) does not change the cost of a step."""
    import numpy as np
    from paper_2003_12811_amd import workloads as W
    from oracle import spec as OS, timestep as T
    spec = W.spec_c3(n=n)
    P = OS.build(spec)
    u = [np.zeros((2, n, n)) for _ in spec['blocks']]
    v = [np.zeros((2, n, n)) for _ in spec['blocks']]
    t = 0.0
    u, v = T.rk4_step(P, u, v, t, dt)       # warm-up step
    t += dt
    t0 = time.perf_counter()
    for _ in range(steps):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
    wall = time.perf_counter() - t0
    npts = len(spec['blocks']) * n * n
    print(json.dumps({"value": npts * steps / wall, "unit": "grid-point updates/s", "cores": 1,
                      "kind": "oracle", "sample": "%d RK4 steps of the headline recipe at reduced block size "
                      "(2x2 blocks of %dx%d, %d points; FP64, NumPy/SciPy, one thread), %.1f s; the oracle's "
                      "cost per point and step does not depend on the block size" % (steps, n, n, npts, wall)}))


def section(spec, dtype, args, tiles, loops, tune_steps, apply_reps, events_in_timed, fixed, steps=None):
    """Tune the launch shape (unless fixed on the command line) and run one workload."""
    shape, table = fixed if args.tile_rows else tune_launch(spec, dtype, tiles=tiles, loops=loops,
                                                            steps=tune_steps)
    r = run_gpu(spec, dtype, steps or args.steps, args.warmup, apply_reps=apply_reps, shape=shape,
                events_in_timed=events_in_timed)
    log('  %.4f ms/step, %.3e updates/s' % (r['ms_per_step'], r['updates_per_s']))
    return r, shape, table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=400)
    ap.add_argument('--warmup', type=int, default=40)
    ap.add_argument('--n', type=int, default=2049, help='block size of the 2x2-block headline workload')
    ap.add_argument('--c2-n', type=int, default=1025, help='size of the single-block workload')
    ap.add_argument('--cpu-n', type=int, default=513, help='block size of the oracle sample')
    ap.add_argument('--cpu-steps', type=int, default=10)
    ap.add_argument('--cpu-dt', type=float, default=1e-4)
    ap.add_argument('--headline-only', action='store_true', help='only the headline workload')
    ap.add_argument('--no-headline', action='store_true',
                    help='skip the headline workload (profiler passes over the other sections); the '
                         'printed line then carries the single-block FP64 result as its value')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-c2', action='store_true')
    ap.add_argument('--no-f32', action='store_true')
    ap.add_argument('--no-wide', action='store_true')
    ap.add_argument('--no-order6', action='store_true')
    ap.add_argument('--tile-rows', type=int, default=0,
                    help='interior tile height of every run (0: pick the launch shape by timing candidates)')
    ap.add_argument('--frame-loop', type=int, default=0,
                    help='frame groups per frame workgroup, used with --tile-rows (0: the library default)')
    ap.add_argument('--cpu-baseline-child', action='store_true')
    ap.add_argument('--no-serve', action='store_true')
    ap.add_argument('--no-gradient', action='store_true')
    ap.add_argument('--no-c1', action='store_true')
    ap.add_argument('--no-3d', action='store_true')
    ap.add_argument('--n3d', type=int, default=97, help='points per direction of the 3-D block')
    # the serving workload (256 shots of 257^2 .. 2049^2, 1500 steps, 20/s) scaled down to a
    # bench-length run with the same offered load: 64 shots, 300 steps, 100/s
    ap.add_argument('--serve-shots', type=int, default=64)
    ap.add_argument('--serve-rate', type=float, default=100.0,
                    help='mean arrival rate of the served stream (shots/s)')
    ap.add_argument('--serve-steps', type=int, default=300)
    ap.add_argument('--serve-sizes', default='257,513,1025,2049')
    ap.add_argument('--serve-workers', type=int, default=4, help='setup threads of both serving forms')
    ap.add_argument('--copy-probe-mib', type=int, default=0,
                    help='first run a plain device-to-device copy of this many MiB (calibrates '
                         'the HBM byte counters of a profiler)')
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.cpu_n, args.cpu_steps, args.cpu_dt)
        return
    world = int(os.environ.get('WORLD_SIZE', '1'))
    if args.gpus != 1 or world != 1:
        print('bench.py measures one GPU only: run it with --gpus 1 (sharding the blocks over '
              'several GPUs is not implemented)', file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_cpu_baseline = args.no_c2 = args.no_f32 = args.no_wide = args.no_order6 = True
        args.no_serve = args.no_gradient = args.no_c1 = args.no_3d = True
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    from paper_2003_12811_amd import workloads as W
    fixed = ((args.tile_rows, args.frame_loop), {})
    n = args.n
    line = {"metric": "grid-point updates/s", "unit": "grid-point updates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic"}
    cbw = None
    if not args.no_headline:
        log('building the headline workload: 2x2 blocks of %dx%d' % (n, n))
        t0 = time.time()
        sp3 = W.spec_c3(n=n)
        log('  built in %.1f s' % (time.time() - t0))
        log('headline, fp64')
        r3, sh3, tb3 = section(sp3, 'f64', args, (20,), (1,), 20, 0, True, fixed)
        k3 = dominant(r3)
        pts3 = swept_points(r3['plan'])
        line.update({
            "value": r3['updates_per_s'], "ms_per_step": r3['ms_per_step'],
            "config": {"workload": "2x2 conforming curvilinear blocks of %dx%d (one smooth global map), random smooth "
                                   "SPD C/rho (seed 0) with contrast 3 between neighbouring blocks, interface SATs, "
                                   "traction top/left and displacement bottom/right, 10 Hz Ricker force, 16 surface "
                                   "receivers, 4th-order SBP-SAT, RK4 CFL 0.5" % (n, n),
                       "points": r3['points'], "dt": r3['dt'], "parallelism": "1 GPU",
                       "tile_rows": sh3[0], "frame_loop": sh3[1], "launch_shape_ms_per_step": tb3},
            "roofline": roofline(k3, r3['kernels'][k3][0], pts3, 8, traffic_key='%s/f64/o4' % k3, tile_rows=sh3[0],
                                 profile='c3_2049'),
            "kernels_ms": {kk: v[0] for kk, v in r3['kernels'].items() if v[1]},
        })
        # (left out of profiler calibration runs, whose copy probe must stay the largest copy)
        cbw = None if args.copy_probe_mib else copy_bandwidth()
        if cbw:
            log('copy bandwidth %.1f GB/s' % cbw)
        if not args.no_f32:
            log('headline workload, fp32')
            r, sh, _ = section(sp3, 'f32', args, (10, 20), (1,), 20, 0, True, fixed)
            k = dominant(r)
            line["c3_f32"] = {"workload": "the headline workload in FP32", "value": r['updates_per_s'],
                              "ms_per_step": r['ms_per_step'], "tile_rows": sh[0],
                              "roofline": roofline(k, r['kernels'][k][0], swept_points(r['plan']), 4),
                              "kernels_ms": {kk: v[0] for kk, v in r['kernels'].items() if v[1]}}
        del sp3

    if not args.no_c2:
        log('building the single-block workload %dx%d' % (args.c2_n, args.c2_n))
        spec = W.spec_c2(n=args.c2_n)
        c2 = "single curvilinear block %dx%d, Gaussian topography, random smooth SPD C/rho (seed 0), " \
             "displacement bottom + traction SATs, 10 Hz Ricker force, 16 receivers" % (args.c2_n, args.c2_n)
        prof = 'c2_%d' % args.c2_n if 'c2_%d' % args.c2_n in TRAFFIC_PROFILES else None
        dtypes = ('f64',) if args.no_f32 else ('f64', 'f32')
        for dt_ in dtypes:
            log('single block, %s' % dt_)
            r, sh, tb = section(spec, dt_, args, TILE_CANDIDATES, FRAME_LOOP_CANDIDATES, 60, 50, False, fixed)
            k = dominant(r)
            pts = swept_points(r['plan'])
            wb = 8 if dt_ == 'f64' else 4
            line["c2_%s" % dt_] = {
                "workload": c2 + ", %s" % dt_.upper(), "value": r['updates_per_s'], "ms_per_step": r['ms_per_step'],
                "ms_per_step_with_events": r['ms_per_step_with_events'],
                "tile_rows": sh[0], "frame_loop": sh[1], "launch_shape_ms_per_step": tb,
                "roofline": roofline(k, r['kernels'][k][0], pts, wb, traffic_key='%s/%s/o4' % (k, dt_),
                                     tile_rows=sh[0], profile=prof),
                "apply_roofline": roofline('interior_apply', r['apply_kernels']['interior_apply'][0], pts, wb,
                                           traffic_key='interior_apply/%s/o4' % dt_, tile_rows=sh[0], profile=prof),
                "kernels_ms": {kk: v[0] for kk, v in r['kernels'].items() if v[1]}}
        if not args.no_wide:
            log('wide-stencil operator, fp64')
            spw = dict(spec)
            spw['operator'] = 'wide'
            r, sh, _ = section(spw, 'f64', args, TILE_CANDIDATES, (1, 2, 4, 8), 60, 50, False, fixed)
            k = dominant(r)
            line["wide"] = {"workload": "the single-block workload with the wide-stencil operator D_i c D_i, FP64",
                            "value": r['updates_per_s'], "ms_per_step": r['ms_per_step'],
                            "tile_rows": sh[0], "frame_loop": sh[1],
                            "roofline": roofline(k, r['kernels'][k][0], swept_points(r['plan']), 8),
                            "apply_roofline": roofline('interior_apply', r['apply_kernels']['interior_apply'][0],
                                                       swept_points(r['plan']), 8),
                            "kernels_ms": {kk: v[0] for kk, v in r['kernels'].items() if v[1]}}
        if not args.no_order6:
            log('sixth-order operators, fp64')
            sp6 = W.spec_c2(n=args.c2_n, order=6)
            r, sh, _ = section(sp6, 'f64', args, (10, 20), (1, 2, 4), 60, 50, False, fixed)
            k = dominant(r)
            line["order6"] = {"workload": "the single-block workload with the sixth-order operators, FP64",
                              "value": r['updates_per_s'], "ms_per_step": r['ms_per_step'],
                              "tile_rows": sh[0], "frame_loop": sh[1],
                              "roofline": roofline(k, r['kernels'][k][0], swept_points(r['plan']), 8),
                              "apply_roofline": roofline('interior_apply', r['apply_kernels']['interior_apply'][0],
                                                         swept_points(r['plan']), 8),
                              "kernels_ms": {kk: v[0] for kk, v in r['kernels'].items() if v[1]}}
    if args.no_headline and "c2_f64" in line:
        line.update(value=line["c2_f64"]["value"], ms_per_step=line["c2_f64"]["ms_per_step"],
                    config={"workload": line["c2_f64"]["workload"], "parallelism": "1 GPU"},
                    roofline=line["c2_f64"]["roofline"])
    if not args.no_serve:
        from paper_2003_12811_amd import serve
        log('served stream vs sequential plain solves')
        # a failure of this section (a shot whose setup fails) is reported in
        # the line instead of ending the run before it is printed
        try:
            sv = serve.serve_and_compare(args.serve_shots, args.serve_rate,
                                         [int(x) for x in args.serve_sizes.split(',')], args.serve_steps,
                                         workers=args.serve_workers)
            sv["scale_down"] = ("the 256-shot stream (20/s, 1500 steps) with 64 shots of 300 steps arriving at "
                                "100/s: the same offered grid-point updates per second")
            if "c2_f32" in line:
                sv["plain_f32_updates_per_s"] = line["c2_f32"]["value"]
                sv["served_over_plain_f32"] = sv["served"]["updates_per_s"] / line["c2_f32"]["value"]
                # the device alone: batched sweeps timed with HIP events, against
                # the plain FP32 rate of one 1025^2 solve
                sv["served_device_over_plain_f32"] = sv["served"]["device_updates_per_s"] / line["c2_f32"]["value"]
            line["serving"] = sv
        except Exception as e:
            log('serving section failed: %r' % (e,))
            line["serving"] = {"error": repr(e)}
    if not args.no_3d:
        log('3-D block, fp64')
        line["block3d"] = bench_3d(args.n3d)
    if not args.no_c1:
        log('plain-method workload (65^2, to t = 0.5): time to solution')
        line["c1_latency"] = c1_latency()
    if not args.no_gradient:
        log('misfit gradient (513^2, 2000 steps, checkpoints every 100)')
        line["gradient"] = gradient_timing()
    if not args.no_cpu_baseline:
        log('cpu baseline (oracle, 1 thread, %d steps of 2x2 blocks of %d^2)' % (args.cpu_steps, args.cpu_n))
        line["cpu_baseline"] = cpu_baseline(args.cpu_n, args.cpu_steps,
                                            args.cpu_dt if args.no_headline else r3['dt'])
    # every roofline also against the measured copy bandwidth
    if cbw is None and not args.copy_probe_mib:
        cbw = copy_bandwidth()
    for sec in [line] + [line[k] for k in ("c3_f32", "c2_f64", "c2_f32", "wide", "order6") if k in line]:
        for key in ("roofline", "apply_roofline"):
            if key in sec and cbw:
                sec[key]["copy_gbs"] = round(cbw, 1)
                sec[key]["frac_of_copy"] = round(sec[key]["achieved"] / cbw, 4)
                sec[key]["frac_of_copy_own_bytes"] = round(sec[key]["achieved_own_bytes"] / cbw, 4)
    print(json.dumps(line), flush=True)


if __name__ == '__main__':
    main()
