#!/usr/bin/env python3
"""Throughput of the RK4-advanced SBP-SAT anisotropic elastic solver on one MI355X.

Workload (the single-GPU configuration the headline metric is quoted on): one
curvilinear block of 1025 x 1025 points with Gaussian topography, smooth random
SPD stiffness and density (8 Fourier modes per field, seed 0), displacement SAT
on the bottom face and traction SATs elsewhere, a 10 Hz Ricker point force and
16 surface receivers; classical RK4 at CFL 0.5.  A step is one full RK4 step
(four right-hand-side evaluations fused into two sweeps over the grid,
sources, receivers).  Inputs are resident in HBM before timing starts.  The
launch shape (tile height, frame groups per frame workgroup) is picked by
timing candidates first; it does not change the results.  The
throughput comes from the timed steps alone; the launch durations of the
roofline come from the same number of steps run again with HIP events around
every launch (the events lengthen a 1025^2 step by 12-19 %).

Prints one JSON line on stdout; progress goes to stderr.  The primary result is
FP64; the FP32 variant, the plain operator apply, the same workload with the
wide-stencil operator, working sets larger than the MALL (one 2049^2 block in
FP64, 2x2 blocks of 2049^2 in FP32) and a served stream of shots (continuous batching against
sequential plain solves, p50/p99 latency) are reported beside it.

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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# measured HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)
# of the 1025^2 workload; ignored once the kernel source has changed
TRAFFIC_PROFILES = {n: os.path.join(ROOT, 'profiles', 'hbm_traffic_c2_%d.md' % n) for n in (1025, 2049)}


def roofline(kind, ms, points, wbytes, traffic_key=None, tile_rows=None, n=1025):
    byts = WORDS[kind] * wbytes * points
    gbs = byts / (ms * 1e-3) / 1e9
    traffic = None
    if traffic_key is not None:
        from paper_2003_12811_amd import profiling
        path = TRAFFIC_PROFILES.get(n)
        t = profiling.read_traffic(path, tile_rows=tile_rows or 10) if path else None
        traffic = t.get(traffic_key) if t else None
    return {"bound": "hbm", "kernel": kind, "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS,
            "unit": "GB/s", "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic,
            "avg_ms": round(ms, 5), "bytes_per_launch": byts}


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


def run_gpu(spec, dtype, steps, warmup, apply_reps=0, shape=(0, 0)):
    import torch
    from paper_2003_12811_amd import sbpe as S
    from paper_2003_12811_amd.solver import Solver
    sol = Solver(spec, dtype, tile_rows=shape[0])
    if shape[1]:
        sol.set_frame_loop(shape[1])
    dt = sol.dt_cfl(spec.get('cfl', 0.5))
    sol.set_state(None, None, 0.0)
    plan = S.sbpe_plan_info(sol.ctx)
    npts = sum(b['X1'].size for b in spec['blocks'])
    sol.advance(warmup, dt)
    sol.synchronize()
    torch.cuda.synchronize()
    # the timed steps, without per-launch events (they cost 12-19 % of a
    # 1025^2 step), give the throughput ...
    t0 = time.perf_counter()
    sol.advance(steps, dt)
    sol.synchronize()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    # ... then the same number of steps again with HIP events around every
    # launch, on the launch's own stream, give the launch durations
    S.sbpe_set_kernel_timing(sol.ctx, 1)
    S.sbpe_get_kernel_timing(sol.ctx)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    sol.advance(steps, dt)
    sol.synchronize()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    kt = S.sbpe_get_kernel_timing(sol.ctx)
    res = dict(dtype=dtype, points=npts, steps=steps, wall_s=wall, ms_per_step=1e3 * wall / steps,
               ms_per_step_with_events=1e3 * (t3 - t2) / steps,
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
    """Wall time of the forward run and of the adjoint gradient on the
    differentiation workload (FP64)."""
    import torch
    from paper_2003_12811_amd import adjoint as ADJ
    from paper_2003_12811_amd import workloads as W
    from paper_2003_12811_amd.solver import Solver
    spec, spec_obs = W.spec_c5(n=n), W.spec_c5(n=n, perturbed=True)
    s = Solver(spec, 'f64')
    dt = s.dt_cfl(0.5)
    s.close()
    obs = ADJ.MisfitGradient(spec_obs, nsteps, dt)
    obs.forward()
    d_obs = obs.traces.copy()
    obs.close()
    mg = ADJ.MisfitGradient(spec, nsteps, dt, d_obs=d_obs, checkpoint_every=ckpt)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = mg.forward()
    t1 = time.perf_counter()
    g_rho, g_c10 = mg.gradient()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    mg.close()
    return {"workload": "%dx%d block, %d RK4 steps, 100 receivers, misfit against the +5%% blob model, "
                        "checkpoints every %d steps, FP64" % (n, n, nsteps, ckpt),
            "J": J, "forward_s": t1 - t0, "gradient_s": t2 - t1, "gradient_over_forward": (t2 - t1) / (t1 - t0),
            "forward_updates_per_s": n * n * nsteps / (t1 - t0)}


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


def cpu_baseline(n, steps):
    """Oracle RK4 steps on the host (single thread), in a child process."""
    env = dict(os.environ, OMP_NUM_THREADS='1', OPENBLAS_NUM_THREADS='1', MKL_NUM_THREADS='1')
    cmd = [sys.executable, os.path.abspath(__file__), '--cpu-baseline-child', '--n', str(n),
           '--cpu-steps', str(steps)]
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


def cpu_baseline_child(n, steps):
    import numpy as np
    from paper_2003_12811_amd import workloads as W
    from oracle import spec as OS, timestep as T
    spec = W.spec_c2(n=n)
    P = OS.build(spec)
    dt = T.dt_cfl(P, 0.5)
    u = [np.zeros((2, n, n))]
    v = [np.zeros((2, n, n))]
    t = 0.0
    u, v = T.rk4_step(P, u, v, t, dt)       # warm-up step
    t += dt
    t0 = time.perf_counter()
    for _ in range(steps):
        u, v = T.rk4_step(P, u, v, t, dt)
        t += dt
    wall = time.perf_counter() - t0
    print(json.dumps({"value": n * n * steps / wall, "unit": "grid-point updates/s", "cores": 1,
                      "kind": "oracle", "sample": "%d RK4 steps of the %dx%d workload (FP64, NumPy/SciPy, "
                      "one thread), %.1f s" % (steps, n, n, wall)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=400)
    ap.add_argument('--warmup', type=int, default=40)
    ap.add_argument('--n', type=int, default=1025)
    ap.add_argument('--cpu-steps', type=int, default=10)
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-large', action='store_true')
    ap.add_argument('--no-wide', action='store_true')
    ap.add_argument('--no-hbm', action='store_true')
    ap.add_argument('--tile-rows', type=int, default=0,
                    help='interior tile height of the 1025^2 runs (0: pick the launch shape by timing candidates)')
    ap.add_argument('--frame-loop', type=int, default=0,
                    help='frame groups per frame workgroup, used with --tile-rows (0: the library default)')
    ap.add_argument('--large-n', type=int, default=2049)
    ap.add_argument('--cpu-baseline-child', action='store_true')
    ap.add_argument('--no-serve', action='store_true')
    ap.add_argument('--no-gradient', action='store_true')
    ap.add_argument('--serve-shots', type=int, default=48)
    ap.add_argument('--serve-rate', type=float, default=200.0,
                    help='mean arrival rate of the served stream (shots/s); the default saturates the GPU')
    ap.add_argument('--serve-steps', type=int, default=300)
    ap.add_argument('--copy-probe-mib', type=int, default=0,
                    help='first run a plain device-to-device copy of this many MiB (calibrates '
                         'the HBM byte counters of a profiler)')
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args.n, args.cpu_steps)
        return
    world = int(os.environ.get('WORLD_SIZE', '1'))
    if args.gpus != 1 or world != 1:
        print('bench.py measures one GPU only: run it with --gpus 1 (sharding the blocks over '
              'several GPUs is not implemented)', file=sys.stderr)
        sys.exit(2)
    if args.copy_probe_mib:
        copy_probe(args.copy_probe_mib)
    from paper_2003_12811_amd import workloads as W
    log('building workload %dx%d' % (args.n, args.n))
    spec = W.spec_c2(n=args.n)
    fixed = ((args.tile_rows, args.frame_loop), {})
    tuned64, tuned32 = fixed, fixed
    if not args.tile_rows:
        log('launch shape, fp64')
        tuned64 = tune_launch(spec, 'f64')
        log('launch shape, fp32')
        tuned32 = tune_launch(spec, 'f32')
    log('fp64 run')
    r64 = run_gpu(spec, 'f64', args.steps, args.warmup, apply_reps=50, shape=tuned64[0])
    log('  %.3f ms/step, %.3e updates/s' % (r64['ms_per_step'], r64['updates_per_s']))
    log('fp32 run')
    r32 = run_gpu(spec, 'f32', args.steps, args.warmup, apply_reps=50, shape=tuned32[0])
    log('  %.3f ms/step, %.3e updates/s' % (r32['ms_per_step'], r32['updates_per_s']))
    pts = swept_points(r64['plan'])
    k = dominant(r64)
    line = {
        "metric": "grid-point updates/s", "value": r64['updates_per_s'], "unit": "grid-point updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": r64['ms_per_step'],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "single curvilinear block %dx%d, Gaussian topography, random smooth SPD C/rho "
                               "(seed 0), displacement bottom + traction SATs, 10 Hz Ricker force, 16 receivers, "
                               "4th-order SBP-SAT, RK4 CFL 0.5" % (args.n, args.n),
                   "points": r64['points'], "dt": r64['dt'], "parallelism": "1 GPU",
                   "tile_rows": tuned64[0][0], "frame_loop": tuned64[0][1],
                   "launch_shape_ms_per_step": tuned64[1]},
        "roofline": roofline(k, r64['kernels'][k][0], pts, 8,
                             traffic_key='%s/f64/o4' % k, tile_rows=tuned64[0][0], n=args.n),
        "kernels_ms": {kk: v[0] for kk, v in r64['kernels'].items() if v[1]},
        "ms_per_step_with_events": r64['ms_per_step_with_events'],
        "apply_roofline": roofline('interior_apply', r64['apply_kernels']['interior_apply'][0], pts, 8,
                                   traffic_key='interior_apply/f64/o4', tile_rows=tuned64[0][0], n=args.n),
        "f32": {"value": r32['updates_per_s'], "ms_per_step": r32['ms_per_step'],
                "tile_rows": tuned32[0][0], "frame_loop": tuned32[0][1],
                "roofline": roofline(dominant(r32), r32['kernels'][dominant(r32)][0], pts, 4,
                                     traffic_key='%s/f32/o4' % dominant(r32), tile_rows=tuned32[0][0], n=args.n),
                "apply_roofline": roofline('interior_apply', r32['apply_kernels']['interior_apply'][0], pts, 4,
                                           traffic_key='interior_apply/f32/o4', tile_rows=tuned32[0][0],
                                           n=args.n)},
    }
    # (left out of profiler calibration runs, whose copy probe must stay the largest copy)
    cbw = None if args.copy_probe_mib else copy_bandwidth()
    if cbw:
        log('copy bandwidth %.1f GB/s' % cbw)
    if not args.no_wide:
        log('wide-stencil operator, fp64')
        spw = dict(spec)
        spw['operator'] = 'wide'
        tw = fixed if args.tile_rows else tune_launch(spw, 'f64', loops=(1, 2, 4, 8))
        rw = run_gpu(spw, 'f64', args.steps, args.warmup, apply_reps=50, shape=tw[0])
        kw = dominant(rw)
        line["wide"] = {"workload": "the same %dx%d workload with the wide-stencil operator D_i c D_i, FP64"
                                    % (args.n, args.n),
                        "value": rw['updates_per_s'], "ms_per_step": rw['ms_per_step'],
                        "tile_rows": tw[0][0], "frame_loop": tw[0][1],
                        "roofline": roofline(kw, rw['kernels'][kw][0], swept_points(rw['plan']), 8),
                        "apply_roofline": roofline('interior_apply', rw['apply_kernels']['interior_apply'][0],
                                                   swept_points(rw['plan']), 8),
                        "kernels_ms": {kk: v[0] for kk, v in rw['kernels'].items() if v[1]}}
        log('  %.3f ms/step, %.3e updates/s' % (rw['ms_per_step'], rw['updates_per_s']))
    if not args.no_hbm:
        # the roofline case beyond the MALL in FP64: one 2049^2 block of the same recipe
        # (about 0.8 GB per sweep; the 1025^2 working set fits the 256 MB MALL)
        log('hbm-bound working set: %dx%d, fp64' % (args.large_n, args.large_n))
        sph = W.spec_c2(n=args.large_n)
        th = fixed if args.tile_rows else tune_launch(sph, 'f64', tiles=(10, 20), loops=(1, 2, 4), steps=20)
        rh = run_gpu(sph, 'f64', max(args.steps // 4, 20), 10, shape=th[0])
        kh = dominant(rh)
        line["hbm_bound"] = {"workload": "the same recipe on one %dx%d block, FP64 (working set beyond the MALL)"
                                         % (args.large_n, args.large_n),
                             "value": rh['updates_per_s'], "ms_per_step": rh['ms_per_step'],
                             "tile_rows": th[0][0], "frame_loop": th[0][1],
                             "roofline": roofline(kh, rh['kernels'][kh][0], swept_points(rh['plan']), 8,
                                                  traffic_key='%s/f64/o4' % kh, tile_rows=th[0][0], n=args.large_n),
                             "kernels_ms": {kk: v[0] for kk, v in rh['kernels'].items() if v[1]}}
        log('  %.3f ms/step, %.3e updates/s' % (rh['ms_per_step'], rh['updates_per_s']))
    if not args.no_large:
        log('large working set: 2x2 blocks of %d^2, fp32' % args.large_n)
        t0 = time.time()
        sp3 = W.spec_c3(n=args.large_n)
        log('  workload built in %.1f s' % (time.time() - t0))
        t3 = fixed if args.tile_rows else tune_launch(sp3, 'f32', tiles=(10, 20), loops=(1,), steps=20)
        r3 = run_gpu(sp3, 'f32', max(args.steps // 4, 20), 10, shape=t3[0])
        k3 = dominant(r3)
        line["large"] = {"workload": "2x2 blocks of %d^2 with interfaces, FP32" % args.large_n,
                         "value": r3['updates_per_s'], "ms_per_step": r3['ms_per_step'], "tile_rows": t3[0][0],
                         "roofline": roofline(k3, r3['kernels'][k3][0], swept_points(r3['plan']), 4),
                         "kernels_ms": {kk: v[0] for kk, v in r3['kernels'].items() if v[1]}}
        log('  %.3f ms/step, %.3e updates/s' % (r3['ms_per_step'], r3['updates_per_s']))
    if not args.no_serve:
        from paper_2003_12811_amd import serve
        log('served stream vs sequential plain solves')
        line["serving"] = serve.serve_and_compare(args.serve_shots, args.serve_rate, [257, 513, 1025],
                                                  args.serve_steps)
    if not args.no_gradient:
        log('misfit gradient (513^2, 2000 steps, checkpoints every 100)')
        line["gradient"] = gradient_timing()
    if not args.no_cpu_baseline:
        log('cpu baseline (oracle, 1 thread, %d steps)' % args.cpu_steps)
        line["cpu_baseline"] = cpu_baseline(args.n, args.cpu_steps)
    # every roofline also against the measured copy bandwidth
    for sec in (line, line["f32"], line.get("wide", {}), line.get("hbm_bound", {}), line.get("large", {})):
        for key in ("roofline", "apply_roofline"):
            if key in sec and cbw:
                sec[key]["copy_gbs"] = round(cbw, 1)
                sec[key]["frac_of_copy"] = round(sec[key]["achieved"] / cbw, 4)
    print(json.dumps(line), flush=True)


if __name__ == '__main__':
    main()
