"""Served forward solves with continuous batching.

A stream of independent shots arrives over time.  Each shot is one
curvilinear block with its own material, a Ricker point source and surface
receivers, run for a fixed number of RK4 steps.  The server keeps every
admitted shot's fields and wavefield resident in HBM and advances all of them
together through a library batch (``sbpe_batch_*``): each RK4 sweep covers the
blocks of every admitted shot in one launch (two, on two streams, when the
batch's tiles alone fill the GPU).

* Admission: a shot is set up (library context, coefficient fields, state)
  as soon as it has arrived and its device memory fits in the HBM budget next
  to the shots already admitted (first come, first served); setup runs on
  worker threads while the GPU advances the batch.
* Between chunks of steps, set-up shots join the batch and finished shots
  leave it, their receiver traces are read back and their memory is freed.
* Latency of a shot = completion time - arrival time; the server reports
  p50/p99 latency, shots/s and grid-point updates/s.

``run_sequential`` runs the same shots one after another with the plain
per-context ``sbpe_advance`` (the comparison for the batched form).
"""
import collections
import queue
import threading
import time

import numpy as np

from . import sbpe as S
from . import workloads as W
from .solver import TorchMemory

WORDS_RESIDENT = 11 + 4 + 4   # coefficients, RK workspace (a1, a2), state (u, v) per point
WORDS_PROBE = 4               # finalize's probe and result fields (freed before the shot runs)
FRAME_R = {2: 2, 4: 6, 6: 9}  # depth of the boundary band (frame) per order
PROBES = {2: 81, 4: 81, 6: 169}   # probing colours per component: a frame row has at most 2 x this many entries


def shot_bytes(n, nrec, steps, dtype, order=4):
    """Upper bound of the device memory a shot needs while it is set up and
    run: resident fields and state, finalize's probe fields, the frame
    operator (at most one entry per probe and row), face data, tables and
    receiver rows.  Admission reserves it; once the shot is set up the
    reservation is replaced by the library's exact figure
    (sbpe_device_bytes) plus the state tensors."""
    w = 8 if dtype == 'f64' else 4
    R = FRAME_R[order]
    frame = 2 * R * n + 2 * R * max(0, n - 2 * R)
    csr = 2 * frame * (2 * PROBES[order] * (w + 4) + 4 + 2 * w)
    faces = 4 * n * 16 * w
    return ((WORDS_RESIDENT + WORDS_PROBE) * n * n * w + csr + faces + steps * nrec * 16 * 2 * 8
            + steps * 64 * 3 * 8 + (1 << 20))


def exact_bytes(shot):
    """Device memory of a set-up shot: the library's (sbpe_device_bytes) and
    its two state tensors."""
    held, _ = S.sbpe_device_bytes(shot.ctx)
    return held + 2 * shot.u.numel() * shot.u.element_size()


def make_requests(nshots, rate, sizes, steps, seed=0, nrec=64):
    """Poisson arrivals (mean rate per second) with sizes drawn uniformly."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, nshots)) if rate > 0 else np.zeros(nshots)
    n = rng.choice(np.asarray(sizes), nshots)
    return [dict(id=k, arrival=float(t[k]), n=int(n[k]), seed=k, steps=steps, nrec=nrec) for k in range(nshots)]


class Shot:
    """A library context for one shot, with its state tensors on the device.
    The context's device memory comes from PyTorch's caching allocator, so a
    retired shot's memory returns to the cache without a device-wide free."""

    def __init__(self, req, spec, dtype, device, stream):
        import torch
        self.req = req
        self.memory = TorchMemory(torch, torch.device('cuda', device))
        self.ctx = S.sbpe_create(device, stream.cuda_stream, S.F64 if dtype == 'f64' else S.F32,
                                 spec['order'], 1.0)
        try:
            self._callbacks = S.sbpe_set_allocator(self.ctx, self.memory.alloc, self.memory.release)
            for b in spec['blocks']:
                bid = S.sbpe_add_block(self.ctx, b['X1'], b['X2'], b['rho'], b['C10'])
                for f, (kind, g, tfn, tp, U) in enumerate(b['bc']):
                    if kind != S.BC_TRACTION:
                        S.sbpe_set_bc(self.ctx, bid, f, kind, U)
                    if g is not None:
                        S.sbpe_set_bc_data(self.ctx, bid, f, g, tfn, tp)
            for (bid, x1, x2, f1, f2, amp, fp, t0) in spec.get('sources', []):
                S.sbpe_add_source(self.ctx, bid, x1, x2, f1, f2, amp, fp, t0)
            for (bid, x1, x2) in spec.get('receivers', []):
                S.sbpe_add_receivers(self.ctx, bid, x1, x2)
            S.sbpe_finalize(self.ctx)
            self.dt = S.sbpe_dt_cfl(self.ctx, spec.get('cfl', 0.5))
            tdt = torch.float64 if dtype == 'f64' else torch.float32
            shape = (2,) + spec['blocks'][0]['X1'].shape
            with torch.cuda.stream(stream):
                self.u = torch.zeros(shape, dtype=tdt, device=device)
                self.v = torch.zeros(shape, dtype=tdt, device=device)
            stream.synchronize()
            S.sbpe_bind_state(self.ctx, [self.u.data_ptr()], [self.v.data_ptr()], 0.0)
        except Exception:
            S.sbpe_destroy(self.ctx)
            self.ctx = None
            raise
        self.nrec = sum(len(r[1]) for r in spec.get('receivers', []))
        self.points = sum(b['X1'].size for b in spec['blocks'])

    def receivers(self):
        return S.sbpe_read_receivers(self.ctx, self.nrec)

    def close(self):
        if self.ctx is not None:
            S.sbpe_destroy(self.ctx)
            self.ctx = None


def default_spec(req, device='cuda'):
    """Client-side inputs of a shot (material sums evaluated with torch on the GPU)."""
    return W.spec_shot(req['n'], req['seed'], nrec=req['nrec'], device=device)


class Server:
    """Continuous-batching server over one GPU.

    hbm_budget: bytes of device memory the admitted shots may hold together.
    chunk: RK4 steps advanced between admission / retirement points.
    """

    def __init__(self, dtype='f32', order=4, device=0, hbm_budget=8 << 30, chunk=50, workers=2,
                 spec_fn=default_spec):
        import torch
        self.torch = torch
        self.dtype, self.order, self.device = dtype, order, device
        self.budget, self.chunk, self.workers = hbm_budget, chunk, workers
        self.spec_fn = spec_fn
        self.stream = torch.cuda.Stream(device=device)       # batch launches
        self.aux = torch.cuda.Stream(device=device)          # per-shot setup and read-back
        self.batch = S.sbpe_batch_create(device, self.stream.cuda_stream, S.F64 if dtype == 'f64' else S.F32,
                                         order)

    def close(self):
        if self.batch is not None:
            S.sbpe_batch_destroy(self.batch)
            self.batch = None

    def run(self, requests, keep_receivers=True, log=None):
        """Serve the requests (arrival times in seconds from the start of the
        call); returns per-shot records and summary statistics."""
        reqs = sorted(requests, key=lambda r: r['arrival'])
        lock = threading.Lock()
        used = [0]
        todo = queue.Queue()          # arrived requests, in arrival order
        ready = queue.Queue()         # set-up shots waiting to join the batch
        retired = queue.Queue()       # shots that left the batch
        done, failed = [], []
        start = time.perf_counter()
        now = lambda: time.perf_counter() - start

        def setup_worker():
            while True:
                req = todo.get()
                if req is None:
                    return
                need = shot_bytes(req['n'], req['nrec'], req['steps'], self.dtype, self.order)
                while True:           # wait for HBM budget
                    with lock:
                        if used[0] + need <= self.budget or used[0] == 0:
                            used[0] += need
                            break
                    time.sleep(0.002)
                try:
                    req['t_setup'] = now()
                    shot = Shot(req, self.spec_fn(req), self.dtype, self.device, self.aux)
                    # the reservation becomes the shot's exact device memory
                    # (its receiver rows for every step are reserved at admission)
                    S.sbpe_reserve_steps(shot.ctx, req['steps'])
                    exact = exact_bytes(shot)
                    with lock:
                        used[0] += exact - need
                    shot.need = exact
                    ready.put(shot)
                except Exception as e:     # reported, never silently dropped
                    with lock:
                        used[0] -= need
                    failed.append((req['id'], repr(e)))
                    ready.put(None)

        def reaper():
            # read back and free retired shots off the launch thread (freeing
            # device memory may wait for the device)
            while True:
                s = retired.get()
                if s is None:
                    return
                rec = s.receivers()       # ordered after the shot's last batched step
                s.req['t_done'] = now()
                s.req['latency'] = s.req['t_done'] - s.req['arrival']
                if keep_receivers:
                    s.req['receivers'] = rec
                s.req['points'] = s.points
                s.close()
                del s.u, s.v
                with lock:
                    used[0] -= s.need
                    done.append(s.req)
                if log:
                    log('shot %d (%d^2) done: latency %.3f s' % (s.req['id'], s.req['n'], s.req['latency']))

        threads = [threading.Thread(target=setup_worker, daemon=True) for _ in range(self.workers)]
        threads.append(threading.Thread(target=reaper, daemon=True))
        for t in threads:
            t.start()
        pending = collections.deque(reqs)
        members = {}
        n_left = len(reqs)            # shots not yet handed to the reaper or failed
        self.launched_points_steps = 0
        # device time of the batched sweeps: HIP events on the batch stream
        # around every chunk (the batch joins its side stream into it)
        chunk_events = []
        while n_left > 0:
            t = now()
            while pending and pending[0]['arrival'] <= t:
                todo.put(pending.popleft())
            while True:               # admit everything that is set up
                try:
                    shot = ready.get_nowait()
                except queue.Empty:
                    break
                if shot is None:
                    n_left -= 1
                    continue
                S.sbpe_batch_add(self.batch, shot.ctx, shot.req['steps'], shot.dt)
                shot.req['t_admit'] = now()
                members[id(shot)] = shot
            if not members:
                wait = pending[0]['arrival'] - now() if pending else 0.0
                time.sleep(min(max(wait, 0.0005), 0.02))
                continue
            info = S.sbpe_batch_info(self.batch)
            k = min(self.chunk, info['min_remaining'])
            e0 = self.torch.cuda.Event(enable_timing=True)
            e1 = self.torch.cuda.Event(enable_timing=True)
            e0.record(self.stream)
            S.sbpe_batch_advance(self.batch, k)
            e1.record(self.stream)
            chunk_events.append((e0, e1))
            self.launched_points_steps += info['points'] * k
            for s in [s for s in members.values() if S.sbpe_batch_remaining(self.batch, s.ctx) == 0]:
                S.sbpe_batch_remove(self.batch, s.ctx)
                del members[id(s)]
                retired.put(s)
                n_left -= 1
        for _ in range(self.workers):
            todo.put(None)
        retired.put(None)
        for t in threads:
            t.join()
        S.sbpe_batch_synchronize(self.batch)
        wall = now()
        lat = np.array([r['latency'] for r in done]) if done else np.zeros(1)
        total_pts = sum(r['points'] * r['steps'] for r in done)
        device_s = 1e-3 * sum(a.elapsed_time(b) for a, b in chunk_events)
        return dict(shots=done, failed=failed, wall_s=wall,
                    p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                    shots_per_s=len(done) / wall, updates_per_s=total_pts / wall,
                    device_s=device_s, device_updates_per_s=self.launched_points_steps / device_s if device_s else 0.0)


def run_sequential(requests, dtype='f32', device=0, spec_fn=default_spec, keep_receivers=True, log=None,
                   workers=2):
    """The same shots, in arrival order, one at a time with sbpe_advance
    (each starts when it has arrived and the previous one has finished).
    `workers` threads set up the next shots while the current one runs, as
    the server's setup workers do, so both forms overlap host setup with
    device work and differ only in how the device is used."""
    import concurrent.futures
    import torch
    reqs = [dict(r) for r in sorted(requests, key=lambda r: r['arrival'])]
    start = time.perf_counter()
    now = lambda: time.perf_counter() - start
    def build(r):
        wait = r['arrival'] - now()
        if wait > 0:
            time.sleep(wait)
        st = torch.cuda.Stream(device=device)     # the shot's own stream
        shot = Shot(r, spec_fn(r), dtype, device, st)
        shot.stream = st
        return shot

    device_s = 0.0
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as pool:
        futs, nxt = {}, 0
        for k, r in enumerate(reqs):
            # at most `workers` shots set up ahead of the one on the device
            while nxt < len(reqs) and nxt <= k + workers:
                futs[nxt] = pool.submit(build, reqs[nxt])
                nxt += 1
            shot = futs.pop(k).result()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(shot.stream)
            S.sbpe_advance(shot.ctx, r['steps'], shot.dt)
            e1.record(shot.stream)
            rec = shot.receivers()
            device_s += 1e-3 * e0.elapsed_time(e1)
            r['t_done'] = now()
            r['latency'] = r['t_done'] - r['arrival']
            r['points'] = shot.points
            if keep_receivers:
                r['receivers'] = rec
            shot.close()
            if log and r['id'] % 16 == 0:
                log('sequential: shot %d done at %.2f s' % (r['id'], r['t_done']))
    wall = now()
    lat = np.array([r['latency'] for r in reqs])
    total_pts = sum(r['points'] * r['steps'] for r in reqs)
    return dict(shots=reqs, wall_s=wall, p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                shots_per_s=len(reqs) / wall, updates_per_s=total_pts / wall,
                device_s=device_s, device_updates_per_s=total_pts / device_s if device_s else 0.0)


def summarize(res):
    keys = ('wall_s', 'p50_s', 'p99_s', 'shots_per_s', 'updates_per_s', 'device_s', 'device_updates_per_s')
    return {k: res[k] for k in keys} | {'shots': len(res['shots'])}


def main(argv=None):
    """Serve a Poisson stream of shots and compare with sequential plain solves.

      python -m paper_2003_12811_amd.serve [--shots 256] [--rate 20] [--sizes 257,513,1025,2049]
          [--steps 1500] [--dtype f32] [--budget-gb 32] [--chunk 50] [--no-sequential]
    Prints one JSON line.
    """
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument('--shots', type=int, default=256)
    ap.add_argument('--rate', type=float, default=20.0)
    ap.add_argument('--sizes', default='257,513,1025,2049')
    ap.add_argument('--steps', type=int, default=1500)
    ap.add_argument('--nrec', type=int, default=64)
    ap.add_argument('--dtype', default='f32')
    ap.add_argument('--budget-gb', type=float, default=32.0)
    ap.add_argument('--chunk', type=int, default=50)
    ap.add_argument('--workers', type=int, default=4)
    ap.add_argument('--seed', type=int, default=0)
    ap.add_argument('--no-sequential', action='store_true')
    args = ap.parse_args(argv)
    out = serve_and_compare(args.shots, args.rate, [int(x) for x in args.sizes.split(',')], args.steps,
                            args.nrec, args.dtype, args.budget_gb, args.chunk, args.workers, args.seed,
                            not args.no_sequential)
    print(json.dumps(out), flush=True)


def serve_and_compare(shots, rate, sizes, steps, nrec=64, dtype='f32', budget_gb=32.0, chunk=50, workers=2,
                      seed=0, sequential=True):
    """Served run of a Poisson stream, then (optionally) the same shots as
    sequential plain solves; returns the summary dictionary."""
    import json
    import sys
    from types import SimpleNamespace
    args = SimpleNamespace(shots=shots, rate=rate, steps=steps, nrec=nrec, dtype=dtype, budget_gb=budget_gb,
                           chunk=chunk, workers=workers, seed=seed, no_sequential=not sequential)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)
    reqs = make_requests(args.shots, args.rate, sizes, args.steps, seed=args.seed, nrec=args.nrec)
    srv = Server(dtype=args.dtype, hbm_budget=int(args.budget_gb * (1 << 30)), chunk=args.chunk,
                 workers=args.workers)
    try:
        log('served: %d shots, sizes %s, %d steps, %.1f/s' % (args.shots, sizes, args.steps, args.rate))
        res = srv.run([dict(r) for r in reqs], log=log if shots > 64 else None)
    finally:
        srv.close()
    out = dict(workload='Poisson stream (%.1f/s, seed %d) of %d shots, n^2 with n uniform in %s, %d RK4 steps, '
                        '%d receivers, %s' % (args.rate, args.seed, args.shots, sizes, args.steps, args.nrec,
                                              args.dtype),
               served=summarize(res), failed=res['failed'])
    log('  served:', json.dumps(out['served']))
    if not args.no_sequential:
        log('sequential plain solves')
        seq = run_sequential([dict(r) for r in reqs], dtype=args.dtype, log=log if shots > 64 else None,
                             workers=args.workers)
        out['sequential'] = summarize(seq)
        log('  sequential:', json.dumps(out['sequential']))
        by_id = {r['id']: r['receivers'] for r in seq['shots']}
        out['bitwise_equal_to_sequential'] = all(np.array_equal(r['receivers'], by_id[r['id']])
                                                 for r in res['shots'])
        out['throughput_ratio'] = res['updates_per_s'] / seq['updates_per_s']
    return out


if __name__ == '__main__':
    main()
