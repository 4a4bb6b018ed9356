"""Summaries of rocprofv3 output for the profiles/ folder, and their reader.

Two kinds of summary are written as short Markdown files:

* kernel statistics (``--kernel-trace --stats -f csv``): calls, average and
  total duration per kernel;
* HBM traffic (two ``--pmc`` passes, FETCH_SIZE then WRITE_SIZE, both in KiB
  per dispatch): every counter is scaled by what the same counter reads for a
  plain device-to-device copy of known size run in the same process
  (``bench.py --copy-probe-mib``), and the result is recorded per kernel
  together with the SHA-256 of the device sources it was measured on.

``read_traffic`` returns the recorded bytes per launch only while the kernel
source is unchanged, so a stale measurement is never reported.

  python -m paper_2003_12811_amd.profiling stats <kernel_stats.csv> <out.md> "<command>"
  python -m paper_2003_12811_amd.profiling traffic <fetch.csv> <write.csv> <copy MiB> <out.md> "<command>"
"""
import collections
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
# every source that decides the device code of the kernels
KERNEL_SOURCE = [os.path.join(HERE, 'csrc', f) for f in
                 ('sbpe_device.h', 'sbpe_kernels.hip', 'sbpe_launch_impl.h', 'sbpe_tables.h', 'sbpe_internal.h')]
COPY_KERNEL = '__amd_rocclr_copyBuffer'


def source_hash(paths=KERNEL_SOURCE):
    h = hashlib.sha256()
    for p in paths:
        with open(p, 'rb') as f:
            h.update(f.read())
    return h.hexdigest()


def kernel_kind(name):
    """'interior_rk1/f64' style label of a library kernel name, or None."""
    m = re.search(r'sbpe::k_(march|pass_wide|pass|frame_sp|frame|wide)<(double|float), (\d)(?:, (\d))?', name)
    if not m:
        return None
    part, ty, order, p = m.group(1), m.group(2), m.group(3), m.group(4)
    dt = 'f64' if ty == 'double' else 'f32'
    if part in ('march', 'pass'):
        # a one-launch sweep (k_pass) also updates the frame points
        return 'interior_%s/%s/o%s' % (('apply', 'rk1', 'rk2')[int(p)], dt, order)
    if part in ('wide', 'pass_wide'):
        # the wide-stencil operator's tiles (a one-launch sweep also updates the frame points)
        return 'wide_%s/%s/o%s' % (('apply', 'rk1', 'rk2')[int(p)], dt, order)
    if part == 'frame_sp':
        return 'frame_%s/%s/o%s' % (('apply', 'rk1', 'rk2')[int(p)], dt, order)
    # the stencil form of the frame rows, run at setup to assemble the operator
    return 'frame_stencil/%s/o%s' % (dt, order)


def summarize_stats(stats_csv, out_md, command):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = ['# Kernel statistics', '', 'Command (run from `/tmp` with `TMPDIR=/tmp`):', '', '```', command, '```', '',
             '| kernel | calls | average µs | total ms | share % |', '|---|---|---|---|---|']
    for r in rows:
        lines.append('| `%s` | %s | %.2f | %.3f | %.2f |' % (
            r['Name'][:90], r['Calls'], float(r['AverageNs']) / 1e3, float(r['TotalDurationNs']) / 1e6,
            float(r['Percentage'])))
    open(out_md, 'w').write('\n'.join(lines) + '\n')


def _per_dispatch(counter_csv):
    out = collections.defaultdict(list)
    for r in csv.DictReader(open(counter_csv)):
        out[r['Kernel_Name']].append(float(r['Counter_Value']))
    return out


def summarize_traffic(fetch_csv, write_csv, copy_mib, out_md, command):
    fe, wr = _per_dispatch(fetch_csv), _per_dispatch(write_csv)
    true_kib = copy_mib * 1024.0
    # the copy probe is the largest copy dispatch of the run
    f_scale = true_kib / max(fe[COPY_KERNEL])
    w_scale = true_kib / max(wr[COPY_KERNEL])
    lines = ['# HBM traffic per launch (rocprofv3 PMC)', '',
             'Commands (run from `/tmp` with `TMPDIR=/tmp`; one counter per pass):', '', '```']
    lines += [command.replace('{COUNTER}', 'FETCH_SIZE'), command.replace('{COUNTER}', 'WRITE_SIZE'), '```', '',
              'Calibration: a device-to-device copy of %d MiB reads FETCH_SIZE %.1f KiB and WRITE_SIZE %.1f KiB, '
              'so FETCH_SIZE is scaled by %.4f and WRITE_SIZE by %.4f.' % (
                  copy_mib, max(fe[COPY_KERNEL]), max(wr[COPY_KERNEL]), f_scale, w_scale), '',
              'kernel source sha256 = %s' % source_hash(), '',
              'interior tile rows = %d' % _tile_rows(command), '',
              '| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | read MB | written MB |',
              '|---|---|---|---|---|---|']
    machine = []
    for name in sorted(fe):
        kind = kernel_kind(name)
        if kind is None or name not in wr:
            continue
        f = sum(fe[name]) / len(fe[name])
        w = sum(wr[name]) / len(wr[name])
        rb, wb = f * 1024 * f_scale, w * 1024 * w_scale
        lines.append('| `%s` | %d | %.1f | %.1f | %.2f | %.2f |' % (kind, len(fe[name]), f, w, rb / 1e6, wb / 1e6))
        machine.append('traffic_bytes %s = %d' % (kind, int(round(rb + wb))))
    lines += ['', 'Scaled bytes per launch (read + written):', '', '```'] + machine + ['```']
    open(out_md, 'w').write('\n'.join(lines) + '\n')


def _tile_rows(command):
    """Interior tile height of a bench.py command line (10 unless given)."""
    m = re.search(r'--tile-rows (\d+)', command)
    return int(m.group(1)) if m else 10


def read_traffic(md_path, source=KERNEL_SOURCE, tile_rows=None):
    """{kind: bytes per launch} from a traffic summary, or None if it is
    missing, was measured on a different kernel source, or (tile_rows given)
    with another interior tile height."""
    if not os.path.exists(md_path):
        return None
    txt = open(md_path).read()
    m = re.search(r'kernel source sha256 = ([0-9a-f]{64})', txt)
    if not m or m.group(1) != source_hash(source):
        return None
    if tile_rows is not None:
        t = re.search(r'interior tile rows = (\d+)', txt)
        if not t or int(t.group(1)) != tile_rows:
            return None
    return {k: int(v) for k, v in re.findall(r'traffic_bytes (\S+) = (\d+)', txt)}


if __name__ == '__main__':
    if sys.argv[1] == 'stats':
        summarize_stats(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == 'traffic':
        summarize_traffic(sys.argv[2], sys.argv[3], int(sys.argv[4]), sys.argv[5], sys.argv[6])
    else:
        raise SystemExit(__doc__)
