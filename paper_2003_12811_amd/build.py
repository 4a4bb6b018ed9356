"""Build the HIP shared library libsbpe.so for gfx950 in-tree.

Usage: python -m paper_2003_12811_amd.build
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'lib', 'libsbpe.so')
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')

# the host runtime, the launchers and small kernels, and one translation unit
# per (precision, order) pair of the large kernels; compiled in parallel
SOURCES = ['sbpe_host.cpp', 'sbpe_kernels.hip', 'sbpe3_kernels.hip'] + sorted(
    os.path.basename(p) for p in glob.glob(os.path.join(CSRC, 'sbpe_inst_*.hip')))
HOST_ONLY_FLAGS = {'sbpe_host.cpp': ['-fopenmp']}
# packed FP32 instructions are disabled for every device compile
DEVICE_FLAGS = ['--offload-arch=gfx950', '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']
COMMON = ['-O3', '-std=c++17', '-fPIC', '-Wall', '-I', os.path.join(ROOT, 'include')]


def _compile(src, obj, verbose):
    cmd = [HIPCC] + COMMON + DEVICE_FLAGS + HOST_ONLY_FLAGS.get(src, []) + ['-c', os.path.join(CSRC, src), '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = '\n'.join(l for l in r.stderr.splitlines() if 'packed-fp32-ops' not in l)
    return cmd, r.returncode, err


def build(verbose=False, jobs=None):
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    objs = [os.path.join(os.path.dirname(LIB), src.rsplit('.', 1)[0] + '.o') for src in SOURCES]
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(SOURCES, objs)))
    for src, (cmd, rc, err) in zip(SOURCES, results):
        if verbose:
            print(' '.join(cmd), flush=True)
        if rc != 0:
            raise RuntimeError('hipcc failed for %s:\n%s' % (src, err))
        if verbose and err.strip():
            print(err)
    tmp = LIB + '.tmp'
    cmd = [HIPCC, '-shared', '-fPIC', '--offload-arch=gfx950', '-fopenmp'] + objs + ['-o', tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError('link failed:\n' + r.stderr)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == '__main__':
    print(build(verbose='-v' in sys.argv))
