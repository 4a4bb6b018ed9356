"""Build the HIP shared library libsbpe.so for gfx950 in-tree.

Usage: python -m paper_2003_12811_amd.build
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'lib', 'libsbpe.so')
HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')

SOURCES = ['sbpe_host.cpp', 'sbpe_kernels.hip']
HOST_ONLY_FLAGS = {'sbpe_host.cpp': ['-fopenmp']}
# packed FP32 instructions are disabled for every device compile
DEVICE_FLAGS = ['--offload-arch=gfx950', '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']
COMMON = ['-O3', '-std=c++17', '-fPIC', '-Wall', '-I', os.path.join(ROOT, 'include')]


def build(verbose=False):
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(os.path.dirname(LIB), src.rsplit('.', 1)[0] + '.o')
        cmd = [HIPCC] + COMMON + DEVICE_FLAGS + HOST_ONLY_FLAGS.get(src, []) + ['-c', os.path.join(CSRC, src), '-o', obj]
        if verbose:
            print(' '.join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        err = '\n'.join(l for l in r.stderr.splitlines() if 'packed-fp32-ops' not in l)
        if r.returncode != 0:
            raise RuntimeError('hipcc failed for %s:\n%s' % (src, err))
        if verbose and err.strip():
            print(err)
        objs.append(obj)
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
