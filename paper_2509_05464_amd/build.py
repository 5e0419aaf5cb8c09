"""Build libfqpd.so (all HIP sources under csrc/) for gfx950, in-tree."""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(HERE, '_build')
LIB = os.path.join(HERE, 'libfqpd.so')

HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
# Packed-FP32 instructions are disabled: hipcc would otherwise pair FP32 math into
# v_pk_* forms.  The host pass warns that it does not know the feature; harmless.
FLAGS = ['--offload-arch=gfx950', '-O3', '-fPIC', '-std=c++17', '-Wall', '-Wno-unused-variable',
         '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src).replace('.hip', '.o'))
    cmd = [HIPCC, *FLAGS, '-c', src, '-o', obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f'hipcc failed on {src}')
    return obj


def build(jobs: int = 8) -> str:
    """Compile every csrc/*.hip and link libfqpd.so (always rebuilds)."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, '*.hip')))
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + '.tmp'
    r = subprocess.run([HIPCC, '--offload-arch=gfx950', '-shared', '-fPIC', '-o', tmp, *objs],
                       capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError('link of libfqpd.so failed')
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build())
