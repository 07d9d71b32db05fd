"""Build the HIP library liblbmib.so for gfx950 in-tree (hipcc), in parallel per source file.

    python -m paper_2607_07432_amd.build          # or build.build() from Python

Device code is compiled with packed-FP32 instruction selection disabled; the host
geometry precompute is compiled without floating-point contraction so its integer
lists are reproducible.
"""
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(HERE, '_build')
LIB = os.path.join(HERE, 'liblbmib.so')
ARCH = 'gfx950'

HIP_FLAGS = ['-O3', '-std=c++17', '-fPIC', f'--offload-arch={ARCH}', '-munsafe-fp-atomics',
             '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops', '-Wno-unused-result']
HOST_FLAGS = ['-O2', '-std=c++17', '-fPIC', '-ffp-contract=off']
HIP_SOURCES = ['sweep_split.hip', 'sweep_fused.hip', 'outlet.hip', 'refine.hip', 'ib.hip', 'api.hip', 'batch.hip', 'nn.hip', 'learn.hip']
HOST_SOURCES = ['precompute.cpp']


def hipcc():
    for cand in (os.path.join(os.environ.get('ROCM_PATH', '/opt/rocm'), 'bin', 'hipcc'), 'hipcc'):
        if os.path.sep not in cand or os.path.exists(cand):
            return cand
    raise RuntimeError('hipcc not found')


def build(verbose=True):
    """Compile every source and link liblbmib.so. Always recompiles."""
    os.makedirs(BUILD, exist_ok=True)
    cc = hipcc()
    jobs = []
    objs = []
    for src in HIP_SOURCES + HOST_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + '.o')
        flags = HIP_FLAGS if src.endswith('.hip') else HOST_FLAGS
        cmd = [cc] + flags + ['-c', path, '-o', obj]
        jobs.append((src, cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    t0 = time.time()
    failed = []
    for src, cmd, proc in jobs:
        out, _ = proc.communicate()
        if proc.returncode != 0:
            failed.append((src, ' '.join(cmd), out.decode(errors='replace')))
    if failed:
        msg = '\n'.join(f'--- {s}\n{c}\n{o}' for s, c, o in failed)
        raise RuntimeError('HIP build failed:\n' + msg)
    tmp = LIB + '.tmp'
    link = [cc, '-shared', '-fPIC', f'--offload-arch={ARCH}'] + objs + ['-o', tmp]
    res = subprocess.run(link, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if res.returncode != 0:
        raise RuntimeError('link failed:\n' + ' '.join(link) + '\n' + res.stdout.decode(errors='replace'))
    os.replace(tmp, LIB)
    if verbose:
        print(f'built {LIB} in {time.time() - t0:.1f} s', file=sys.stderr)
    return LIB


if __name__ == '__main__':
    build()
