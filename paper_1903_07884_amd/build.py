"""Build libvie.so (HIP for gfx950) in-tree with hipcc.

Usage: python -m paper_1903_07884_amd.build   (or build() from Python)
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, 'csrc')
LIB = os.path.join(HERE, 'libvie.so')
SOURCES = ['api.cpp', 'fft_host.cpp', 'profile.cpp', 'tune.cpp', 'generator.hip', 'matvec.hip', 'precond.hip', 'block_solve.hip', 'krylov.hip', 'serve.cpp']


def hipcc():
    exe = shutil.which('hipcc') or '/opt/rocm/bin/hipcc'
    if not os.path.exists(exe):
        raise RuntimeError('hipcc not found')
    return exe


def build(verbose=False, jobs=8):
    """Compile every source for gfx950 and link libvie.so next to this file."""
    objdir = os.path.join(HERE, '_build')
    os.makedirs(objdir, exist_ok=True)
    common = ['--offload-arch=gfx950', '-O3', '-fPIC', '-std=c++17', '-Wall', '-Wno-unused-function',
              '-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops',
              '-I', os.path.join(HERE, '..', 'include')]
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + '.o')
        objs.append(obj)
        lang = ['-x', 'hip'] if src.endswith('.hip') else ['-x', 'hip']
        cmd = [hipcc()] + common + lang + ['-c', os.path.join(CSRC, src), '-o', obj]
        if verbose:
            print(' '.join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len([p for _, p in procs if p.poll() is None]) >= jobs:
            procs[0][1].wait()
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors='replace')
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            print(text)
    if failed:
        msg = '\n'.join('== %s ==\n%s' % f for f in failed)
        raise RuntimeError('HIP build failed:\n' + msg)
    tmp = LIB + '.tmp'
    cmd = [hipcc(), '--offload-arch=gfx950', '-shared', '-fPIC', '-o', tmp] + objs
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError('link failed:\n' + r.stdout.decode(errors='replace'))
    os.replace(tmp, LIB)
    return LIB


if __name__ == '__main__':
    print(build(verbose='-v' in sys.argv))
