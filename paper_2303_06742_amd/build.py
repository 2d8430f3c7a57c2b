"""Build the HIP library libstgmg.so for gfx950 with hipcc (in-tree)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, 'csrc')
BUILD = os.path.join(ROOT, '_build')
LIB = os.path.join(HERE, 'libstgmg.so')
HOSTLIB = os.path.join(HERE, 'libstgmg_host.so')  # host-only setup code, for CPU tests

HIPCC = os.environ.get('HIPCC', '/opt/rocm/bin/hipcc')
ARCH = '--offload-arch=gfx950'
COMMON = ['-O3', '-std=c++17', '-fPIC', '-I', os.path.join(ROOT, 'include'), '-I', CSRC]
# packed FP32 instructions are disabled for all device code
DEVICE = ['-Xclang', '-target-feature', '-Xclang', '-packed-fp32-ops']

SOURCES = [
    ('host_setup.cpp', False),
    ('kernels.hip', True),
    ('gj_mfma.hip', True),
    ('source.hip', True),
    ('api.hip', True),
    ('server.cpp', True),
]


def run(cmd):
    print(' '.join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=True):
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    for src, is_hip in SOURCES:
        obj = os.path.join(BUILD, src + '.o')
        cmd = [HIPCC] + COMMON
        if is_hip:
            cmd += [ARCH] + DEVICE + ['-x', 'hip']
        else:
            cmd += ['-x', 'c++']
        cmd += ['-c', os.path.join(CSRC, src), '-o', obj]
        cmds.append(cmd)
        objs.append(obj)
    # the translation units compile independently
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as ex:
        list(ex.map(run, cmds))
    tmp = LIB + '.tmp'
    run([HIPCC, ARCH, '-shared', '-fPIC', '-o', tmp] + objs + ['-pthread'])
    os.replace(tmp, LIB)
    build_host()
    return LIB


def build_host():
    """Host-only library of the setup code (assembly, patches, transfers) for CPU tests."""
    tmp = HOSTLIB + '.tmp'
    run(['g++', '-O2', '-std=c++17', '-fPIC', '-shared', '-I', CSRC, '-o', tmp,
         os.path.join(CSRC, 'host_setup.cpp'), os.path.join(CSRC, 'host_export.cpp'), '-pthread'])
    os.replace(tmp, HOSTLIB)
    return HOSTLIB


if __name__ == '__main__':
    build()
    sys.exit(0)
