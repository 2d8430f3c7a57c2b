"""bench.py without a GPU: a run on more than one GPU is refused with a message (the library has
no multi-GPU path) and exit status 2; the key of the HBM-counter records follows the code of the
kernel source, not its comments."""
import importlib.util
import json
import os
import shutil
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, 'bench.py'), '--gpus', '2', '--steps', '1'],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert 'one GPU' in r.stderr
    assert r.stdout.strip() == ''


def _bench_in(root):
    spec = importlib.util.spec_from_file_location('bench_copy', os.path.join(root, 'bench.py'))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_counter_records_follow_the_code(tmp_path):
    """A comment edit keeps kernel_source_hash (and so the recorded traffic); a code edit changes it
    and the record no longer applies."""
    csrc = tmp_path / 'paper_2303_06742_amd' / 'csrc'
    csrc.mkdir(parents=True)
    (tmp_path / 'profiles').mkdir()
    shutil.copy(os.path.join(ROOT, 'bench.py'), tmp_path / 'bench.py')
    src = open(os.path.join(ROOT, 'paper_2303_06742_amd', 'csrc', 'kernels.hip')).read()
    (csrc / 'kernels.hip').write_text(src)
    b = _bench_in(str(tmp_path))
    h0 = b.kernel_source_hash()
    rec = {'workload': '2d-256x256-dg2-vertex', 'precision': 'fp64', 'role': 'patch', 'kernels_hip_sha256': h0,
           'bytes_per_launch': 123}
    (tmp_path / 'profiles' / 'hbm_traffic.json').write_text(json.dumps({'entries': [rec]}))
    assert b.measured_traffic(rec['workload'], rec['precision'], rec['role']) == 123
    (csrc / 'kernels.hip').write_text(src.replace('// ', '//  ', 3) + '\n// a note\n\n')
    assert b.kernel_source_hash() == h0
    (csrc / 'kernels.hip').write_text(src.replace('constexpr int RED_MAXB = 2;', 'constexpr int RED_MAXB = 3;'))
    assert b.kernel_source_hash() != h0
    assert b.measured_traffic(rec['workload'], rec['precision'], rec['role']) is None
