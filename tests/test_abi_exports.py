"""The C-ABI library loads without a GPU and exports every function include/stgmg.h declares
(no compute calls here), and the ctypes binding names exactly those functions."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, 'include', 'stgmg.h')
LIB = os.path.join(ROOT, 'paper_2303_06742_amd', 'libstgmg.so')


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r'/\*.*?\*/', ' ', text, flags=re.S)  # comments
    return sorted(set(re.findall(r'\b(stgmg_[a-z0-9_]+)\s*\(', text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ('stgmg_setup', 'stgmg_solve', 'stgmg_solve_noalloc', 'stgmg_destroy', 'stgmg_solve_batch',
                 'stgmg_server_submit', 'stgmg_status_string', 'stgmg_last_error'):
        assert must in names
    assert len(names) >= 20


def test_library_exports_every_declared_function():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    src = open(os.path.join(ROOT, 'paper_2303_06742_amd', 'capi.py')).read()
    listed = set(re.findall(r"'(stgmg_[a-z0-9_]+)'", src[src.index('EXPORTED'):]))
    assert listed == set(declared_functions())
