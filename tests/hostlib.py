"""ctypes access to the host-only setup library (assembly, patches, transfers)."""
import ctypes
import os

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PATH = os.path.join(ROOT, 'paper_2303_06742_amd', 'libstgmg_host.so')


def load():
    if not os.path.exists(PATH):
        from paper_2303_06742_amd import build
        build.build_host()
    lib = ctypes.CDLL(PATH)
    D, I, LL, P = ctypes.c_double, ctypes.c_int, ctypes.c_longlong, ctypes.c_void_p
    lib.stgmg_host_build.restype = LL
    lib.stgmg_host_build.argtypes = [I, I, I, I, I, D, D, D, D, D, D, D, P]
    lib.stgmg_host_nnz.restype = LL
    lib.stgmg_host_nnz.argtypes = [I]
    lib.stgmg_host_csr.argtypes = [I, P, P, P]
    lib.stgmg_host_npatch.restype = LL
    lib.stgmg_host_patch_total.restype = LL
    lib.stgmg_host_patches.argtypes = [P, P, P]
    lib.stgmg_host_prolongation.restype = LL
    lib.stgmg_host_prolongation.argtypes = [I, I, I, I]
    lib.stgmg_host_time.argtypes = [I, D, P, P, P, P, P]
    lib.stgmg_host_source.argtypes = [D, D, D, D, D, D, P]
    lib.stgmg_host_interpolate.argtypes = [D, P]
    lib.stgmg_host_sym_slot_elem.restype = LL
    lib.stgmg_host_sym_slot_elem.argtypes = [I, I, I, I]
    return lib


def ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def csr(lib, which, nrows):
    import scipy.sparse as sp
    nnz = lib.stgmg_host_nnz(which)
    p = np.zeros(nrows + 1, dtype=np.int64)
    c = np.zeros(nnz, dtype=np.int32)
    v = np.zeros(nnz)
    lib.stgmg_host_csr(which, ptr(p), ptr(c), ptr(v))
    return sp.csr_matrix((v, c, p), shape=(nrows, nrows if which != 2 else int(c.max()) + 1 if nnz else 0))


def sizes(lib, d, r, k, N, kind):
    out = np.zeros(19, dtype=np.int64)
    lib.stgmg_host_sizes.argtypes = [ctypes.c_int] * 5 + [ctypes.c_void_p]
    lib.stgmg_host_sizes(d, r, k, N, kind, ptr(out))
    return dict(zip(['n', 'nnzA', 'nnzMM', 'nnzP', 'npatch', 'sum_np', 'sum_np_ld', 'max_np', 'nnzKK',
                    'sum_red_fixed', 'sum_nr_ldr', 'max_nr', 'max_nn', 'nnzCface', 'sum_tiles', 'sum_tiles2',
                    'nodeQQ', 'nodeQP', 'sum_tiles4'], out.tolist()))


def node_op(lib, nQ, d):
    """The node-pair form of the velocity rows of the last built level, or None."""
    lib.stgmg_host_node_build.restype = ctypes.c_longlong
    lib.stgmg_host_node_cnnz.restype = ctypes.c_longlong
    lib.stgmg_host_node_arrays.argtypes = [ctypes.c_void_p] * 7
    nnz = lib.stgmg_host_node_build()
    if nnz < 0:
        return None
    cnnz = lib.stgmg_host_node_cnnz()
    out = dict(ptr=np.zeros(nQ + 1, dtype=np.int64), col=np.zeros(nnz, dtype=np.int32), m=np.zeros(nnz),
               a=np.zeros(nnz * d * d), cptr=np.zeros(nQ + 1, dtype=np.int64), ccol=np.zeros(cnnz, dtype=np.int32),
               c=np.zeros(cnnz * d))
    lib.stgmg_host_node_arrays(*[ptr(out[k]) for k in ('ptr', 'col', 'm', 'a', 'cptr', 'ccol', 'c')])
    return out
