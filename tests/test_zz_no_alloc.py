"""stgmg_solve_noalloc (FGMRES workspace in the library's static device array) against
stgmg_solve on the same handles: two calls in a row, the second on a smaller problem, and the
size limit of the static workspace."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import CONFIGS, require_gpu, to_dev, to_host
from paper_2303_06742_amd import workloads

pytestmark = pytest.mark.gpu


def _capi():
    require_gpu()
    from paper_2303_06742_amd import capi
    return capi


def _solve_noalloc(c, S, F, x, rtol=1e-8, restart=30):
    info = c.Info()
    st = c.stgmg_solve_noalloc(S.h, ctypes.c_void_p(F.data_ptr()), ctypes.c_void_p(x.data_ptr()), rtol, restart,
                               1000, ctypes.byref(info))
    return st, info.as_dict()


def test_noalloc_matches_solve_twice_then_smaller():
    c = _capi()
    big = c.Solver(CONFIGS['c2s'])
    small = c.Solver(CONFIGS['c1'])
    for S, seed in ((big, 81), (small, 82)):
        print(f"[noalloc] {S.cfg.name} n={S.n}", flush=True)
        F = to_dev(workloads.random_vector(S.n, seed))
        x_ref = S.empty()
        i_ref = S.solve(F, x_ref)
        x = S.empty()
        st, info = _solve_noalloc(c, S, F, x)
        assert st == c.STGMG_OK, c.stgmg_last_error()
        assert info['converged'] == 1 and info['iters'] == i_ref['iters']
        # the same kernels in the same order on a different workspace: the same bits
        assert np.array_equal(to_host(x), to_host(x_ref))
    big.close()
    small.close()


def test_noalloc_rejects_workspace_beyond_the_static_array():
    c = _capi()
    S = c.Solver(CONFIGS['c1'])
    F = to_dev(workloads.random_vector(S.n, 83))
    x = S.empty()
    # (2 restart + 2) n doubles must fit in STGMG_NOALLOC_SCRATCH_BYTES: c1 has 2,474 unknowns
    st, _ = _solve_noalloc(c, S, F, x, restart=30)
    assert st == c.STGMG_OK
    S.close()
    big = c.Solver(CONFIGS['c2_64'])  # 212,367 unknowns: restart 100 needs about 343 MB
    F = to_dev(workloads.random_vector(big.n, 84))
    x = big.empty()
    st, _ = _solve_noalloc(c, big, F, x, restart=100)
    assert st == c.STGMG_ERR_UNSUPPORTED
    assert b"static scratch" in c.stgmg_last_error()
    assert float(x.abs().max()) == 0.0  # nothing was run
    st, info = _solve_noalloc(c, big, F, x, restart=30)
    assert st == c.STGMG_OK and info['converged'] == 1
    big.close()
