"""Edge cases and error paths of the C ABI on the GPU."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import CONFIGS, require_gpu, to_dev, to_host
from paper_2303_06742_amd import workloads

pytestmark = pytest.mark.gpu


def capi():
    require_gpu()
    from paper_2303_06742_amd import capi as c
    return c


def test_invalid_params_rejected():
    c = capi()
    p = c.Params(dim=4, coarse_cells=2, levels=2, r=2, k=1, patch=0, smoother_prec=0, n_smooth=4, omega=0.7,
                 tau=0.01, rho=1, lam=1, mu=1, alpha=0.9, c0=0.01, K=1.0, K_cells=None)
    h = ctypes.c_void_p()
    assert c.stgmg_setup(ctypes.byref(p), None, ctypes.byref(h)) == c.STGMG_ERR_INVALID_ARG
    assert b"dim" in c.stgmg_last_error()
    p.dim, p.k = 2, 7
    assert c.stgmg_setup(ctypes.byref(p), None, ctypes.byref(h)) == c.STGMG_ERR_UNSUPPORTED
    p.k, p.tau = 1, -1.0
    assert c.stgmg_setup(ctypes.byref(p), None, ctypes.byref(h)) == c.STGMG_ERR_INVALID_ARG


def test_solve_edge_cases():
    c = capi()
    S = c.Solver(CONFIGS['c1'])
    n = S.n
    # zero right-hand side: x stays zero, converged, no iterations
    x = S.empty()
    info = S.solve(S.empty(), x)
    assert info['converged'] == 1 and info['iters'] == 0 and float(x.abs().max()) == 0.0
    # NaN in the right-hand side
    F = workloads.random_vector(n, 1)
    F[5] = np.nan
    with pytest.raises(c.StgmgError) as e:
        S.solve(to_dev(F), S.empty())
    assert e.value.status == c.STGMG_ERR_NONFINITE
    # iteration cap: not converged, x holds the last iterate
    F = workloads.random_vector(n, 2)
    x = S.empty()
    info = S.solve(to_dev(F), x, rtol=1e-14, max_iters=1)
    assert info['converged'] == 0 and info['iters'] == 1 and info['rel_res_true'] < 1.0
    # warm start: the initial residual reported is that of x0 (the previous solution)
    x2 = x.clone()
    info = S.solve(to_dev(F), x2, rtol=1e-8)
    info2 = S.solve(to_dev(F), x2, rtol=1e-8)
    assert info2['res0'] <= 1e-8 * info['res0'] * (1 + 1e-6)
    # bad level index and wrong sizes
    assert c.stgmg_apply_operator(S.h, 9, ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(x.data_ptr())) == c.STGMG_ERR_INVALID_ARG
    with pytest.raises(ValueError):
        S.solve(to_dev(np.zeros(n + 1)), S.empty())
    S.close()


def test_restart_short_cycles():
    """Restart length 2: more cycles, same answer to the tolerance."""
    c = capi()
    S = c.Solver(CONFIGS['c1'])
    F = to_dev(workloads.random_vector(S.n, 3))
    a, b = S.empty(), S.empty()
    ia = S.solve(F, a, restart=30)
    ib = S.solve(F, b, restart=2)
    assert ia['converged'] and ib['converged']
    d = np.abs(to_host(a) - to_host(b)).max() / np.abs(to_host(a)).max()
    assert d < 1e-6


def test_bad_pointers_rejected_before_launch():
    """Vector arguments are checked before anything is enqueued: NULL is INVALID_ARG; pinned host
    memory, pageable host memory and a misaligned device address are BAD_POINTER.  The handle
    stays usable afterwards."""
    import torch
    c = capi()
    S = c.Solver(CONFIGS['c1'])
    n = S.n
    x = S.empty()
    y = S.empty()
    dp = lambda t: ctypes.c_void_p(t.data_ptr())  # noqa: E731
    assert c.stgmg_apply_operator(S.h, -1, None, dp(y)) == c.STGMG_ERR_INVALID_ARG
    pinned = torch.zeros(n, dtype=torch.float64).pin_memory()
    assert c.stgmg_apply_operator(S.h, -1, dp(pinned), dp(y)) == c.STGMG_ERR_BAD_POINTER
    assert b"device memory" in c.stgmg_last_error()
    host = np.zeros(n)
    assert c.stgmg_apply_vcycle(S.h, host.ctypes.data_as(ctypes.c_void_p), dp(y)) == c.STGMG_ERR_BAD_POINTER
    buf = S.empty(n + 1)
    mis = ctypes.c_void_p(buf.data_ptr() + 4)
    assert c.stgmg_apply_operator(S.h, -1, dp(x), mis) == c.STGMG_ERR_BAD_POINTER
    assert b"aligned" in c.stgmg_last_error()
    info = c.Info()
    assert c.stgmg_solve(S.h, dp(pinned), dp(x), 1e-8, 30, 100, ctypes.byref(info)) == c.STGMG_ERR_BAD_POINTER
    assert c.stgmg_solve(S.h, dp(x), dp(x), 1e-8, 30, 100, ctypes.byref(info)) == c.STGMG_ERR_INVALID_ARG
    # still usable
    F = to_dev(workloads.random_vector(n, 5))
    info = S.solve(F, x)
    assert info['converged'] == 1
    assert 0.0 < info['t_vcycle_ms'] <= info['t_solve_ms']
    S.close()


def test_invalid_waves_rejected():
    c = capi()
    p, _K = c.make_params(CONFIGS['c1'], waves=3)
    h = ctypes.c_void_p()
    assert c.stgmg_setup(ctypes.byref(p), None, ctypes.byref(h)) == c.STGMG_ERR_INVALID_ARG
    assert b"waves_per_patch" in c.stgmg_last_error()


@pytest.mark.parametrize("key", ['c2s', 'c1_full', 'c1_tb', 'c2d', 'c3v'])
def test_singular_patch_reported(key, monkeypatch):
    """A patch block with a zero pivot (zeroed on the device by the setup's test hook) makes
    stgmg_setup return SINGULAR_PATCH naming the patch; the inversion kernel flags the pivot and
    finishes normally, and a following setup without the hook succeeds."""
    c = capi()
    monkeypatch.setenv('STGMG_TEST_ZERO_PATCH', '3')
    with pytest.raises(c.StgmgError) as e:
        c.Solver(CONFIGS[key])
    assert e.value.status == c.STGMG_ERR_SINGULAR_PATCH
    assert 'patch 3 ' in str(e.value)
    monkeypatch.delenv('STGMG_TEST_ZERO_PATCH')
    S = c.Solver(CONFIGS[key])
    info = S.solve(to_dev(workloads.random_vector(S.n, 6)), S.empty())
    assert info['converged'] == 1
    S.close()
