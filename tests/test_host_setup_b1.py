"""The C++ host setup of Problem B.1 (-C(d_t u, psi) in the third equation) against the oracle,
entry by entry, on the CPU: slab operator, spatial MM and KK, the boundary part of C that the
right-hand side's jump needs, and the closed-form sizes."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import problem
from tests import hostlib

LIB = hostlib.load()
LIB.stgmg_host_set_pressure.argtypes = [ctypes.c_int]
LIB.stgmg_host_set_form.argtypes = [ctypes.c_int]


@pytest.fixture(params=['cont', 'disc'])
def pressure(request):
    LIB.stgmg_host_set_pressure(1 if request.param == 'disc' else 0)
    LIB.stgmg_host_set_form(1)
    yield request.param
    LIB.stgmg_host_set_pressure(0)
    LIB.stgmg_host_set_form(0)


def build(d, N, r, k, kind, prm, tau=0.05):
    K = np.broadcast_to(np.asarray(prm.K, dtype=float), (N ** d,)).copy()
    n = LIB.stgmg_host_build(d, r, k, N, 1 if kind == 'vertex' else 0, tau, 0.7, prm.rho, prm.lam, prm.mu,
                             prm.alpha, prm.c0, hostlib.ptr(K))
    assert n > 0
    return n


@pytest.mark.parametrize("d,N,r,k", [(2, 3, 2, 1), (2, 2, 3, 2), (3, 2, 2, 1)])
def test_operator_and_boundary_c_match_oracle(pressure, d, N, r, k):
    rng = np.random.default_rng(13)
    prm = problem.Params(rho=1.3, lam=2.5, mu=0.8, alpha=0.7, c0=0.02, K=np.exp(rng.standard_normal(N ** d)),
                         pressure=pressure, form='dtu')
    n = build(d, N, r, k, 'cell', prm)
    blocks = problem.SpaceBlocks(d, N, r, prm)
    ref = problem.slab_operator(blocks, k, 0.05)
    A = hostlib.csr(LIB, 0, n)
    diff = abs(A - ref)
    tol = 1e-13 * abs(ref).max(axis=1).toarray().ravel() + 1e-15 * abs(ref).max()
    assert (diff.max(axis=1).toarray().ravel() <= tol).all()
    for which, M in ((1, blocks.MM), (3, blocks.KK)):
        H = hostlib.csr(LIB, which, blocks.ns)
        assert abs(H - M).max() <= 1e-13 * abs(M).max()
    # boundary-face part of C: C minus its volume part
    nnz = LIB.stgmg_host_nnz(4)
    p = np.zeros(blocks.nP + 1, dtype=np.int64)
    c = np.zeros(nnz, dtype=np.int32)
    v = np.zeros(nnz)
    LIB.stgmg_host_csr(4, hostlib.ptr(p), hostlib.ptr(c), hostlib.ptr(v))
    Cf = sp.csr_matrix((v, c, p), shape=(blocks.nP, blocks.nv))
    Cref = blocks.C - blocks.Cv
    assert abs(Cf - Cref).max() <= 1e-14 * abs(blocks.C).max()


@pytest.mark.parametrize("d,r,k,N,kind", [(2, 2, 1, 4, 'cell'), (2, 2, 2, 4, 'vertex'), (3, 2, 1, 2, 'cell'),
                                          (2, 3, 1, 2, 'vertex')])
def test_closed_form_sizes(pressure, d, r, k, N, kind):
    prm = problem.Params(pressure=pressure, form='dtu')
    n = build(d, N, r, k, kind, prm)
    S = hostlib.sizes(LIB, d, r, k, N, 1 if kind == 'vertex' else 0)
    assert S['n'] == n
    assert S['nnzA'] == LIB.stgmg_host_nnz(0)
    assert S['nnzMM'] == LIB.stgmg_host_nnz(1)
    assert S['nnzKK'] == LIB.stgmg_host_nnz(3)
    assert S['nnzCface'] == LIB.stgmg_host_nnz(4)
