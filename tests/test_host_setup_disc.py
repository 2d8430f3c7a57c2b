"""The C++ host setup with the discontinuous pressure pair Q_r^d / P_{r-1}^disc (interior
penalty form of Def:B) against the oracle, entry by entry, on the CPU."""
import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import gmg, problem
from tests import hostlib
from paper_2303_06742_amd import workloads

LIB = hostlib.load()
LIB.stgmg_host_set_pressure.argtypes = [ctypes.c_int]


@pytest.fixture(autouse=True)
def disc_mode():
    LIB.stgmg_host_set_pressure(1)
    yield
    LIB.stgmg_host_set_pressure(0)


def build(d, N, r, k, kind, prm, tau=0.01, omega=0.7):
    K = np.broadcast_to(np.asarray(prm.K, dtype=float), (N ** d,)).copy()
    n = LIB.stgmg_host_build(d, r, k, N, 1 if kind == 'vertex' else 0, tau, omega, prm.rho, prm.lam, prm.mu,
                             prm.alpha, prm.c0, hostlib.ptr(K))
    assert n > 0
    return n


@pytest.mark.parametrize("d,N,r,k", [(2, 2, 2, 1), (2, 3, 2, 2), (2, 3, 3, 1), (3, 2, 2, 1), (2, 2, 4, 0)])
def test_operator_matches_oracle(d, N, r, k):
    rng = np.random.default_rng(11)
    prm = problem.Params(rho=1.3, lam=2.5, mu=0.8, alpha=0.7, c0=0.02, K=np.exp(rng.standard_normal(N ** d)),
                         pressure='disc')
    n = build(d, N, r, k, 'cell', prm, tau=0.05)
    A = hostlib.csr(LIB, 0, n)
    blocks = problem.SpaceBlocks(d, N, r, prm)
    ref = problem.slab_operator(blocks, k, 0.05)
    assert A.shape == ref.shape
    diff = abs(A - ref)
    scale = abs(ref).max(axis=1).toarray().ravel()
    # rounding: 1e-13 of the row, plus 1e-15 of the largest (Nitsche penalty) entries,
    # which enter sums whose results can be much smaller
    tol = 1e-13 * scale + 1e-15 * abs(ref).max()
    assert (diff.max(axis=1).toarray().ravel() <= tol).all()
    # the spatial MM and KK the factored operator and the patch setup use
    ns = blocks.ns
    for which, M in ((1, blocks.MM), (3, blocks.KK)):
        H = hostlib.csr(LIB, which, ns)
        assert abs(H - M).max() <= 1e-13 * abs(M).max()


@pytest.mark.parametrize("kind", ["cell", "vertex"])
@pytest.mark.parametrize("d,N,k,r", [(2, 3, 1, 2), (3, 2, 1, 2), (2, 2, 2, 3)])
def test_patches_match_oracle(kind, d, N, k, r):
    prm = problem.Params(pressure='disc')
    n = build(d, N, r, k, kind, prm, omega=0.7)
    npatch = LIB.stgmg_host_npatch()
    poff = np.zeros(npatch + 1, dtype=np.int64)
    pdof = np.zeros(LIB.stgmg_host_patch_total(), dtype=np.int32)
    winv = np.zeros(n)
    LIB.stgmg_host_patches(hostlib.ptr(poff), hostlib.ptr(pdof), hostlib.ptr(winv))
    blocks = problem.SpaceBlocks(d, N, r, prm)
    cells = gmg.patch_cells(blocks.mesh, kind)
    assert len(cells) == npatch
    cnt = np.zeros(n)
    for q, c in enumerate(cells):
        Z = gmg.patch_dofs(blocks, k, c)
        assert np.array_equal(pdof[poff[q]:poff[q + 1]], Z)
        cnt[Z] += 1
    assert np.allclose(winv, 0.7 / cnt, rtol=1e-15)


@pytest.mark.parametrize("d,r,k,Nc", [(2, 2, 1, 2), (2, 3, 0, 1), (3, 2, 1, 1), (2, 4, 1, 2)])
def test_prolongation_matches_oracle(d, r, k, Nc):
    nnz = LIB.stgmg_host_prolongation(d, r, k, Nc)
    assert nnz > 0
    prm = problem.Params(pressure='disc')
    ref = gmg.prolongation(problem.SpaceBlocks(d, Nc, r, prm), problem.SpaceBlocks(d, 2 * Nc, r, prm), k)
    ref.eliminate_zeros()
    p = np.zeros(ref.shape[0] + 1, dtype=np.int64)
    c = np.zeros(nnz, dtype=np.int32)
    v = np.zeros(nnz)
    LIB.stgmg_host_csr(2, hostlib.ptr(p), hostlib.ptr(c), hostlib.ptr(v))
    P = sp.csr_matrix((v, c, p), shape=ref.shape)
    assert abs(P - ref).max() < 1e-14
    assert P.nnz == ref.nnz


@pytest.mark.parametrize("d,N,r,K", [(2, 3, 2, None), (3, 2, 2, 'hetero'), (2, 2, 3, 'hetero')])
def test_source_and_projection_match_oracle(d, N, r, K):
    rng = np.random.default_rng(1)
    Kc = np.exp(rng.standard_normal(N ** d)) if K else 1.0
    prm = problem.Params(rho=1.2, lam=1.5, mu=0.9, alpha=0.8, c0=0.03, K=Kc, pressure='disc')
    build(d, N, r, 1, 'cell', prm)
    blocks = problem.SpaceBlocks(d, N, r, prm)
    sol = problem.ExactSolution(d, *workloads.builtin_solution_exprs(d), prm)
    for t in (0.0, 0.37):
        out = np.zeros(blocks.ns)
        LIB.stgmg_host_source(t, prm.rho, prm.lam, prm.mu, prm.alpha, prm.c0, hostlib.ptr(out))
        ref = problem.source_vector(blocks, sol, t)
        # as for the continuous pressure: the oracle's Nitsche data terms of the (zero)
        # boundary values leave ~1e-11 of rounding
        assert np.abs(out - ref).max() < 1e-10 * np.abs(ref).max()
        LIB.stgmg_host_interpolate(t, hostlib.ptr(out))
        assert np.abs(out - problem.interpolate(blocks, sol, t)).max() < 1e-14


@pytest.mark.parametrize("d,r,k,N,kind", [(2, 2, 1, 4, 'cell'), (2, 2, 2, 4, 'vertex'), (2, 3, 1, 2, 'vertex'),
                                          (3, 2, 1, 2, 'cell'), (3, 2, 2, 2, 'vertex'), (2, 2, 0, 1, 'vertex'),
                                          (2, 4, 1, 2, 'cell')])
def test_closed_form_sizes(d, r, k, N, kind):
    prm = problem.Params(pressure='disc')
    n = build(d, N, r, k, kind, prm)
    S = hostlib.sizes(LIB, d, r, k, N, 1 if kind == 'vertex' else 0)
    assert S['n'] == n
    assert S['nnzA'] == LIB.stgmg_host_nnz(0)
    assert S['nnzMM'] == LIB.stgmg_host_nnz(1)
    assert S['nnzKK'] == LIB.stgmg_host_nnz(3)
    assert S['npatch'] == LIB.stgmg_host_npatch() and S['sum_np'] == LIB.stgmg_host_patch_total()
    poff = np.zeros(S['npatch'] + 1, dtype=np.int64)
    pdof = np.zeros(LIB.stgmg_host_patch_total(), dtype=np.int32)
    LIB.stgmg_host_patches(hostlib.ptr(poff), hostlib.ptr(pdof), hostlib.ptr(np.zeros(n)))
    npp = np.diff(poff)
    assert S['max_np'] == npp.max() and S['sum_np_ld'] == int(np.sum(npp * ((npp + 3) // 4 * 4)))
    if N >= 2 and N % 2 == 0:
        assert S['nnzP'] == LIB.stgmg_host_prolongation(d, r, k, N // 2)
