"""The node-pair form of the velocity rows of the level operator (the data of the device's
structured residual kernel), extracted on the host from the spatial MM and KK: its products
equal the CSR products, and its sizes equal the closed-form counts of the footprint."""
import numpy as np
import pytest

from oracle import problem
from tests import hostlib

LIB = hostlib.load()

CASES = [  # d, N, r, k, pressure, form
    (2, 4, 2, 1, 'cont', 'v'), (2, 3, 2, 2, 'cont', 'v'), (2, 4, 3, 2, 'disc', 'v'), (2, 3, 2, 1, 'cont', 'dtu'),
    (2, 2, 4, 3, 'cont', 'v'), (3, 2, 2, 1, 'cont', 'v'), (3, 2, 2, 1, 'disc', 'dtu'), (2, 4, 2, 0, 'cont', 'v')]


@pytest.mark.parametrize("d,N,r,k,pressure,form", CASES)
def test_node_form_reproduces_velocity_rows(d, N, r, k, pressure, form):
    rng = np.random.default_rng(11)
    prm = problem.Params(rho=1.3, lam=2.5, mu=0.8, alpha=0.7, c0=0.02, K=np.exp(rng.standard_normal(N ** d)))
    LIB.stgmg_host_set_pressure(1 if pressure == 'disc' else 0)
    LIB.stgmg_host_set_form(1 if form == 'dtu' else 0)
    try:
        K = np.asarray(prm.K, dtype=float)
        n = LIB.stgmg_host_build(d, r, k, N, 0, 0.05, 0.7, prm.rho, prm.lam, prm.mu, prm.alpha, prm.c0,
                                 hostlib.ptr(K))
        assert n > 0
        ns = n // (k + 1)
        nQ = (r * N + 1) ** d
        nv = d * nQ
        MM = hostlib.csr(LIB, 1, ns)
        KK = hostlib.csr(LIB, 3, ns)
        node = hostlib.node_op(LIB, nQ, d)
        S = hostlib.sizes(LIB, d, r, k, N, 0)
    finally:
        LIB.stgmg_host_set_pressure(0)
        LIB.stgmg_host_set_form(0)
    assert node is not None
    assert len(node['col']) == S['nodeQQ'] and len(node['ccol']) == S['nodeQP']
    x = rng.standard_normal(ns)
    V, U, P = x[:nv].reshape(nQ, d), x[nv:2 * nv].reshape(nQ, d), x[2 * nv:]
    mu_ = np.zeros((nQ, d))
    ku = np.zeros((nQ, d))
    mv = np.zeros((nQ, d))
    kv = np.zeros((nQ, d))
    A = node['a'].reshape(-1, d, d)
    C = node['c'].reshape(-1, d)
    for i in range(nQ):
        s, e = node['ptr'][i], node['ptr'][i + 1]
        j, m = node['col'][s:e], node['m'][s:e]
        mu_[i] = m @ U[j]
        ku[i] = -(m @ V[j])
        mv[i] = m @ V[j]
        kv[i] = np.einsum('tcd,td->c', A[s:e], U[j])
        cs, ce = node['cptr'][i], node['cptr'][i + 1]
        kv[i] += C[cs:ce].T @ P[node['ccol'][cs:ce]]
    for got, Mat, rows in ((mu_, MM, slice(0, nv)), (ku, KK, slice(0, nv)), (mv, MM, slice(nv, 2 * nv)),
                           (kv, KK, slice(nv, 2 * nv))):
        ref = (Mat @ x)[rows]
        bound = (abs(Mat) @ abs(x))[rows]
        assert np.all(np.abs(got.ravel() - ref) <= 1e-14 * bound + 1e-300)
