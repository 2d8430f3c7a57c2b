"""Helpers for the GPU tests: device transfer and oracle hierarchies of a config."""
import functools

import numpy as np
import pytest


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def to_host(t):
    return t.detach().cpu().numpy()


@functools.lru_cache(maxsize=8)
def oracle_hierarchy(cfg_key):
    from oracle import gmg, problem
    cfg = CONFIGS[cfg_key]
    K = cfg.K_cells()
    prm = problem.Params(rho=cfg.rho, lam=cfg.lam, mu=cfg.mu, alpha=cfg.alpha, c0=cfg.c0,
                         K=cfg.K if K is None else K)
    # coarse levels take the mean of the children's K, as the library does
    H = gmg.Hierarchy(cfg.dim, cfg.coarse_cells, cfg.levels - 1, cfg.r, cfg.k, cfg.tau, prm,
                      patch_kind=cfg.patch, J=cfg.n_smooth, omega=cfg.omega) if K is None else \
        hetero_hierarchy(cfg, prm, K)
    return H


def hetero_hierarchy(cfg, prm, Kfine):
    """Hierarchy with per-cell K: the oracle's levels are rebuilt with the averaged K."""
    from oracle import gmg, problem
    d = cfg.dim
    Ks = [Kfine]
    for _ in range(cfg.levels - 1):
        Nf = int(round(len(Ks[0]) ** (1.0 / d)))
        Kf = Ks[0].reshape((Nf,) * d)  # index order: [z][y][x]
        Kc = Kf.reshape(*([Nf // 2, 2] * d)).mean(axis=tuple(range(1, 2 * d, 2)))
        Ks.insert(0, Kc.reshape(-1))
    H = gmg.Hierarchy.__new__(gmg.Hierarchy)
    H.J, H.omega = cfg.n_smooth, cfg.omega
    H.levels = []
    for l in range(cfg.levels):
        p = problem.Params(rho=prm.rho, lam=prm.lam, mu=prm.mu, alpha=prm.alpha, c0=prm.c0, K=Ks[l])
        H.levels.append(gmg.Level(d, cfg.coarse_cells * 2 ** l, cfg.r, cfg.k, cfg.tau, p, cfg.patch))
    for lev in H.levels[1:]:
        lev.build_smoother()
    H.P = [None] + [gmg.prolongation(H.levels[l - 1].prob.blocks, H.levels[l].prob.blocks, cfg.k)
                    for l in range(1, cfg.levels)]
    import scipy.linalg as sla
    A0 = H.levels[0].A.toarray()
    H.coarse_scale = 1.0 / np.abs(A0).max(axis=1)
    H.coarse_lu = sla.lu_factor(H.coarse_scale[:, None] * A0)
    return H


from paper_2303_06742_amd import workloads as W  # noqa: E402

CONFIGS = {
    'c1': W.C1,
    'c2s': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex'),          # C2 physics, 16^2, 3 levels
    'c2s_cell': W.scaled(W.C2, 3, name='2d-16x16-dg2-cell', patch='cell'),
    'c3s': W.scaled(W.C3, 2, name='3d-8cube-dg1-cell-lognormal'),   # C3 physics, 8^3, 2 levels
    'k0': W.scaled(W.C1, 2, name='2d-8x8-dg0-vertex', k=0, patch='vertex'),
    'one_level': W.scaled(W.C1, 1, name='2d-4x4-dg1-direct'),
}
