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


def oracle_params(cfg):
    from oracle import problem
    K = cfg.K_cells()
    return problem.Params(rho=cfg.rho, lam=cfg.lam, mu=cfg.mu, alpha=cfg.alpha, c0=cfg.c0,
                          K=cfg.K if K is None else K, pressure=cfg.pressure, form=cfg.form)


def oracle_direct_solve(cfg, F):
    """The oracle's sparse direct solve of the fine-level slab system of a config."""
    from oracle import problem
    prob = problem.SlabProblem(cfg.dim, cfg.fine_cells, cfg.r, cfg.k, cfg.tau, oracle_params(cfg))
    return prob.direct_solve(F), prob.A


@functools.lru_cache(maxsize=64)
def oracle_hierarchy(cfg_key):
    from oracle import gmg
    # the storage of the patch solves does not change the operator
    cfg_key = cfg_key.replace('_full', '').replace('_tb', '').replace('_red', '')
    cfg = CONFIGS[cfg_key]
    prm = oracle_params(cfg)
    return gmg.Hierarchy(cfg.dim, cfg.coarse_cells, cfg.levels - 1, cfg.r, cfg.k, cfg.tau, prm,
                         patch_kind=cfg.patch, J=cfg.n_smooth, omega=cfg.omega)


from paper_2303_06742_amd import workloads as W  # noqa: E402

CONFIGS = {
    'c1': W.C1,
    'c2s': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex'),          # C2 physics, 16^2, 3 levels
    'c2s_cell': W.scaled(W.C2, 3, name='2d-16x16-dg2-cell', patch='cell'),
    'c3s': W.scaled(W.C3, 2, name='3d-8cube-dg1-cell-lognormal'),   # C3 physics, 8^3, 2 levels
    'k0': W.scaled(W.C1, 2, name='2d-8x8-dg0-vertex', k=0, patch='vertex'),
    'k3': W.scaled(W.C1, 2, name='2d-8x8-dg3-cell', k=3),  # two complex eigenvalue pairs
    'one_level': W.scaled(W.C1, 1, name='2d-4x4-dg1-direct'),
    # 3D vertex patches (up to 1,554 rows; reduced solves of 402-row Schur blocks), 4^3 fine
    'c3v': W.scaled(W.C3, 2, name='3d-4cube-dg1-vertex-lognormal', coarse_cells=2, patch='vertex'),
    # the same operators with the full space-time patch inverses
    'c1_full': W.scaled(W.C1, 2, name='2d-8x8-dg1-cell-full', time_blocks=0),
    'c2s_full': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex-full', time_blocks=0),
    'c3s_full': W.scaled(W.C3, 2, name='3d-8cube-dg1-cell-lognormal-full', time_blocks=0),
    # time-block solves without the elimination of the u-equation rows
    'c1_tb': W.scaled(W.C1, 2, name='2d-8x8-dg1-cell-tb', time_blocks=1),
    'c2s_tb': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex-tb', time_blocks=1),
    'c3s_tb': W.scaled(W.C3, 2, name='3d-8cube-dg1-cell-lognormal-tb', time_blocks=1),
    'k0_tb': W.scaled(W.C1, 2, name='2d-8x8-dg0-vertex-tb', k=0, patch='vertex', time_blocks=1),
    # the discontinuous pressure pair with the interior penalty form
    'c1_disc': W.scaled(W.C1, 2, name='2d-8x8-q2p1disc-dg1-cell', pressure='disc'),
    'c2d': W.scaled(W.C2D, 2, name='2d-8x8-q3p2disc-dg2-vertex'),
    'c3s_disc': W.scaled(W.C3, 2, name='3d-8cube-q2p1disc-dg1-cell-lognormal', pressure='disc'),
    'c2d_full': W.scaled(W.C2D, 2, name='2d-8x8-q3p2disc-dg2-vertex-full', time_blocks=0),
    # Problem B.1 (-C(d_t u, psi)): reduced, time-block and full patch solves, both pressure pairs
    'c2s_b1': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex-b1', form='dtu'),
    'c1_b1': W.scaled(W.C1, 2, name='2d-8x8-dg1-cell-b1', form='dtu'),
    # reduced solves with the square (column-major) Schur inverses instead of symmetric tiles
    'c2s_red': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex-red', time_blocks=2),
    'c3s_red': W.scaled(W.C3, 2, name='3d-8cube-dg1-cell-lognormal-red', time_blocks=2),
    'k3_red': W.scaled(W.C1, 2, name='2d-8x8-dg3-cell-red', k=3, time_blocks=2),
    'c3v_red': W.scaled(W.C3, 2, name='3d-4cube-dg1-vertex-lognormal-red', coarse_cells=2, patch='vertex',
                        time_blocks=2),
    'c2d_red': W.scaled(W.C2D, 2, name='2d-8x8-q3p2disc-dg2-vertex-red', time_blocks=2),
    'c2s_b1_red': W.scaled(W.C2, 3, name='2d-16x16-dg2-vertex-b1-red', form='dtu', time_blocks=2),
    'c1_b1_tb': W.scaled(W.C1, 2, name='2d-8x8-dg1-cell-b1-tb', form='dtu', time_blocks=1),
    'c1_b1_full': W.scaled(W.C1, 2, name='2d-8x8-dg1-cell-b1-full', form='dtu', time_blocks=0),
    'c3s_disc_b1': W.scaled(W.C3, 2, name='3d-8cube-q2p1disc-dg1-cell-lognormal-b1', pressure='disc', form='dtu'),
    # the elements of Table C.1 (Q4^2/Q3) and Table 5.2 (Q4^2/P3^disc) with dG(3), 4x4 cells
    # (2 levels from 2x2), cell patches; two complex eigenvalue pairs in time
    'r4': W.scaled(W.C1, 2, name='2d-4x4-q4q3-dg3-cell', coarse_cells=2, r=4, k=3),
    'r4_disc': W.scaled(W.C1, 2, name='2d-4x4-q4p3disc-dg3-cell', coarse_cells=2, r=4, k=3, pressure='disc'),
    # the benchmark's physics on 64^2 (5 levels): 4,225 finest patches, where the tiled patch solve
    # picks one wave per patch by itself (four on the coarser levels)
    'c2_64': W.scaled(W.C2, 5, name='2d-64x64-dg2-vertex'),
}
