"""Seeded synthetic workloads shared by the tests and the benchmark.

Holds none of the method's arithmetic: configurations (mesh, levels, orders,
material parameters), seeded random fields and vectors, and the formula of the
built-in prescribed solution as text.
"""
from dataclasses import dataclass, field

import numpy as np


def builtin_solution_exprs(d):
    """u_i = S sin t (every component), p = S cos t, S = prod_j sin(pi x_j)."""
    S = '*'.join(f'sin(pi*{v})' for v in 'xyz'[:d])
    return [f'{S}*sin(t)'] * d, f'{S}*cos(t)'


@dataclass
class Config:
    name: str
    dim: int
    coarse_cells: int
    levels: int
    k: int
    patch: str            # 'cell' or 'vertex'
    tau: float
    slabs: int
    rho: float = 1.0
    lam: float = 1.0
    mu: float = 1.0
    alpha: float = 0.9
    c0: float = 0.01
    K: float = 1.0
    K_logsd: float = 0.0  # > 0: lognormal K per fine cell with this log standard deviation
    seed: int = 0
    r: int = 2
    precision: str = 'fp64'
    n_smooth: int = 4
    omega: float = 0.7
    restart: int = 30
    rtol: float = 1e-8
    extra: dict = field(default_factory=dict)

    @property
    def fine_cells(self):
        return self.coarse_cells << (self.levels - 1)

    def K_cells(self):
        """Per-fine-cell permeability (lexicographic, x fastest), or None for constant K."""
        if self.K_logsd <= 0:
            return None
        rng = np.random.default_rng(self.seed)
        return np.exp(self.K_logsd * rng.standard_normal(self.fine_cells ** self.dim))


# 2D unit square, 8x8 quads (levels 4^2, 8^2), Q2/Q2/Q1, dG(1), one slab, cell patches, FP64
C1 = Config('2d-8x8-dg1-cell', dim=2, coarse_cells=4, levels=2, k=1, patch='cell', tau=0.01, slabs=1)
# 2D unit square, 256x256 quads (7 levels from 4^2), dG(2), 20 slabs of 1e-3, 2x2-cell (vertex) patches
C2 = Config('2d-256x256-dg2-vertex', dim=2, coarse_cells=4, levels=7, k=2, patch='vertex', tau=1e-3, slabs=20)
# 3D unit cube, 32^3 hexes (4 levels), dG(1), 10 slabs, lognormal K (log-sd 1), alpha=1, c0=1e-3, cell patches
C3 = Config('3d-32cube-dg1-cell', dim=3, coarse_cells=4, levels=4, k=1, patch='cell', tau=1e-3, slabs=10,
            alpha=1.0, c0=1e-3, K_logsd=1.0, seed=0)


def scaled(cfg, levels, name=None, **kw):
    """The same physics on fewer levels (smaller grids) for tests."""
    d = dict(cfg.__dict__)
    d.update(kw)
    d['levels'] = levels
    d['name'] = name or f'{cfg.name}-L{levels}'
    d['extra'] = dict(cfg.extra)
    return Config(**d)


def random_vector(n, seed):
    return np.random.default_rng(seed).standard_normal(n)
