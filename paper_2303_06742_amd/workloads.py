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
    # patch solves: 3 reduced with symmetric tiled Schur inverses, 2 reduced (square), 1 time
    # blocks, 0 full inverses
    time_blocks: int = 3
    pressure: str = 'cont'  # 'cont': Q_{r-1} (Taylor-Hood); 'disc': P_{r-1}^disc with interior penalty
    form: str = 'v'         # 'v': Problem 3.1; 'dtu': Problem B.1
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
# the same 3D physics with vertex patches (2x2x2 cells, the paper's 3D smoother); stored with the
# reduced time-block solves it takes about 104 GB (FP64)
C3V = Config('3d-32cube-dg1-vertex', dim=3, coarse_cells=4, levels=4, k=1, patch='vertex', tau=1e-3, slabs=10,
             alpha=1.0, c0=1e-3, K_logsd=1.0, seed=0)


# the discontinuous-pressure pair of the paper's convergence study (Q3^2/P2^disc, dG(2), Table 5.1)
# on 128x128 quads (6 levels from 4^2), vertex patches, 10 slabs of 1e-3
C2D = Config('2d-128x128-q3p2disc-dg2-vertex', dim=2, coarse_cells=4, levels=6, k=2, patch='vertex', tau=1e-3,
             slabs=10, r=3, pressure='disc')


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


def _random_physics(rng):
    """lambda, mu ~ U[0.5, 5], alpha ~ U[0.5, 1], c0 = 10^U[-4,-1], K = 10^U[-3,0], rho = 1."""
    return dict(lam=float(rng.uniform(0.5, 5)), mu=float(rng.uniform(0.5, 5)), alpha=float(rng.uniform(0.5, 1)),
                c0=float(10 ** rng.uniform(-4, -1)), K=float(10 ** rng.uniform(-3, 0)), rho=1.0)


def batch_configs(count, seed=0, sizes=(16, 32, 64, 128)):
    """Independent 2D problems: N ~ U(sizes) cells per axis from a 4x4 coarsest grid, dG(1) or dG(2),
    vertex patches, one slab of tau = 1e-3, random physics, FP32 smoother."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        N = int(rng.choice(sizes))
        k = int(rng.integers(1, 3))
        levels = int(np.log2(N // 4)) + 1
        out.append(Config(f'batch{i}-2d-{N}-dg{k}', dim=2, coarse_cells=4, levels=levels, k=k, patch='vertex',
                          tau=1e-3, slabs=1, precision='fp32', **_random_physics(rng)))
    return out


def serve_mix(count, seed=0, sizes2d=(32, 64, 128), sizes3d=(8, 16), p3d=0.3, p_follow=0.5):
    """Request stream of the serving workload: 70% 2D (vertex patches) and 30% 3D (cell patches)
    problems, dG(1)/dG(2), random physics, FP32 smoother; about half the requests are follow-on
    slabs of an earlier problem (same key).  Returns a list of (key, Config)."""
    rng = np.random.default_rng(seed)
    problems = []
    out = []
    for i in range(count):
        if problems and rng.random() < p_follow:
            key, cfg = problems[int(rng.integers(len(problems)))]
        else:
            k = int(rng.integers(1, 3))
            if rng.random() < p3d:
                N = int(rng.choice(sizes3d))
                cfg = Config(f'serve{i}-3d-{N}-dg{k}', dim=3, coarse_cells=2, levels=int(np.log2(N // 2)) + 1, k=k,
                             patch='cell', tau=1e-3, slabs=1, precision='fp32', **_random_physics(rng))
            else:
                N = int(rng.choice(sizes2d))
                cfg = Config(f'serve{i}-2d-{N}-dg{k}', dim=2, coarse_cells=4, levels=int(np.log2(N // 4)) + 1, k=k,
                             patch='vertex', tau=1e-3, slabs=1, precision='fp32', **_random_physics(rng))
            key = len(problems) + 1
            problems.append((key, cfg))
        out.append((key, cfg))
    return out
