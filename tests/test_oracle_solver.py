"""Pins of the multigrid pieces (Sec. 4) and FGMRES against definitions,
invariants and brute force."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fgmres, gmg, problem


def prm():
    return problem.Params(rho=1.0, lam=1.0, mu=1.0, alpha=0.9, c0=0.01, K=1.0)


@pytest.mark.parametrize("d,p", [(2, 2), (2, 1), (3, 2), (3, 1)])
def test_prolongation_reproduces_coarse_polynomials(d, p):
    """Interpolation is exact for Q_p functions of the coarse mesh (here global Q_p polynomials)."""
    Nc = 2
    I = gmg.interp_nd(p, Nc, d)
    rng = np.random.default_rng(d * 10 + p)
    coef = rng.standard_normal((p + 1,) * d)
    def f(xs):
        out = np.zeros(len(xs))
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([xs[:, a] ** idx[a] for a in range(d)], axis=0)
        return out
    xc = problem.Mesh(d, Nc).node_coords(p)
    xf = problem.Mesh(d, 2 * Nc).node_coords(p)
    assert np.abs(I @ f(xc) - f(xf)).max() < 1e-12
    # partition of unity and the 1D weights of Q2: 3/8, 3/4, -1/8
    assert np.allclose(I @ np.ones(I.shape[1]), 1.0)
    if p == 2 and d == 2:
        I1 = gmg.interp_1d(2, 1).toarray()
        assert np.allclose(I1[1], [3 / 8, 3 / 4, -1 / 8])


def small_hierarchy(kind, k=1):
    return gmg.Hierarchy(2, 2, 1, 2, k, 0.01, prm(), patch_kind=kind)


@pytest.mark.parametrize("kind", ["cell", "vertex"])
def test_patch_sizes(kind):
    H = small_hierarchy(kind, k=2)
    sizes = sorted(set(len(Z) for Z in H.fine.patches))
    # closure dofs: 2D cell patch (9 Q2 + 4 Q1 nodes), vertex patches 1/2/4 cells, times (k+1)
    assert sizes == ([120] if kind == 'cell' else [120, 198, 327])


@pytest.mark.parametrize("kind", ["cell", "vertex"])
def test_exact_local_solve_zeroes_patch_residual(kind):
    """Def:VankaOP with omega = 1: the local update zeroes the patch residual."""
    H = small_hierarchy(kind)
    lev = H.fine
    rng = np.random.default_rng(1)
    b = rng.standard_normal(lev.n)
    d = rng.standard_normal(lev.n)
    res = b - lev.A @ d
    for Z, Ainv in list(zip(lev.patches, lev.inv))[::3]:
        dn = d.copy()
        dn[Z] += Ainv @ res[Z]
        r2 = (b - lev.A @ dn)[Z]
        assert np.abs(r2).max() < 1e-9 * np.abs(res).max()


def test_averaging_identities():
    """sum_P E_P R_P x / p = x, and Alg. 4.1 equals d + omega * (sum_P E_P A_P^{-1} R_P r) / p."""
    H = small_hierarchy('vertex')
    lev = H.fine
    rng = np.random.default_rng(2)
    x = rng.standard_normal(lev.n)
    z = np.zeros(lev.n)
    for Z in lev.patches:
        z[Z] += x[Z]
    assert np.allclose(z / lev.count, x)
    b = rng.standard_normal(lev.n)
    d0 = rng.standard_normal(lev.n)
    d1 = gmg.vanka_smooth(lev, b, d0, 1, 0.7)
    r = b - lev.A @ d0
    acc = np.zeros(lev.n)
    for Z, Ainv in zip(lev.patches, lev.inv):
        acc[Z] += Ainv @ r[Z]
    assert np.abs(d1 - (d0 + 0.7 * acc / lev.count)).max() < 1e-12 * np.abs(d1).max()


def test_one_level_vcycle_is_direct_solve():
    H = gmg.Hierarchy(2, 2, 0, 2, 1, 0.01, prm())
    A = H.levels[0].A
    rng = np.random.default_rng(3)
    b = rng.standard_normal(A.shape[0])
    x, info = fgmres.fgmres(A, b, H.precondition, rtol=1e-8)
    assert info['iters'] == 1
    assert np.linalg.norm(b - A @ x) <= 1e-8 * np.linalg.norm(b)


@pytest.mark.parametrize("kind,k", [("cell", 1), ("vertex", 1), ("vertex", 2)])
def test_fgmres_gmg_matches_direct_solve(kind, k):
    H = gmg.Hierarchy(2, 2, 2, 2, k, 0.01, prm(), patch_kind=kind)
    f = H.fine.prob
    rng = np.random.default_rng(4)
    F = rng.standard_normal(f.n)
    x, info = fgmres.fgmres(f.A, F, H.precondition, rtol=1e-10)
    assert info['converged'] and info['iters'] <= 10
    xd = f.direct_solve(F)
    assert np.linalg.norm(F - f.A @ x) <= 1e-10 * np.linalg.norm(F)
    assert np.abs(x - xd).max() < 1e-6 * np.abs(xd).max()


def test_fgmres_minimises_residual_bruteforce():
    """With a fixed preconditioner B, j FGMRES steps give the minimal residual over x0 + B K_j(A B, r0)."""
    rng = np.random.default_rng(5)
    n = 12
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)
    B = np.eye(n) + 0.1 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    for j in (1, 3, 6):
        x, info = fgmres.fgmres(A, b, lambda v: B @ v, rtol=0.0, restart=30, fixed_iters=j)
        K = [b]
        for _ in range(j - 1):
            K.append(A @ (B @ K[-1]))
        BK = B @ np.array(K).T
        y, *_ = np.linalg.lstsq(A @ BK, b, rcond=None)
        assert np.abs(x - BK @ y).max() < 1e-10
        assert abs(info['resid_history'][-1] - np.linalg.norm(b - A @ x)) < 1e-10


def test_fgmres_finite_termination_and_restart():
    rng = np.random.default_rng(6)
    n = 8
    A = rng.standard_normal((n, n)) + 3 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = fgmres.fgmres(A, b, lambda v: v, rtol=1e-12, restart=30)
    assert info['iters'] <= n and np.linalg.norm(A @ x - b) < 1e-11 * np.linalg.norm(b)
    x2, info2 = fgmres.fgmres(A, b, lambda v: v, rtol=1e-12, restart=3, maxiter=500)
    assert info2['converged'] and np.linalg.norm(A @ x2 - b) <= 1e-12 * np.linalg.norm(b)


def test_coarsened_permeability_is_child_mean():
    """Coarse-level K (per cell) = mean of the 2^d children, in lexicographic cell order."""
    for d in (2, 3):
        Nf = 4
        K = np.arange(Nf ** d, dtype=float)
        Kc = gmg.coarsen_K(K, d, Nf)
        for c in range(2 ** d):
            ci = [(c >> a) & 1 for a in range(d)]  # coarse multi-index (x, y[, z]) with 2 cells per axis
            kids = []
            for ch in range(2 ** d):
                fi = [2 * ci[a] + ((ch >> a) & 1) for a in range(d)]
                kids.append(sum(fi[a] * Nf ** a for a in range(d)))
            assert Kc[sum(ci[a] * 2 ** a for a in range(d))] == np.mean(K[kids])
