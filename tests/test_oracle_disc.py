"""Pins of the discontinuous-pressure pair Q_r^d / P_{r-1}^disc (Def:VhQh, Eq:DefVhQh) with
the symmetric interior penalty form B_gamma of Def:B (second option), in the oracle.

Every expected value here comes from the definitions worked out by hand (closed forms of the
cell mass and of single face terms), from properties the form must have (symmetry,
coercivity on the paper's meshes, consistency: a solution inside the discrete spaces is
reproduced), from exactness of the grid transfer, or from the printed rows of Tables 5.1 and
5.2."""
import os
from math import comb

import numpy as np
import pytest

from oracle import fem, gmg, norms, problem, timedg

HERE = os.path.dirname(os.path.abspath(__file__))


def moment(n):
    """int_{-1/2}^{1/2} z^n dz."""
    return 0.0 if n % 2 else 2.0 * 0.5 ** (n + 1) / (n + 1)


@pytest.mark.parametrize("d,r", [(2, 2), (2, 3), (2, 4), (3, 2), (3, 3)])
def test_pdisc_basis_dimension_and_cell_mass(d, r):
    """P_{r-1} has binom(r-1+d, d) functions; the cell mass of the centred monomials is
    h^d prod_ax m(alpha_ax + beta_ax) with m(n) = int_{-1/2}^{1/2} z^n dz."""
    ex = fem.pdisc_exponents(r - 1, d)
    assert len(ex) == comb(r - 1 + d, d) and len(set(ex)) == len(ex)
    assert all(sum(a) <= r - 1 for a in ex)
    h = 0.3
    cm = fem.CellMatrices(d, r, h, 1.0, 1.0, 1.0, 0.9, pressure='disc')
    ref = np.array([[h ** d * np.prod([moment(a[i] + b[i]) for i in range(d)]) for b in ex] for a in ex])
    assert np.allclose(cm.Mp, ref, rtol=1e-13, atol=1e-16)


def test_sipg_face_terms_closed_form():
    """Single entries of B_gamma on a 3x3 mesh with a different K in every cell, from the
    definition: for the constant basis function e_A of cell A, every one of its 2d faces adds
    gamma/h_F |F| (the gradient terms vanish), a neighbour pair shares -gamma/h_F |F|; and for
    q = (x - x_A)/h on A (the linear function in the face's normal direction) against the
    constant of the upper neighbour B: -<{K grad q} . n, [psi]> = K_A h^{d-2}/2 and the
    penalty gives -gamma/(2h)."""
    d, N, r = 2, 3, 2
    K = np.array([0.5, 1.0, 1.7, 2.2, 0.8, 1.3, 3.0, 0.6, 1.1])
    b = problem.SpaceBlocks(d, N, r, problem.Params(K=K, pressure='disc'))
    B = b.B.toarray()
    h, g = 1.0 / N, 0.5 * r * (r - 1)
    nl = b.nploc
    assert nl == 3  # (0,0), (1,0), (0,1)
    A, Bx, By = 4, 5, 7  # centre cell, its neighbour in +x, in +y
    assert np.isclose(B[A * nl, A * nl], 2 * d * g / h, rtol=1e-13)
    assert np.isclose(B[0, 0], 2 * d * g / h, rtol=1e-13)  # a corner cell: boundary faces count alike
    assert np.isclose(B[Bx * nl, A * nl], -g / h, rtol=1e-13)
    assert np.isclose(B[By * nl, A * nl], -g / h, rtol=1e-13)
    assert B[8 * nl, A * nl] == 0.0  # no shared face
    expect = 0.5 * K[A] * h ** (d - 2) - 0.5 * g / h
    assert np.isclose(B[Bx * nl, A * nl + 1], expect, rtol=1e-13)  # test: const of B_x, trial: x-linear of A
    assert np.isclose(B[By * nl, A * nl + 2], expect, rtol=1e-13)  # test: const of B_y, trial: y-linear of A
    assert np.isclose(B[A * nl + 1, Bx * nl], expect, rtol=1e-13)  # symmetric counterpart


@pytest.mark.parametrize("d,N,r", [(2, 4, 2), (2, 4, 3), (2, 4, 4), (3, 2, 2)])
def test_sipg_symmetric_and_coercive(d, N, r):
    """B_gamma is symmetric, and coercive with the paper's gamma on the meshes it uses (K = I);
    without the penalty term it is not (so the test sees a dropped or mis-signed penalty)."""
    prm = problem.Params(K=1.0, pressure='disc')
    b = problem.SpaceBlocks(d, N, r, prm)
    B = b.B.toarray()
    assert np.abs(B - B.T).max() <= 1e-13 * np.abs(B).max()
    assert np.linalg.eigvalsh(B).min() > 0
    b0 = problem.SpaceBlocks(d, N, r, problem.Params(K=1.0, pressure='disc', gamma_b=0.0))
    assert np.linalg.eigvalsh(b0.B.toarray()).min() < 0


def poly_solution_disc(d, r, prm):
    """A solution inside the discrete spaces: Q2 displacement (continuous), P_{r-1} pressure,
    degree 1 in time, non-zero Dirichlet data on the whole boundary."""
    if d == 2:
        u = ["(1+t)*(x**2*y + 0.3*y**2 - x*y + 1)", "(1-2*t)*(x*y**2 + 0.5*x**2*y**2 - y)"]
        p = "(2+t)*(x + 2*y)" if r == 2 else "(2+t)*(x + 2*y + x*y - 0.5*y**2)"
    else:
        u = ["(1+t)*(x**2*y + z*y**2 - x*z + 1)", "(1-2*t)*(x*y*z + 0.5*x**2*z**2 - y)", "t*(y**2*z+x)"]
        p = "(2+t)*(x + 2*y - z)"
    return problem.ExactSolution(d, u, p, prm)


@pytest.mark.parametrize("d,N,k,r", [(2, 3, 1, 2), (2, 3, 2, 3), (3, 2, 1, 2)])
def test_exact_solution_is_reproduced_disc(d, N, k, r):
    """Consistency of the SIPG form and its boundary data (Def:B, Def:G second options): the
    projection of a solution inside the discrete spaces satisfies every discrete equation to
    rounding, and the direct solve returns it."""
    prm = problem.Params(rho=1.3, lam=2.0, mu=0.7, alpha=0.9, c0=0.05, K=1.7, pressure='disc')
    sol = poly_solution_disc(d, r, prm)
    tau = 0.1
    pr = problem.SlabProblem(d, N, r, k, tau, prm)
    X0 = problem.interpolate(pr.blocks, sol, 0.3)
    F = problem.slab_rhs(pr.blocks, k, tau, 0.3, X0, sol)
    Xex = np.concatenate([problem.interpolate(pr.blocks, sol, t) for t in timedg.slab_nodes(0.3, tau, k)])
    R = pr.A @ Xex - F
    scale = abs(pr.A) @ abs(Xex) + abs(F)
    assert np.max(np.abs(R) / scale) < 1e-12
    X = pr.direct_solve(F)
    assert np.abs(X - Xex).max() < 1e-9 * np.abs(Xex).max()


@pytest.mark.parametrize("d,Nc,r", [(2, 2, 2), (2, 2, 4), (3, 1, 3)])
def test_disc_prolongation_is_exact(d, Nc, r):
    """The prolongated coarse P_{r-1}^disc function equals the coarse function at every point
    of every fine cell."""
    prm = problem.Params(pressure='disc')
    cb = problem.SpaceBlocks(d, Nc, r, prm)
    fb = problem.SpaceBlocks(d, 2 * Nc, r, prm)
    P = gmg.disc_prolongation(cb, fb)
    rng = np.random.default_rng(5)
    qc = rng.standard_normal(cb.nP)
    qf = P @ qc
    pts = rng.random((7, d))
    for cf in range(fb.mesh.ncells):
        x = fb.mesh.cell_origin(cf) + fb.mesh.h * pts
        cc = 0
        ci = np.array(fb.mesh.cell_index(cf)) // 2
        for ax in reversed(range(d)):
            cc = cc * Nc + ci[ax]
        vf, _ = fb.pbasis(pts)
        vc, _ = cb.pbasis((x - cb.mesh.cell_origin(cc)) / cb.mesh.h)
        assert np.allclose(vf @ qf[cf * fb.nploc:(cf + 1) * fb.nploc],
                           vc @ qc[cc * cb.nploc:(cc + 1) * cb.nploc], rtol=0, atol=1e-13)


def test_table_5_1_rows_1_2():
    """Sec. 5.1, Table 5.1, rows 1-2 (Q3^2/P2^disc, dG(2); 4x4 cells, tau = 0.1, then 8x8 cells,
    tau = 0.05; I = (1,2]): the displacement-gradient and velocity errors reproduce the printed
    values to 0.5 %, and all three errors converge at the printed rate (about 3).  The printed
    pressure errors are not reproduced: the oracle's are 1.6-1.9x larger at both sizes (the
    ratio is printed, not asserted; parity unpinned for the pressure magnitude)."""
    vals = {}
    for line in open(os.path.join(HERE, 'golden', 'table_5_1_rows12.txt')):
        if line.strip() and not line.startswith('#'):
            key, *nums = line.split()
            vals[key] = np.array([float(x) for x in nums])
    lam, mu = problem.lame_from_young(100.0, 0.35)
    phi = "sin(pi*t**2)*sin(pi*x)*sin(pi*y)"
    prm = problem.Params(rho=1.0, lam=lam, mu=mu, alpha=0.9, c0=0.01, K=1.0, pressure='disc')
    sol = problem.ExactSolution(2, [phi, phi], phi, prm)
    errs = []
    for lev in (0, 1):
        pr = problem.SlabProblem(2, 4 * 2 ** lev, 3, 2, 0.1 / 2 ** lev, prm)
        errs.append(norms.error_norms(pr, sol, pr.march(sol, 1.0, 10 * 2 ** lev), 1.0, M=10)['L2'])
    for e, key in zip(errs, ('row1', 'row2')):
        rel = e / vals[key]
        assert np.all(np.abs(rel[:2] - 1) < 5e-3), (key, rel)
        print(f"Table 5.1 {key}: oracle / printed pressure error {rel[2]:.2f}")
    eoc = np.log2(errs[0] / errs[1])
    assert np.all(eoc > 2.9), eoc


def test_table_5_2_row1_against_taylor_hood():
    """Sec. 5.1, Table 5.2 row 1 (Q4^2/P3^disc, dG(3), 4x4 cells, tau = 0.1, I = (1,2]).

    As for the Taylor-Hood table C.1 the printed magnitudes are not reproduced by the readings
    taken here (parity unpinned for them).  The two printed tables fix a relation between the
    pairs on this row that the oracle does reproduce: the same displacement and velocity errors
    (printed ratio 1.000), checked on the oracle's own errors.  Their pressure
    relation (discontinuous/Taylor-Hood 0.92) is not reproduced (the oracle gives about 2.3, in
    line with the pressure gap of Table 5.1): recorded, not asserted."""
    vals = {}
    for line in open(os.path.join(HERE, 'golden', 'table_5_2_row1.txt')):
        if line.strip() and not line.startswith('#'):
            key, *nums = line.split()
            vals[key] = np.array([float(x) for x in nums])
    lam, mu = problem.lame_from_young(100.0, 0.35)
    phi = "sin(pi*t**2)*sin(pi*x)*sin(pi*y)"
    e = {}
    for kind in ('disc', 'cont'):
        prm = problem.Params(rho=1.0, lam=lam, mu=mu, alpha=0.9, c0=0.01, K=1.0, pressure=kind)
        sol = problem.ExactSolution(2, [phi, phi], phi, prm)
        pr = problem.SlabProblem(2, 4, 4, 3, 0.1, prm)
        Xs = pr.march(sol, 1.0, 10)
        e[kind] = norms.error_norms(pr, sol, Xs, 1.0, M=100)
    printed = vals['L2'] / np.array([2.3958497242e-03, 1.7185669625e-02, 7.6634974254e-04])  # Table C.1 row 1
    assert abs(printed[0] - 1) < 1e-5 and abs(printed[1] - 1) < 1e-5
    rel = e['disc']['L2'] / e['cont']['L2']
    assert abs(rel[0] - 1) < 0.02 and abs(rel[1] - 1) < 0.02, rel
