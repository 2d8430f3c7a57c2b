"""Pins of the whole slab discretisation (Problem 3.1 / Problem 4.1)."""
import os

import numpy as np
import pytest

from oracle import norms, problem, timedg

HERE = os.path.dirname(os.path.abspath(__file__))


def poly_solution(d, prm):
    """A solution inside the discrete spaces: Q2 in space for u, Q1 for p, degree 1 in time,
    with non-zero Dirichlet data for u, v = u_t and p on the whole boundary."""
    if d == 2:
        u = ["(1+t)*(x**2*y + 0.3*y**2 - x*y + 1)", "(1-2*t)*(x*y**2 + 0.5*x**2*y**2 - y)"]
        p = "(2+t)*(x + 2*y + x*y)"
    else:
        u = ["(1+t)*(x**2*y + z*y**2 - x*z + 1)", "(1-2*t)*(x*y*z + 0.5*x**2*z**2 - y)", "t*(y**2*z+x)"]
        p = "(2+t)*(x + 2*y + x*y*z)"
    return problem.ExactSolution(d, u, p, prm)


@pytest.mark.parametrize("d,N,k", [(2, 3, 1), (2, 3, 2), (3, 2, 1)])
def test_exact_solution_is_reproduced(d, N, k):
    """Consistency + uniqueness: a solution in the discrete space is reproduced exactly.

    Checks both that the interpolant satisfies every discrete equation to rounding
    (row-wise relative residual) and that the direct solve returns it."""
    prm = problem.Params(rho=1.3, lam=2.0, mu=0.7, alpha=0.9, c0=0.05, K=1.7)
    sol = poly_solution(d, prm)
    tau = 0.1
    pr = problem.SlabProblem(d, N, 2, k, tau, prm)
    X0 = problem.interpolate(pr.blocks, sol, 0.3)
    F = problem.slab_rhs(pr.blocks, k, tau, 0.3, X0, sol)
    Xex = np.concatenate([problem.interpolate(pr.blocks, sol, t) for t in timedg.slab_nodes(0.3, tau, k)])
    R = pr.A @ Xex - F
    scale = abs(pr.A) @ abs(Xex) + abs(F)
    assert np.max(np.abs(R) / scale) < 1e-13
    X = pr.direct_solve(F)
    assert np.abs(X - Xex).max() < 1e-10 * np.abs(Xex).max()


def test_temporal_superconvergence():
    """Space-exact solution, smooth in time: error at t_n is O(tau^(2k+1)) (Sec. 5.1, Eq:MDN, Table 5.3 analogue).

    As in Eq:givensolution2 the time-dependent part vanishes on the boundary;
    time-dependent Dirichlet data enforced by the stiff Nitsche penalty would
    reduce the nodal order of this Radau-type scheme."""
    prm = problem.Params(rho=1.0, lam=1.0, mu=1.0, alpha=0.9, c0=0.01, K=1.0)
    u = ["sin(3*t)*x*(1-x)*y*(1-y)", "cos(2*t)*x*(1-x)*y*(1-y)"]
    p = "x + 2*y + x*y"
    sol = problem.ExactSolution(2, u, p, prm)
    for k in (1, 2):
        errs = []
        for nt in (2, 4, 8):
            tau = 0.4 / nt
            pr = problem.SlabProblem(2, 2, 2, k, tau, prm)
            Xs = pr.march(sol, 0.0, nt)
            ex = problem.interpolate(pr.blocks, sol, 0.4)
            errs.append(np.abs(pr.end_block(Xs[-1]) - ex).max())
        rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
        assert rates[-1] > 2 * k + 1 - 0.3, (k, errs, rates)


def test_space_time_eoc():
    """Optimal rates on the C1 manufactured solution, h and tau halved together (Eq:ApFES):
    ||grad(u-u_h)||, ||v-v_h||, ||p-p_h|| all converge at least like h^2 for Q2/Q1, dG(1)."""
    prm = problem.Params(rho=1.0, lam=1.0, mu=1.0, alpha=0.9, c0=0.01, K=1.0)
    S = "sin(pi*x)*sin(pi*y)"
    sol = problem.ExactSolution(2, [S + "*sin(t)", S + "*sin(t)"], S + "*cos(t)", prm)
    errs = []
    for N in (4, 8):
        tau = 0.1 * 2 / N
        pr = problem.SlabProblem(2, N, 2, 1, tau, prm)
        Xs = pr.march(sol, 0.0, int(round(0.2 / tau)))
        errs.append(norms.error_norms(pr, sol, Xs, 0.0, M=10)['L2'])
    eoc = np.log2(errs[0] / errs[1])
    assert np.all(eoc > 1.8), eoc


def test_energy_decay():
    """Zero data: A_gamma(u,u) + rho|v|^2 + c0|p|^2 at t_n never grows (Lemma 3.2, Eq:ExUniDS_3)."""
    prm = problem.Params(rho=1.1, lam=2.0, mu=0.5, alpha=0.9, c0=0.03, K=0.8)
    pr = problem.SlabProblem(2, 3, 2, 2, 0.05, prm)
    b = pr.blocks
    rng = np.random.default_rng(3)
    X = rng.standard_normal(b.ns)
    solve = pr.factor()
    def energy(Y):
        V, U, P = Y[:b.nv], Y[b.nv:2 * b.nv], Y[2 * b.nv:]
        return U @ b.A @ U + V @ b.Mrho @ V + prm.c0 * P @ b.Mp @ P
    E = [energy(X)]
    for _ in range(6):
        X = pr.end_block(solve(problem.slab_rhs(b, 2, 0.05, 0.0, X)))
        E.append(energy(X))
    assert np.all(np.diff(E) < 1e-12 * E[0]), E
    assert E[-1] < E[0]


@pytest.mark.slow
def test_table_c1_asymptotic_rates():
    """Appendix C, Table C.1 (Q4^2/Q3, dG(3), I = (1,2], tau and h halved together): the oracle's
    L2(L2) orders between rows 2 and 3 (8x8 cells, tau = 0.05; 16x16, tau = 0.025) equal the
    printed asymptotic orders, those between rows 4 and 5 (4.00, 4.09, 4.03), to 0.1.

    The printed magnitudes are not reproduced: the oracle's row-1 errors are 0.36 / 0.14 / 0.20
    of the printed ones and its rows 2-3 already sit in the asymptotic regime, while the printed
    row 1 is pre-asymptotic (orders 4.5 / 5.0 / 4.3 to row 2).  The readings tried (penalty
    face size, rounded Lame constants, source quadrature in time, norm quadrature, interval,
    displacement direction) leave the gap; the magnitudes are parity unpinned."""
    vals = {}
    for line in open(os.path.join(HERE, 'golden', 'table_c1_row1.txt')):
        if line.strip() and not line.startswith('#'):
            key, *nums = line.split()
            vals[key] = np.array([float(x) for x in nums])
    printed = np.log2(vals['L2_row4'] / vals['L2_row5'])
    lam, mu = problem.lame_from_young(100.0, 0.35)
    prm = problem.Params(rho=1.0, lam=lam, mu=mu, alpha=0.9, c0=0.01, K=1.0)
    phi = "sin(pi*t**2)*sin(pi*x)*sin(pi*y)"
    sol = problem.ExactSolution(2, [phi, phi], phi, prm)
    errs = []
    for lev in (1, 2):
        pr = problem.SlabProblem(2, 4 * 2 ** lev, 4, 3, 0.1 / 2 ** lev, prm)
        errs.append(norms.error_norms(pr, sol, pr.march(sol, 1.0, 10 * 2 ** lev), 1.0, M=4)['L2'])
    eoc = np.log2(errs[0] / errs[1])
    assert np.all(np.abs(eoc - printed) < 0.1), (eoc, printed)
