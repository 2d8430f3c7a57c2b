"""Flexible restarted GMRES (right preconditioning), as cited in Sec. 4 (Saad's
FGMRES): one preconditioner application z_j = B v_j per iteration, modified
Gram-Schmidt Arnoldi on w = A z_j, Givens rotations for the small least-squares
problem, and x = x0 + Z_m y_m at the end of each cycle.

Stopping test: ||b - A x|| <= rtol * ||b - A x0|| (the estimate |g_{j+1}| during
a cycle; every restart recomputes the true residual).  The paper prints an
absolute 1e-8; the relative form here is the one this library reports.
"""
import numpy as np


def fgmres(A, b, precond, x0=None, rtol=1e-8, restart=30, maxiter=1000, fixed_iters=None):
    """Return (x, info) with info = dict(iters, resid_history, converged).

    ``A`` is anything supporting ``A @ x``; ``precond(v)`` returns B v.
    With ``fixed_iters`` the loop runs exactly that many iterations (used to
    compare two implementations at equal iteration counts).
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else x0.astype(float).copy()
    r = b - A @ x
    beta0 = np.linalg.norm(r)
    hist = [beta0]
    its = 0
    if beta0 == 0.0:
        return x, dict(iters=0, resid_history=hist, converged=True)
    target = rtol * beta0
    while True:
        r = b - A @ x
        beta = np.linalg.norm(r)
        if fixed_iters is None and beta <= target:
            return x, dict(iters=its, resid_history=hist, converged=True)
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = A @ Z[j]
            for i in range(j + 1):
                H[i, j] = np.dot(w, V[i])
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] == 0.0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            # apply the previous rotations to the new column, then make a new one
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            its += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]))
            if breakdown and fixed_iters is None:
                break  # happy breakdown: the Krylov space holds the solution
            if fixed_iters is not None:
                if its >= fixed_iters:
                    break
            elif abs(g[j + 1]) <= target or its >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_done, :j_done]), g[:j_done])
        x = x + Z[:j_done].T @ y
        if fixed_iters is not None and its >= fixed_iters:
            return x, dict(iters=its, resid_history=hist, converged=None)
        if its >= maxiter:
            r = b - A @ x
            return x, dict(iters=its, resid_history=hist, converged=bool(np.linalg.norm(r) <= target))
