"""dG(k) time discretisation on one slab I_n = (t_{n-1}, t_n].

Paper, Sec. 2, the quadrature formula labelled Eq:GF: the right-sided (k+1)-point Gauss-Radau
rule on [-1, 1], exact for polynomials of degree 2k, whose last node is +1
(the slab end t_n).  Sec. 4, expansion Eq:TimeExp: the discrete
trajectories are expanded in the Lagrange basis chi_1..chi_{k+1} at those nodes.

From Problem 3.1 (Eq:DPQ_A0) the time parts of the slab operator are

    D^t[b, a] = Q_n( d/dt chi_a * chi_b ) + chi_a(t_{n-1}^+) chi_b(t_{n-1}^+)
    M^t[b, a] = Q_n( chi_a * chi_b )

(row = test function b, column = trial function a), and the jump vector
e[b] = chi_b(t_{n-1}^+) carries the previous slab's end value into the
right-hand side.  D^t does not depend on tau (the 2/tau of d/dt cancels the
tau/2 of the rule); M^t = tau/2 * diag(w).
"""
import numpy as np
from numpy.polynomial import legendre as L
from numpy.polynomial import polynomial as Pw


def gauss_radau_right(k):
    """Nodes and weights of the (k+1)-point right Gauss-Radau rule on [-1, 1].

    The nodes are the roots of P_k - P_{k+1} (Legendre polynomials), which
    vanishes at x = +1; the weights follow from exactness on 1, x, ..., x^k
    (a (k+1)x(k+1) moment system).  Returned in increasing order.
    """
    if k == 0:
        return np.array([1.0]), np.array([2.0])
    c = np.zeros(k + 2)
    c[k] = 1.0
    c[k + 1] = -1.0
    x = np.sort(np.real(L.legroots(c)))
    x[-1] = 1.0  # the root at +1 is exact
    V = np.vander(x, k + 1, increasing=True).T  # V[q, j] = x_j^q
    moments = np.array([(1.0 - (-1.0) ** (q + 1)) / (q + 1) for q in range(k + 1)])
    w = np.linalg.solve(V, moments)
    return x, w


def lagrange_basis(nodes):
    """Power-series coefficients of the Lagrange polynomials on ``nodes``."""
    polys = []
    for a, xa in enumerate(nodes):
        others = np.delete(nodes, a)
        num = Pw.polyfromroots(others) if len(others) else np.array([1.0])
        polys.append(num / Pw.polyval(xa, num))
    return polys


def time_matrices(k, tau):
    """Return (D^t, M^t, e, nodes, weights) for dG(k) on a slab of length tau.

    D^t and M^t are written exactly as the quadrature of Problem 3.1, not in a
    simplified closed form, so that a reader can check them against the paper.
    """
    x, w = gauss_radau_right(k)
    chi = lagrange_basis(x)
    dchi = [Pw.polyder(c) if len(c) > 1 else np.array([0.0]) for c in chi]
    n = k + 1
    Dt = np.zeros((n, n))
    Mt = np.zeros((n, n))
    e = np.array([Pw.polyval(-1.0, chi[b]) for b in range(n)])
    for b in range(n):
        for a in range(n):
            # Q_n(d/dt chi_a chi_b): (tau/2) sum_mu w_mu (2/tau) chi_a'(x_mu) chi_b(x_mu)
            Dt[b, a] = sum(w[m] * Pw.polyval(x[m], dchi[a]) * Pw.polyval(x[m], chi[b]) for m in range(n))
            Dt[b, a] += Pw.polyval(-1.0, chi[a]) * Pw.polyval(-1.0, chi[b])
            Mt[b, a] = 0.5 * tau * sum(w[m] * Pw.polyval(x[m], chi[a]) * Pw.polyval(x[m], chi[b]) for m in range(n))
    return Dt, Mt, e, x, w


def slab_nodes(t_start, tau, k):
    """Physical Gauss-Radau nodes t_{n,1..k+1} of the slab (t_start, t_start + tau]."""
    x, _ = gauss_radau_right(k)
    return t_start + 0.5 * tau * (1.0 + x)


def eval_basis(k, xhat):
    """Values chi_a(xhat) of the Lagrange time basis at reference points xhat in [-1, 1]."""
    x, _ = gauss_radau_right(k)
    chi = lagrange_basis(x)
    xhat = np.atleast_1d(np.asarray(xhat, dtype=float))
    return np.array([[Pw.polyval(t, chi[a]) for a in range(k + 1)] for t in xhat])
