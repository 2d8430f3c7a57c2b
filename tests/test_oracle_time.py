"""Pins of the dG(k) time discretisation (right Gauss-Radau rule, Sec. 2 Eq:GF;
time matrices of Problem 3.1) against closed forms."""
import math

import numpy as np
import pytest

from oracle import timedg


@pytest.mark.parametrize("k", [0, 1, 2, 3])
def test_gauss_radau_exactness(k):
    x, w = timedg.gauss_radau_right(k)
    assert len(x) == k + 1 and x[-1] == 1.0 and np.all(np.diff(x) > 0)
    for q in range(2 * k + 1):  # exact up to degree 2k
        exact = (1.0 - (-1.0) ** (q + 1)) / (q + 1)
        assert abs(np.sum(w * x ** q) - exact) < 1e-13
    q = 2 * k + 1  # and not beyond
    assert abs(np.sum(w * x ** q) - (1.0 - (-1.0) ** (q + 1)) / (q + 1)) > 1e-6


def test_known_nodes():
    x, w = timedg.gauss_radau_right(1)
    assert np.allclose(x, [-1 / 3, 1]) and np.allclose(w, [1.5, 0.5])
    x, w = timedg.gauss_radau_right(2)
    s6 = math.sqrt(6.0)
    assert np.allclose(x, [(-1 - s6) / 5, (-1 + s6) / 5, 1])
    assert np.allclose(w, [(16 - s6) / 18, (16 + s6) / 18, 2 / 9])


def pade_k_kp1(k, z):
    """(k, k+1) Pade approximant of exp(z) from its classical closed form."""
    n, m = k, k + 1
    num = sum(math.factorial(n + m - j) * math.factorial(n) / (math.factorial(n + m) * math.factorial(j) * math.factorial(n - j)) * z ** j
              for j in range(n + 1))
    den = sum(math.factorial(n + m - j) * math.factorial(m) / (math.factorial(n + m) * math.factorial(j) * math.factorial(m - j)) * (-z) ** j
              for j in range(m + 1))
    return num / den


@pytest.mark.parametrize("k", [0, 1, 2, 3])
@pytest.mark.parametrize("z", [-0.3, -2.0, -50.0, 0.7, 1e-3])
def test_slab_end_is_pade(k, z):
    """dG(k) with the right Radau rule on y' = lam y maps y_{n-1} to the (k,k+1) Pade value of exp(lam tau)."""
    tau = 0.37
    lam = z / tau
    Dt, Mt, e, _, _ = timedg.time_matrices(k, tau)
    Y = np.linalg.solve(Dt - lam * Mt, e * 1.0)
    assert abs(Y[-1] - pade_k_kp1(k, z)) < 1e-12 * max(1.0, abs(pade_k_kp1(k, z)))


def test_k0_is_backward_euler():
    Dt, Mt, e, _, _ = timedg.time_matrices(0, 0.25)
    assert np.allclose(Dt, [[1.0]]) and np.allclose(Mt, [[0.25]]) and np.allclose(e, [1.0])


@pytest.mark.parametrize("k", [1, 2, 3])
def test_time_matrix_values(k):
    """D^t reproduces the slab integral of p' q plus the jump term for polynomials of degree k."""
    Dt, Mt, e, x, w = timedg.time_matrices(k, 2.0)  # tau = 2: reference interval itself
    rng = np.random.default_rng(k)
    a = rng.standard_normal(k + 1)  # coefficients of p in powers of t
    b = rng.standard_normal(k + 1)
    P = np.polynomial.Polynomial(a)
    Q = np.polynomial.Polynomial(b)
    exact = (P.deriv() * Q).integ()(1.0) - (P.deriv() * Q).integ()(-1.0) + P(-1.0) * Q(-1.0)
    assert abs(Q(x) @ Dt @ P(x) - exact) < 1e-12
    exact_m = (P * Q).integ()(1.0) - (P * Q).integ()(-1.0)
    assert abs(Q(x) @ Mt @ P(x) - exact_m) < 1e-12
    assert np.allclose(e @ P(x), P(-1.0))
