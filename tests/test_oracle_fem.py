"""Pins of the element integrals and assembled spatial forms (Sec. 3, Def:ACB,
Def:ab) against closed forms and structural facts."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, problem


def lin_field(blocks, fn):
    """Nodal interpolant of a vector field fn(x) -> (n, d) on the Q_r lattice, interleaved."""
    xs = blocks.mesh.node_coords(blocks.r)
    return fn(xs).reshape(-1)


@pytest.mark.parametrize("d", [2, 3])
def test_cell_closed_forms(d):
    h, lam, mu, rho, alpha = 0.37, 1.9, 0.6, 1.4, 0.8
    cm = fem.CellMatrices(d, 2, h, lam, mu, rho, alpha)
    # sum of all entries of the vector mass = rho * d * |cell|
    assert abs(cm.Mrho.sum() - rho * d * h ** d) < 1e-12
    assert abs(cm.Mp.sum() - h ** d) < 1e-13
    lat = np.array(fem.local_lattice(2, d), dtype=float) * h / 2  # local node coordinates
    # rigid motions have zero strain: translations and infinitesimal rotations
    for c in range(d):
        t = np.zeros((len(lat), d))
        t[:, c] = 1.0
        assert np.abs(cm.Avol @ t.reshape(-1)).max() < 1e-12
    rot = np.zeros((len(lat), d))
    rot[:, 0], rot[:, 1] = -lat[:, 1], lat[:, 0]
    assert np.abs(cm.Avol @ rot.reshape(-1)).max() < 1e-11
    # u = (x, 0, ..): eps = e1 e1^T, sigma:eps = 2 mu + lam
    u = np.zeros((len(lat), d))
    u[:, 0] = lat[:, 0]
    assert abs(u.reshape(-1) @ cm.Avol @ u.reshape(-1) - (2 * mu + lam) * h ** d) < 1e-12
    # u = x (all components): div = d, C(u, 1) volume part = -alpha d |cell|
    one_p = np.ones(cm.Mp.shape[0])
    assert abs(one_p @ cm.Cvol @ lat.reshape(-1) + alpha * d * h ** d) < 1e-12
    # grad of a constant vanishes; <grad x, grad x> = |cell|
    assert np.abs(cm.Bvol @ one_p).max() < 1e-12
    lat1 = np.array(fem.local_lattice(1, d), dtype=float) * h
    assert abs(lat1[:, 0] @ cm.Bvol @ lat1[:, 0] - h ** d) < 1e-12


@pytest.mark.parametrize("d", [2, 3])
def test_face_closed_forms(d):
    h, lam, mu, alpha = 0.5, 1.0, 1.0, 0.9
    cm = fem.CellMatrices(d, 2, h, lam, mu, 1.0, alpha)
    lat = np.array(fem.local_lattice(2, d), dtype=float) * h / 2
    lat1 = np.array(fem.local_lattice(1, d), dtype=float) * h
    for (axis, side), Af in cm.Aface.items():
        # a constant displacement has no traction: only the penalty term remains
        c = np.zeros((len(lat), d))
        c[:, 0] = 1.0
        assert abs(c.reshape(-1) @ Af @ c.reshape(-1) - cm.gamma_a / cm.hF * h ** (d - 1)) < 1e-6 * cm.gamma_a
        # alpha <chi . n, 1> for chi = n on that face equals alpha |face|
        nvec = np.zeros((len(lat), d))
        nvec[:, axis] = 1.0 if side == 1 else -1.0
        assert abs(np.ones(len(lat1)) @ cm.Cface[(axis, side)] @ nvec.reshape(-1) - alpha * h ** (d - 1)) < 1e-12
        # -<grad q . n, 1> - <q, grad 1 . n> for q = x_axis: -(+-1)|face|
        q = lat1[:, axis]
        sgn = 1.0 if side == 1 else -1.0
        assert abs(np.ones(len(lat1)) @ cm.Bface_K[(axis, side)] @ q + sgn * h ** (d - 1)) < 1e-12


@pytest.mark.parametrize("d,N", [(2, 3), (3, 2)])
def test_symmetry_and_coercivity(d, N):
    """M, A_gamma, B_gamma symmetric; A_gamma and B_gamma positive definite (Appendix A)."""
    prm = problem.Params(rho=1.2, lam=3.0, mu=0.8, alpha=0.9, c0=0.02, K=0.7)
    b = problem.SpaceBlocks(d, N, 2, prm)
    for M in (b.Mrho, b.A, b.B, b.Mp):
        assert abs(M - M.T).max() <= 1e-12 * abs(M).max()
    assert np.linalg.eigvalsh(b.A.toarray()).min() > 0
    assert np.linalg.eigvalsh(b.B.toarray()).min() > 0
    assert np.linalg.eigvalsh(b.Mrho.toarray()).min() > 0


def test_lame_from_young():
    lam, mu = problem.lame_from_young(100.0, 0.35)
    assert abs(lam - 86.41975308641975) < 1e-10 and abs(mu - 37.03703703703704) < 1e-10
    assert round(lam, 1) == 86.4 and round(mu, 1) == 37.0  # values printed in Sec. 5.1


def test_global_mass_and_divergence():
    """Assembled forms on a 3x3 mesh: mass of constants and the Gauss theorem for C."""
    prm = problem.Params(rho=2.0, alpha=0.5)
    b = problem.SpaceBlocks(2, 3, 2, prm)
    ones_v = np.ones(b.nv)
    assert abs(ones_v @ b.Mrho @ ones_v - 2.0 * 2) < 1e-12
    # C(chi, 1) = -alpha int div chi + alpha int_G chi.n = 0 for any chi (divergence theorem)
    rng = np.random.default_rng(0)
    chi = rng.standard_normal(b.nv)
    assert abs(np.ones(b.nP) @ b.C @ chi) < 1e-12 * np.abs(chi).max() * b.nv
