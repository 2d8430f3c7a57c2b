"""Tensor-product Lagrange elements and the cell/face integrals of the forms.

Paper, Sec. 2 (Def:VhQh, Eq:DefVhQh): V_h = continuous Q_r^d for u and v,
Q_h = continuous Q_{r-1} for p (Taylor-Hood) or the broken space P_{r-1}^disc,
on a mesh of axis-parallel squares/cubes.  Sec. 3 (Def:ACB, Def:ab) gives the forms

    A_gamma(w, chi) = <C eps(w), eps(chi)> - <C eps(w) n, chi>_G + a_gamma(w, chi)
    a_gamma(w, chi) = -<w, C eps(chi) n>_G + gamma_a/h_F <w, chi>_G
    C(chi, q)       = -alpha <div chi, q> + alpha <chi . n, q>_G
    B_gamma(q, psi) = <K grad q, grad psi> - <K grad q . n, psi>_G + b_gamma(q, psi)
    b_gamma(q, psi) = -<q, K grad psi . n>_G + gamma_b/h_F <q, psi>_G

with C eps(w) = 2 mu eps(w) + lambda div(w) I (isotropic), G = the Dirichlet
boundary (all of the boundary here), gamma_a = 5e4 r (r+1), gamma_b = r(r-1)/2
and, on a boundary face, h_F = |K|_d, the d-dimensional measure of the cell.

For Q_h = P_{r-1}^disc, B_gamma is the symmetric interior penalty form of Def:B
(second option): the volume term per cell, and on every face F (interior and
boundary) -<{K grad q} . n, [psi]>_F - <[q], {K grad psi} . n>_F
+ gamma/h_F <[q], [psi]>_F with {w} = (w+ + w-)/2, [w] = w+ - w- and n the unit
normal pointing out of K+ (on a boundary face {w} = [w] = w|K), gamma = gamma_b,
h_F = (|K+|_d + |K-|_d)/2 (= |K|_d on this uniform mesh), and no separate
b_gamma term (N^B omitted, Problem 4.1).  On a boundary face this is the same
expression as the continuous-pressure boundary terms.

Everything here works on one reference cell [0, h]^d: basis functions are
evaluated at Gauss points and the integrals are sums over those points.  The
local node order is lexicographic on the (p+1)^d lattice, x fastest; a vector
basis function (node a, component c) has local index d*a + c.
"""
import itertools

import numpy as np
from numpy.polynomial import legendre as L


def gauss01(n):
    """n-point Gauss-Legendre rule on [0, 1]."""
    x, w = L.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def basis_1d(p, xi):
    """(values, derivatives) of the degree-p Lagrange basis on the equispaced nodes of [0, 1] at
    reference points xi; shape (len(xi), p+1).  Evaluated in product form,
    l_a(x) = prod_{b != a} (x - x_b)/(x_a - x_b), so that l_a is exactly 0 at every other node
    (the stiff Nitsche penalty would amplify rounding noise there)."""
    nodes = np.linspace(0.0, 1.0, p + 1)
    xi = np.asarray(xi, dtype=float)
    v = np.ones((len(xi), p + 1))
    dv = np.zeros((len(xi), p + 1))
    for a in range(p + 1):
        others = [b for b in range(p + 1) if b != a]
        for b in others:
            v[:, a] *= (xi - nodes[b]) / (nodes[a] - nodes[b])
        for c in others:  # derivative: one factor differentiated at a time
            t = np.full(len(xi), 1.0 / (nodes[a] - nodes[c]))
            for b in others:
                if b != c:
                    t *= (xi - nodes[b]) / (nodes[a] - nodes[b])
            dv[:, a] += t
    return v, dv


def local_lattice(p, d):
    """Local node multi-indices (ix, iy[, iz]) in lexicographic order, x fastest."""
    return [tuple(reversed(t)) for t in itertools.product(range(p + 1), repeat=d)]


def scalar_basis(p, d, pts, h):
    """Values (nq, nloc) and physical gradients (nq, nloc, d) of Q_p on [0,h]^d at reference points pts (nq, d)."""
    pts = np.atleast_2d(pts)
    nq = pts.shape[0]
    lat = local_lattice(p, d)
    v1 = []
    dv1 = []
    for ax in range(d):
        v, dv = basis_1d(p, pts[:, ax])
        v1.append(v)
        dv1.append(dv)
    val = np.ones((nq, len(lat)))
    grad = np.ones((nq, len(lat), d))
    for a, idx in enumerate(lat):
        for ax in range(d):
            val[:, a] *= v1[ax][:, idx[ax]]
            for g in range(d):
                grad[:, a, g] *= (dv1[ax][:, idx[ax]] / h) if g == ax else v1[ax][:, idx[ax]]
    return val, grad


def pdisc_exponents(p, d):
    """Exponents alpha (|alpha| <= p) of the P_p^disc basis: the lexicographic order of the
    (p+1)^d lattice (x fastest), keeping total degree <= p."""
    return [a for a in local_lattice(p, d) if sum(a) <= p]


def pdisc_basis(p, d, pts, h):
    """Values (nq, n) and physical gradients (nq, n, d) of the broken P_p basis on [0,h]^d at
    reference points pts: the monomials prod_ax (xi_ax - 1/2)^alpha_ax, centred in the cell."""
    pts = np.atleast_2d(pts)
    z = pts - 0.5
    ex = pdisc_exponents(p, d)
    val = np.ones((pts.shape[0], len(ex)))
    grad = np.ones((pts.shape[0], len(ex), d))
    for j, a in enumerate(ex):
        for ax in range(d):
            val[:, j] *= z[:, ax] ** a[ax]
            for g in range(d):
                if g == ax:
                    grad[:, j, g] *= a[ax] * z[:, ax] ** max(a[ax] - 1, 0) / h
                else:
                    grad[:, j, g] *= z[:, ax] ** a[ax]
    return val, grad


def pressure_basis(kind, r, d, pts, h):
    """Pressure basis of the pair: 'cont' = Q_{r-1} (nodal), 'disc' = P_{r-1}^disc (monomials)."""
    return scalar_basis(r - 1, d, pts, h) if kind == 'cont' else pdisc_basis(r - 1, d, pts, h)


def cell_rule(n, d, h):
    """Tensor Gauss rule with n points per axis on [0,h]^d: reference points (nq,d), weights (nq,)."""
    x, w = gauss01(n)
    pts = np.array([tuple(reversed(t)) for t in itertools.product(x, repeat=d)])
    wts = np.array([np.prod(t) for t in itertools.product(w, repeat=d)]) * h ** d
    return pts, wts


def face_rule(n, d, h, axis, side):
    """Gauss rule on the face {xi_axis = side} of [0,h]^d; returns points, weights, outward normal."""
    x, w = gauss01(n)
    pts = []
    wts = []
    for t, wt in zip(itertools.product(x, repeat=d - 1), itertools.product(w, repeat=d - 1)):
        t = list(reversed(t))
        t.insert(axis, float(side))
        pts.append(t)
        wts.append(np.prod(wt))
    normal = np.zeros(d)
    normal[axis] = 1.0 if side == 1 else -1.0
    return np.array(pts), np.array(wts) * h ** (d - 1), normal


def vector_fields(val, grad, d):
    """For vector basis functions (node a, comp c) -> index d*a + c, return
    values (nq, nv, d) and gradient tensors G[q, i, comp, j] = d_j w_comp."""
    nq, ns = val.shape
    nv = d * ns
    W = np.zeros((nq, nv, d))
    G = np.zeros((nq, nv, d, d))
    for a in range(ns):
        for c in range(d):
            W[:, d * a + c, c] = val[:, a]
            G[:, d * a + c, c, :] = grad[:, a, :]
    return W, G


def stress(G, lam, mu):
    """sigma = 2 mu eps + lambda tr(eps) I for gradient tensors G[..., i, j]."""
    eps = 0.5 * (G + np.swapaxes(G, -1, -2))
    tr = np.trace(eps, axis1=-2, axis2=-1)
    d = G.shape[-1]
    return 2.0 * mu * eps + lam * tr[..., None, None] * np.eye(d)


class CellMatrices:
    """All cell and boundary-face matrices on the cell [0,h]^d for Q_r^d / Q_{r-1}.

    Matrices are indexed [test, trial].  K-dependent parts are returned for K=1
    and scaled by the caller with the cell's permeability.  With pressure='disc' the
    pressure basis is P_{r-1}^disc and Bint holds the interior-face parts of the SIPG form.
    """

    def __init__(self, d, r, h, lam, mu, rho, alpha, gamma_a=None, gamma_b=None, nq=None, pressure='cont'):
        self.d, self.r, self.h = d, r, h
        self.pressure = pressure
        self.gamma_a = 5e4 * r * (r + 1) if gamma_a is None else gamma_a
        self.gamma_b = 0.5 * r * (r - 1) if gamma_b is None else gamma_b
        self.hF = h ** d  # boundary face: the measure of its cell
        nq = r + 1 if nq is None else nq
        pts, wts = cell_rule(nq, d, h)
        sv, sg = scalar_basis(r, d, pts, h)
        pv, pg = pressure_basis(pressure, r, d, pts, h)
        W, G = vector_fields(sv, sg, d)
        S = stress(G, lam, mu)
        eps = 0.5 * (G + np.swapaxes(G, -1, -2))
        div = np.trace(G, axis1=-2, axis2=-1)
        # mass of the vector space times rho: rho <w, chi>
        self.Mrho = rho * np.einsum('q,qic,qjc->ij', wts, W, W)
        # elasticity volume term <C eps(w), eps(chi)>
        self.Avol = np.einsum('q,qjab,qiab->ij', wts, S, eps)
        # C(chi, q) volume part; rows = pressure test, cols = vector trial
        self.Cvol = -alpha * np.einsum('q,qr,qj->rj', wts, pv, div)
        # <grad q, grad psi> (times K) and <q, psi>
        self.Bvol = np.einsum('q,qra,qsa->rs', wts, pg, pg)
        self.Mp = np.einsum('q,qr,qs->rs', wts, pv, pv)
        # boundary faces: key (axis, side)
        self.Aface, self.Cface, self.Bface_K, self.Bface_pen = {}, {}, {}, {}
        for axis in range(d):
            for side in (0, 1):
                fp, fw, n = face_rule(nq, d, h, axis, side)
                sv_, sg_ = scalar_basis(r, d, fp, h)
                pv_, pg_ = pressure_basis(pressure, r, d, fp, h)
                W_, G_ = vector_fields(sv_, sg_, d)
                S_ = stress(G_, lam, mu)
                Sn = np.einsum('qiab,b->qia', S_, n)  # traction sigma(w) n
                # -<C eps(w) n, chi> - <w, C eps(chi) n> + gamma_a/h_F <w, chi>
                Af = -np.einsum('q,qja,qia->ij', fw, Sn, W_)
                Af += -np.einsum('q,qja,qia->ij', fw, W_, Sn)
                Af += (self.gamma_a / self.hF) * np.einsum('q,qja,qia->ij', fw, W_, W_)
                self.Aface[(axis, side)] = Af
                # alpha <chi . n, q>
                self.Cface[(axis, side)] = alpha * np.einsum('q,qr,qja,a->rj', fw, pv_, W_, n)
                # -<grad q . n, psi> - <q, grad psi . n>   (times K)
                gn = np.einsum('qsa,a->qs', pg_, n)
                self.Bface_K[(axis, side)] = -np.einsum('q,qs,qr->rs', fw, gn, pv_) - np.einsum('q,qs,qr->rs', fw, pv_, gn)
                # gamma_b/h_F <q, psi>
                self.Bface_pen[(axis, side)] = (self.gamma_b / self.hF) * np.einsum('q,qs,qr->rs', fw, pv_, pv_)
        # interior faces (disc only): Bint[axis][(b, a)] = (T1, T2, Pen) for the face between
        # K+ = the lower cell (its side-1 face, n = +e_axis) and K- = the upper cell; a, b = 0
        # for K+, 1 for K-; the block of test functions on cell b and trial functions on cell
        # a is K_a T1 + K_b T2 + Pen
        self.Bint = {}
        if pressure == 'disc':
            sgn = (1.0, -1.0)
            for axis in range(d):
                fp1, fw, n = face_rule(nq, d, h, axis, 1)
                fp0, _, _ = face_rule(nq, d, h, axis, 0)
                v, g = [None, None], [None, None]
                v[0], gr0 = pdisc_basis(r - 1, d, fp1, h)
                v[1], gr1 = pdisc_basis(r - 1, d, fp0, h)
                g[0], g[1] = gr0 @ n, gr1 @ n
                blocks = {}
                for b in (0, 1):
                    for a in (0, 1):
                        # -<{K grad q} . n, [psi]>: q on cell a, average weight 1/2, jump sign of b
                        T1 = -0.5 * sgn[b] * np.einsum('q,qs,qr->rs', fw, g[a], v[b])
                        # -<[q], {K grad psi} . n>
                        T2 = -0.5 * sgn[a] * np.einsum('q,qs,qr->rs', fw, v[a], g[b])
                        Pen = (self.gamma_b / self.hF) * sgn[a] * sgn[b] * np.einsum('q,qs,qr->rs', fw, v[a], v[b])
                        blocks[(b, a)] = (T1, T2, Pen)
                self.Bint[axis] = blocks
