"""Discrete error norms of Sec. 5.1.

* L2(L2): sqrt( sum_n int_{I_n} ||w(t)||^2 dt ), in time with (k+2)-point Gauss
  per slab, in space with (r+2)^d Gauss points per cell.
* L-infinity(L2): the maximum of ||w(t)|| over M = 100 Gauss points per slab
  (the approximation stated right after the prescribed solution Eq:givensolution).
* l-infinity(L2) at the slab ends t_n (Eq:MDN).

The errors measured are ||grad(u - u_h)||, ||v - v_h|| and ||p - p_h||.
"""
import numpy as np

from . import fem, timedg


class _Evaluator:
    def __init__(self, blocks, nq):
        d, r, m = blocks.d, blocks.r, blocks.mesh
        self.b = blocks
        pts, self.wts = fem.cell_rule(nq, d, m.h)
        sv, sg = fem.scalar_basis(r, d, pts, m.h)
        self.W, self.G = fem.vector_fields(sv, sg, d)
        self.pv, _ = blocks.pbasis(pts)
        origins = np.array([m.cell_origin(c) for c in range(m.ncells)])
        self.xs = (origins[:, None, :] + m.h * pts[None, :, :]).reshape(-1, d)
        self.nc, self.nq = m.ncells, len(self.wts)

    def sq_errors(self, Xblock, sol, t):
        """Squared spatial L2 norms of grad(u-u_h), v-v_h, p-p_h at time t for one time-node block."""
        b = self.b
        V = Xblock[:b.nv]
        U = Xblock[b.nv:2 * b.nv]
        Pp = Xblock[2 * b.nv:]
        Uc, Vc, Pc = U[b.vdofs], V[b.vdofs], Pp[b.pdofs]
        gu = np.einsum('qiab,ci->cqab', self.G, Uc).reshape(-1, b.d, b.d)
        vh = np.einsum('qia,ci->cqa', self.W, Vc).reshape(-1, b.d)
        ph = np.einsum('qr,cr->cq', self.pv, Pc).reshape(-1)
        w = np.tile(self.wts, self.nc)
        eg = np.sum(w * np.sum((sol.grad_u(self.xs, t) - gu) ** 2, axis=(1, 2)))
        ev = np.sum(w * np.sum((sol.v(self.xs, t) - vh) ** 2, axis=1))
        ep = np.sum(w * (sol.p(self.xs, t) - ph) ** 2)
        return np.array([eg, ev, ep])


def slab_value(X, ns, k, that):
    """Spatial coefficient vector of the discrete trajectory at reference time that in [-1, 1]."""
    chi = timedg.eval_basis(k, [that])[0]
    return sum(chi[m] * X[m * ns:(m + 1) * ns] for m in range(k + 1))


def error_norms(prob, sol, Xs, t0, M=100):
    """Return dict with 'L2' and 'Linf' arrays (grad u, v, p) and 'l_inf_end' (at slab ends)."""
    b, k, tau = prob.blocks, prob.k, prob.tau
    ev = _Evaluator(b, b.r + 2)
    xg, wg = np.polynomial.legendre.leggauss(k + 2)
    xm, _ = np.polynomial.legendre.leggauss(M)
    l2 = np.zeros(3)
    linf = np.zeros(3)
    lend = np.zeros(3)
    for n, X in enumerate(Xs):
        ts = t0 + n * tau
        for x, w in zip(xg, wg):
            l2 += 0.5 * tau * w * ev.sq_errors(slab_value(X, b.ns, k, x), sol, ts + 0.5 * tau * (1 + x))
        for x in xm:
            linf = np.maximum(linf, np.sqrt(ev.sq_errors(slab_value(X, b.ns, k, x), sol, ts + 0.5 * tau * (1 + x))))
        lend = np.maximum(lend, np.sqrt(ev.sq_errors(slab_value(X, b.ns, k, 1.0), sol, ts + tau)))
    return {'L2': np.sqrt(l2), 'Linf': linf, 'l_inf_end': lend}
