"""Geometric multigrid V-cycle with the patchwise Vanka smoother (Sec. 4).

* Levels l = 0..L on N_l = N_c 2^l cells per axis; A_l is re-assembled on each
  level (the paper uses deal.II level matrices); a per-cell permeability is
  averaged over the children of each coarse cell.
* Prolongation = interpolation of the coarse finite element function at the
  fine nodes, per field, component and Gauss-Radau node (no coarsening in
  time); restriction = its transpose (Sec. 4, list of GMRES-GMG ingredients).
  A discontinuous pressure is prolongated by the L2 projection onto each child
  cell, which is exact: the coarse P_{r-1} piece restricted to a child is in
  P_{r-1} there.
* Patches P_l^m (Eq:DefPlm): the union of the cells that touch grid node
  xi_l^m ("vertex" patches: 4 cells in 2D / 8 in 3D inside, fewer at the
  boundary), or single cells ("cell" patches).  Z_l(P) = every degree of freedom
  (all fields, components and time nodes) of the closed patch.
* Local Vanka operator (Def:VankaOP, Eq:VankaOP0):
      S_P(d) = R_P d + omega A_P^{-1} R_P (b - A d),   A_P = A[Z_P, Z_P]
  and Algorithm 4.1: every sweep applies S_P of every patch to the same
  iterate d, adds the images into z, counts the contributions in p and sets
  d = z / p.
* Coarsest level: direct solve.
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem, problem


def interp_1d(p, Nc):
    """(p*2Nc+1) x (p*Nc+1) matrix evaluating the coarse 1D Q_p basis at the fine lattice nodes."""
    Nf = 2 * Nc
    xf = np.arange(p * Nf + 1) / (p * Nf)
    M = np.zeros((p * Nf + 1, p * Nc + 1))
    for i, x in enumerate(xf):
        c = min(int(np.floor(x * Nc)), Nc - 1)
        xi = x * Nc - c
        v, _ = fem.basis_1d(p, [xi])
        for a in range(p + 1):
            M[i, p * c + a] += v[0, a]
    # a coarse basis function at a coarse node of another index is exactly 0; the
    # evaluation leaves rounding noise (up to ~1e-14 at r = 4)
    M[np.abs(M) < 1e-12] = 0.0
    return sp.csr_matrix(M)


def interp_nd(p, Nc, d):
    """Tensor-product interpolation on the lexicographic lattice (x fastest)."""
    I1 = interp_1d(p, Nc)
    out = I1
    for _ in range(d - 1):
        out = sp.kron(I1, out)
    return out.tocsr()


def disc_prolongation(coarse, fine):
    """P_{r-1}^disc prolongation: on each fine cell, the L2 projection of the parent cell's
    basis functions onto the fine cell's basis."""
    d, r, Nc = coarse.d, coarse.r, coarse.N
    mf = fine.mesh
    pts, wts = fem.cell_rule(r + 1, d, mf.h)
    vf, _ = fine.pbasis(pts)
    Mf = np.einsum('q,qr,qs->rs', wts, vf, vf)
    nl = fine.nploc
    rows, cols, vals = [], [], []
    for cf in range(mf.ncells):
        fi = np.array(mf.cell_index(cf))
        ci = fi // 2
        cc = 0
        for ax in reversed(range(d)):
            cc = cc * Nc + ci[ax]
        # the fine points in the reference coordinates of the parent cell
        vc, _ = coarse.pbasis(((fi % 2)[None, :] + pts) / 2.0)
        blk = np.linalg.solve(Mf, np.einsum('q,qr,qs->rs', wts, vf, vc))
        for i in range(nl):
            for j in range(nl):
                rows.append(cf * nl + i)
                cols.append(cc * nl + j)
                vals.append(blk[i, j])
    out = sp.csr_matrix((vals, (rows, cols)), shape=(fine.nP, coarse.nP))
    # coefficients of fine functions absent from the parent's expansion are zero up to the
    # rounding of the solve with the (monomial) cell mass
    out.data[np.abs(out.data) < 1e-12] = 0.0
    out.eliminate_zeros()
    return out


def prolongation(coarse, fine, k):
    """Space-time prolongation from level l-1 to l: block-diagonal over time nodes and fields."""
    d, r = coarse.d, coarse.r
    IQ = sp.kron(interp_nd(r, coarse.N, d), sp.eye(d))
    IP = interp_nd(r - 1, coarse.N, d) if coarse.pressure == 'cont' else disc_prolongation(coarse, fine)
    one = sp.block_diag([IQ, IQ, IP])
    return sp.block_diag([one] * (k + 1)).tocsr()


def patch_cells(mesh, kind):
    """List of cell-number arrays, one per patch, in the order of the grid nodes (vertex) or cells."""
    d, N = mesh.d, mesh.N
    if kind == 'cell':
        return [np.array([c]) for c in range(mesh.ncells)]
    out = []
    nv1 = N + 1
    for v in range(nv1 ** d):
        vi = []
        t = v
        for _ in range(d):
            vi.append(t % nv1)
            t //= nv1
        ranges = [[c for c in (vi[ax] - 1, vi[ax]) if 0 <= c < N] for ax in range(d)]
        cells = []
        for idx in np.ndindex(*[len(rg) for rg in ranges]):
            ci = [ranges[ax][idx[ax]] for ax in range(d)]
            num = 0
            for ax in reversed(range(d)):
                num = num * N + ci[ax]
            cells.append(num)
        out.append(np.array(sorted(cells)))
    return out


def patch_dofs(blocks, k, cells):
    """Z_l(P): sorted global space-time dof numbers of the closure of the patch cells."""
    v = np.unique(blocks.vdofs[cells].reshape(-1))
    p = np.unique(blocks.pdofs[cells].reshape(-1))
    one = np.concatenate([v, blocks.nv + v, 2 * blocks.nv + p])
    return np.sort(np.concatenate([m * blocks.ns + one for m in range(k + 1)]))


def coarsen_K(K, d, Nf):
    """Per-cell K of the next coarser mesh: the mean over the 2^d children of each cell."""
    Kf = np.asarray(K, dtype=float).reshape((Nf,) * d)  # index order [z][y][x]
    return Kf.reshape(*([Nf // 2, 2] * d)).mean(axis=tuple(range(1, 2 * d, 2))).reshape(-1)


def level_params(prm, d, Nfine, N):
    """Parameters of the level with N cells per axis; a per-cell K given on the finest
    mesh is averaged over the children on every coarser level."""
    if np.ndim(prm.K) == 0:
        return prm
    K = np.asarray(prm.K, dtype=float)
    n = Nfine
    while n > N:
        K = coarsen_K(K, d, n)
        n //= 2
    return problem.Params(rho=prm.rho, lam=prm.lam, mu=prm.mu, alpha=prm.alpha, c0=prm.c0, K=K,
                          gamma_a=prm.gamma_a, gamma_b=prm.gamma_b, pressure=prm.pressure, form=prm.form)


class Level:
    def __init__(self, d, N, r, k, tau, prm, patch_kind):
        self.prob = problem.SlabProblem(d, N, r, k, tau, prm)
        self.A = self.prob.A
        self.n = self.A.shape[0]
        self.patches = []
        self.inv = []
        self.patch_kind = patch_kind

    def build_smoother(self):
        b = self.prob.blocks
        Ad = self.A.tocsr()
        cells = patch_cells(b.mesh, self.patch_kind)
        self.patches = [patch_dofs(b, self.prob.k, c) for c in cells]
        self.inv = [np.linalg.inv(Ad[Z][:, Z].toarray()) for Z in self.patches]
        cnt = np.zeros(self.n)
        for Z in self.patches:
            cnt[Z] += 1
        self.count = cnt


def vanka_smooth(level, b, d, J, omega):
    """Algorithm 4.1 with the local operator of Def:VankaOP, starting from the given d."""
    A = level.A
    d = d.copy()
    for _ in range(J):
        p = np.zeros(level.n)
        z = np.zeros(level.n)
        res = b - A @ d
        for Z, Ainv in zip(level.patches, level.inv):
            y = d[Z] + omega * (Ainv @ res[Z])  # S_P(d)
            z[Z] += y                            # z += E_P y
            p[Z] += 1
        d = z / p
    return d


class Hierarchy:
    """Levels 0..L, transfers and the coarse factorisation."""

    def __init__(self, d, Nc, L, r, k, tau, prm, patch_kind='vertex', J=4, omega=0.7):
        self.J, self.omega = J, omega
        self.levels = [Level(d, Nc * 2 ** l, r, k, tau, level_params(prm, d, Nc * 2 ** L, Nc * 2 ** l), patch_kind)
                       for l in range(L + 1)]
        for lev in self.levels[1:]:
            lev.build_smoother()
        self.P = [None] + [prolongation(self.levels[l - 1].prob.blocks, self.levels[l].prob.blocks, k)
                           for l in range(1, L + 1)]
        A0 = self.levels[0].A.toarray()
        # row-equilibrated dense LU of the coarsest operator (same solution as A0^{-1} b)
        self.coarse_scale = 1.0 / np.abs(A0).max(axis=1)
        self.coarse_lu = sla.lu_factor(self.coarse_scale[:, None] * A0)

    @property
    def fine(self):
        return self.levels[-1]

    def coarse_solve(self, b):
        return sla.lu_solve(self.coarse_lu, self.coarse_scale * b)

    def vcycle(self, l, b):
        """B(l, b): one V-cycle for A_l d = b with zero initial guess."""
        if l == 0:
            return self.coarse_solve(b)
        lev = self.levels[l]
        d = vanka_smooth(lev, b, np.zeros(lev.n), self.J, self.omega)
        r = b - lev.A @ d
        e = self.vcycle(l - 1, self.P[l].T @ r)
        d = d + self.P[l] @ e
        d = vanka_smooth(lev, b, d, self.J, self.omega)
        return d

    def precondition(self, b):
        return self.vcycle(len(self.levels) - 1, b)
