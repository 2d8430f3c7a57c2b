"""The reduced time-block patch solve, checked on the CPU with the host-assembled spatial
MM and KK and the host patch tables.

Each spatial block lam MM_P + KK_P has the u-equation rows [-rho M, lam rho M, 0] on the
columns (V, U, P).  So V = lam U - (rho M)^{-1} r_u can be eliminated, and (U, P) solve a
Schur complement S(lam) of n_P/(k+1) - nU rows.  These tests check two things.  First, the
structural facts the elimination uses hold exactly in the assembled matrices.  Second, the
reduced solve, with the index mapping and formulas of the device setup and apply kernels
restated in numpy, reproduces the direct solve for real and complex lam."""
import ctypes

import numpy as np
import pytest

from tests import hostlib

LIB = hostlib.load()


def build(d, N, k, kind, K=1.0):
    Kc = np.full(N ** d, K)
    n = LIB.stgmg_host_build(d, 2, k, N, 1 if kind == 'vertex' else 0, 0.01, 0.7, 1.3, 2.5, 0.8, 0.7, 0.02,
                             hostlib.ptr(Kc))
    assert n > 0
    ns = n // (k + 1)
    MM = hostlib.csr(LIB, 1, ns).toarray()
    KK = hostlib.csr(LIB, 3, ns).toarray()
    npatch = LIB.stgmg_host_npatch()
    poff = np.zeros(npatch + 1, dtype=np.int64)
    pdof = np.zeros(LIB.stgmg_host_patch_total(), dtype=np.int32)
    LIB.stgmg_host_patches(hostlib.ptr(poff), hostlib.ptr(pdof), hostlib.ptr(np.zeros(n)))
    nq = (2 * N + 1) ** d
    return MM, KK, poff, pdof, d * nq, ns


def patch_blocks(MM, KK, poff, pdof, nv, k, p):
    ns = (poff[p + 1] - poff[p]) // (k + 1)
    dofs = pdof[poff[p]:poff[p] + ns]  # time node 0: the spatial numbers
    nU = int(np.sum(dofs < nv))
    return MM[np.ix_(dofs, dofs)], KK[np.ix_(dofs, dofs)], nU


def reduced_solve(MMp, KKp, nU, d, lam, rhs):
    """(lam MM_P + KK_P)^{-1} rhs through the u-equation elimination, with the same
    formulas and index mapping as the device form and apply kernels."""
    ns = MMp.shape[0]
    nP = ns - 2 * nU
    nr = nU + nP
    nn = nU // d
    Mn = MMp[0:nU:d, nU:2 * nU:d]  # rho M on the nodes: component 0 of (u-rows, U columns)
    Minv = np.linalg.inv(Mn)
    S = np.zeros((nr, nr), dtype=complex)
    for x in range(nr):
        for y in range(nr):
            A2 = MMp[nU + x, y] if y < nU else 0.0
            A1 = MMp[nU + x, nU + y] + (KKp[nU + x, y] if y < nU else 0.0)
            A0 = KKp[nU + x, nU + y]
            S[x, y] = lam * lam * A2 + lam * A1 + A0
    Kpv = KKp[2 * nU:, :nU]
    G = np.zeros((nP, nU))  # KK_pV ((rho M)^{-1} (x) I_d), folded at setup
    for x in range(nP):
        for col in range(nU):
            m, c = divmod(col, d)
            G[x, col] = sum(Kpv[x, b * d + c] * Minv[b, m] for b in range(nn))
    ru, rv, rp = rhs[:nU], rhs[nU:2 * nU], rhs[2 * nU:]
    w = np.zeros(nU, dtype=complex)
    for i in range(nU):
        w[i] = sum(Minv[i // d, b] * ru[b * d + i % d] for b in range(nn))
    z = np.concatenate([rv + lam * ru, rp + G @ ru])
    t = np.linalg.solve(S, z)
    return np.concatenate([lam * t[:nU] - w, t])


@pytest.mark.parametrize("d,N,k,kind", [(2, 4, 2, 'vertex'), (2, 3, 1, 'cell'), (3, 2, 1, 'cell'),
                                        (3, 2, 0, 'vertex')])
def test_u_rows_have_the_eliminated_structure(d, N, k, kind):
    MM, KK, poff, pdof, nv, ns = build(d, N, k, kind)
    V, U, P = slice(0, nv), slice(nv, 2 * nv), slice(2 * nv, ns)
    # u-equation rows: MM = [0, rho M, 0], KK = [-rho M, 0, 0]
    assert not MM[V, V].any() and not MM[V, P].any()
    assert not KK[V, U].any() and not KK[V, P].any()
    assert np.array_equal(KK[V, V], -MM[V, U])
    # v-equation rows: MM = [rho M, 0, 0] with the same rho M; KK has no V columns
    assert np.array_equal(MM[U, V], MM[V, U])
    assert not MM[U, U].any() and not MM[U, P].any() and not KK[U, V].any()
    # p-equation rows: no U columns at all, no V columns in MM
    assert not MM[P, V].any() and not MM[P, U].any() and not KK[P, U].any()
    # rho M couples equal components only and is the same scalar matrix for each
    Mv = MM[V, U]
    for c in range(d):
        for c2 in range(d):
            blk = Mv[c::d, c2::d]
            assert (not blk.any()) if c != c2 else np.array_equal(blk, Mv[0::d, 0::d])


@pytest.mark.parametrize("d,N,k,kind", [(2, 4, 2, 'vertex'), (3, 2, 1, 'cell'), (2, 2, 1, 'vertex')])
def test_reduced_solve_reproduces_the_block_inverse(d, N, k, kind):
    MM, KK, poff, pdof, nv, ns = build(d, N, k, kind, K=0.3)
    nt = k + 1
    lam = np.zeros(2 * nt); cplx = np.zeros(nt, dtype=np.int32)
    tin = np.zeros(2 * nt * nt); qout = np.zeros(2 * nt * nt)
    LIB.stgmg_host_time_blocks.restype = ctypes.c_int
    LIB.stgmg_host_time_blocks.argtypes = [ctypes.c_int, ctypes.c_double] + [ctypes.c_void_p] * 4
    nb = LIB.stgmg_host_time_blocks(k, 0.01, *[hostlib.ptr(a) for a in (lam, cplx, tin, qout)])
    lams = lam[0::2][:nb] + 1j * lam[1::2][:nb]
    rng = np.random.default_rng(3)
    npatch = len(poff) - 1
    for p in sorted({0, npatch // 2, npatch - 1, int(rng.integers(npatch))}):  # corner, interior, random
        MMp, KKp, nU = patch_blocks(MM, KK, poff, pdof, nv, k, p)
        assert 0 < nU and nU % d == 0 and MMp.shape[0] - 2 * nU > 0
        for l in list(lams) + [1.7, 0.4 + 2.1j]:
            B = l * MMp + KKp
            rhs = rng.standard_normal(MMp.shape[0]) + 1j * rng.standard_normal(MMp.shape[0])
            ref = np.linalg.solve(B, rhs)
            got = reduced_solve(MMp, KKp, nU, d, l, rhs)
            assert np.abs(got - ref).max() <= 1e-9 * np.abs(ref).max(), (p, l)


@pytest.mark.parametrize("d,r,k,N,kind", [(2, 2, 2, 8, 'vertex'), (3, 2, 1, 4, 'cell'), (2, 2, 1, 4, 'cell'),
                                          (3, 2, 1, 2, 'vertex')])
def test_reduced_storage_sizes_closed_form(d, r, k, N, kind):
    """Closed-form sums of the reduced storage equal the counts over the built patches."""
    MM, KK, poff, pdof, nv, ns = build(d, N, k, kind)
    S = hostlib.sizes(LIB, d, r, k, N, 1 if kind == 'vertex' else 0)
    ld4 = lambda v: (v + 3) // 4 * 4
    fixed = nrl = max_nr = max_nn = tiles = tiles2 = tiles4 = 0
    for p in range(len(poff) - 1):
        nsp = (poff[p + 1] - poff[p]) // (k + 1)
        nU = int(np.sum(pdof[poff[p]:poff[p] + nsp] < nv))
        nP, nn = nsp - 2 * nU, nU // d
        nr = nU + nP
        fixed += nn * ld4(nn) + nU * ld4(nP)
        nrl += nr * ld4(nr)
        ntl = len(tile_entries(nr)[0])
        tiles += ntl
        tiles2 += len(pair_tiles(np.zeros(64 * ntl), nr, 2)) // 64
        tiles4 += len(pair_tiles(np.zeros(64 * ntl), nr, 4)) // 64
        max_nr, max_nn = max(max_nr, nr), max(max_nn, nn)
    assert (S['sum_red_fixed'], S['sum_nr_ldr'], S['max_nr'], S['max_nn']) == (fixed, nrl, max_nr, max_nn)
    assert S['sum_tiles'] == tiles and S['sum_tiles2'] == tiles2 and S['sum_tiles4'] == tiles4


def sym_factors(lam):
    """mu1, mu2 with D1 S(lam) D2 symmetric, D1 = diag(I_nU, mu1 I), D2 = diag(I_nU, mu2 I):
    mu2 = principal sqrt(lam), mu1 = -1/mu2 (then mu2 C^T = (-lam mu1 C)^T and mu1 mu2 = -1)."""
    mu2 = np.sqrt(complex(lam))
    return -1.0 / mu2, mu2


def tile_entries(nr):
    """(row, col) of the 64 entries of each stored tile in order, (-1, -1) where the tile holds a
    zero, the number of off-diagonal tiles and the number of 8x8 tiles.  Block rows of 8, nb of them; when the last one holds at
    most 4 rows and nb is even it is stored last, as nb/2 tiles of 4x16 (entry (r, c) at 4c + r,
    its diagonal block in full), and nd = nb - 1 block rows remain, else nd = nb.  Those are
    stored as 8x8 tiles, entry (r, c) at 8c + r: the off-diagonal tiles (I, J), J < I, I-major;
    then the pair tiles, pair k holding the lower triangle of diagonal block 2k at r >= c and
    the strict lower triangle of block 2k+1 transposed at r < c; then the diagonal tiles.  The
    diagonal entries of the odd blocks form one list, entry s being row 16(s // 8) + 8 + s % 8;
    when nd is odd the last pair has no block 2k+1 and its lanes r < c hold the list's first 28
    entries (s = c(c-1)/2 + r); the rest fill the diagonal tiles 64 to a tile."""
    nb = (nr + 7) // 8
    half = nb >= 2 and nb % 2 == 0 and nr - 8 * (nb - 1) <= 4
    nd = nb - 1 if half else nb
    ndl = 8 * (nd // 2)
    ent = lambda row, col: (row, col) if row < nr and col < nr else (-1, -1)
    lst = lambda s: ent(16 * (s // 8) + 8 + s % 8, 16 * (s // 8) + 8 + s % 8) if s < ndl else (-1, -1)
    tiles = [[ent(8 * I + e % 8, 8 * J + e // 8) for e in range(64)] for I in range(nd) for J in range(I)]
    for k in range((nd + 1) // 2):
        A, B = 2 * k, 2 * k + 1
        tile = []
        for e in range(64):
            r, c = e % 8, e // 8
            if r >= c:
                tile.append(ent(8 * A + r, 8 * A + c))
            elif B < nd:
                tile.append(ent(8 * B + c, 8 * B + r))
            else:
                tile.append(lst(c * (c - 1) // 2 + r))
        tiles.append(tile)
    s0 = 28 if nd % 2 else 0
    tiles += [[lst(s0 + 64 * m + e) for e in range(64)] for m in range(-(-max(ndl - s0, 0) // 64))]
    nfull = len(tiles)
    if half:
        tiles += [[ent(8 * (nb - 1) + e % 4, 16 * q + e // 4) for e in range(64)] for q in range(nb // 2)]
    return tiles, nd * (nd - 1) // 2, nfull


def pack_tiles(X, nr):
    """The stored tiles of tile_entries(nr) of the symmetric X, concatenated; X is symmetrised as
    (X + X^T)/2."""
    Xs = 0.5 * (X + X.T)
    return np.array([Xs[row, col] if row >= 0 else 0.0 for tile in tile_entries(nr)[0] for row, col in tile])


def pair_tiles(tiles, nr, P):
    """The storage order with P tiles interleaved per unit (P = 2 for FP32, 4 for BF16 values): the
    off-diagonal, the pair and diagonal, and the 4x16 tile counts each padded with zero tiles to a
    multiple of P, then entry e of slot t at (t // P * 64 + e) * P + t % P."""
    _, no, nf = tile_entries(nr)
    T = tiles.reshape(-1, 64)
    pad = lambda A: np.concatenate([A, np.zeros((-len(A) % P, 64), dtype=A.dtype)])
    S = np.concatenate([pad(T[:no]), pad(T[no:nf]), pad(T[nf:])])
    return S.reshape(-1, P, 64).transpose(0, 2, 1).reshape(-1)


def tile_apply(tiles, nr, zt):
    """y = X zt from the stored tiles the way the waves do it: every entry X[row][col] adds
    X[row][col] zt[col] to the row and, off the diagonal and outside the diagonal block that the
    4x16 tiles hold in full, X[row][col] zt[row] to the column."""
    nb = (nr + 7) // 8
    y = np.zeros(8 * nb, dtype=complex)
    entries, _, nfull = tile_entries(nr)
    for t, tile in enumerate(entries):
        for e, (row, col) in enumerate(tile):
            if row < 0:
                continue
            v = tiles[64 * t + e]
            y[row] += v * zt[col]
            if row != col and (t < nfull or col < 8 * (nb - 1)):
                y[col] += v * zt[row]
    return y


@pytest.mark.parametrize("P", [1, 2, 4])
@pytest.mark.parametrize("nr", [1, 5, 8, 9, 12, 13, 16, 18, 20, 21, 27, 29, 36, 40, 59, 60, 61, 64, 84, 89, 100])
def test_tile_layout_positions(nr, P):
    """The kernels' and the readback's position of X[row][col] (tile_layout.h) is the position
    of that entry in pack_tiles (P = 1) and in its FP32 and BF16 interleavings (P = 2, 4); every stored tile is 64
    values, and the 4x16 tiles are used exactly when the last block row holds at most 4 rows and
    the block rows are even."""
    X = np.arange(nr * nr, dtype=float).reshape(nr, nr)
    X = X + X.T + 1.0  # distinct symmetric values
    tiles = pack_tiles(X, nr).real
    stored = pair_tiles(tiles, nr, P)
    assert np.count_nonzero(stored) == np.count_nonzero(tiles)
    seen = set()
    for row in range(nr):
        for col in range(row + 1):
            e = LIB.stgmg_host_sym_slot_elem(nr, P, row, col)
            assert stored[e] == 0.5 * (X[row, col] + X[col, row]), (row, col, e)
            seen.add(e)
    assert len(seen) == nr * (nr + 1) // 2
    nb = (nr + 7) // 8
    entries, noff, nfull = tile_entries(nr)
    half = len(entries) > nfull
    assert half == (nb >= 2 and nb % 2 == 0 and nr - 8 * (nb - 1) <= 4)
    # every lower entry is held once, except the upper triangle of the diagonal block in 4x16 tiles
    held = [(r, c) for tile in entries for r, c in tile if r >= 0]
    assert len(held) == len(set(held))
    assert {(r, c) for r, c in held if r >= c} == {(r, c) for r in range(nr) for c in range(r + 1)}
    assert all(r // 8 == nb - 1 and c // 8 == nb - 1 for r, c in held if r < c)
    # the stored 8x8 tiles: the triangles of nd diagonal blocks take ceil(nd/2) pair tiles plus
    # the diagonal list of the odd blocks beyond what a last, half-empty pair holds
    nd = nb - 1 if half else nb
    ndiag = -(-max(8 * (nd // 2) - (28 if nd % 2 else 0), 0) // 64)
    assert noff == nd * (nd - 1) // 2 and nfull == noff + (nd + 1) // 2 + ndiag


@pytest.mark.parametrize("d,N,k,kind", [(2, 4, 2, 'vertex'), (3, 2, 1, 'cell'), (2, 2, 1, 'vertex')])
def test_symmetric_tiles_reproduce_the_schur_inverse(d, N, k, kind):
    """The balanced scaling makes D1 S(lam) D2 symmetric for real and complex lam, and the
    packed lower tiles of X = (D1 S D2)^{-1}, applied as D2 X D1 z, reproduce S(lam)^{-1} z."""
    MM, KK, poff, pdof, nv, ns = build(d, N, k, kind, K=0.3)
    rng = np.random.default_rng(4)
    for p in sorted({0, (len(poff) - 1) // 2, len(poff) - 2}):
        MMp, KKp, nU = patch_blocks(MM, KK, poff, pdof, nv, k, p)
        nsp = MMp.shape[0]
        nP = nsp - 2 * nU
        nr = nU + nP
        for lam in (1.7, 0.4 + 2.1j, 3.3 - 0.7j):
            S = np.zeros((nr, nr), dtype=complex)
            for x in range(nr):
                for y in range(nr):
                    A2 = MMp[nU + x, y] if y < nU else 0.0
                    A1 = MMp[nU + x, nU + y] + (KKp[nU + x, y] if y < nU else 0.0)
                    S[x, y] = lam * lam * A2 + lam * A1 + KKp[nU + x, nU + y]
            mu1, mu2 = sym_factors(lam)
            D1 = np.diag([1.0] * nU + [mu1] * nP)
            D2 = np.diag([1.0] * nU + [mu2] * nP)
            Ssym = D1 @ S @ D2
            assert np.abs(Ssym - Ssym.T).max() <= 1e-13 * np.abs(Ssym).max()
            X = np.linalg.inv(Ssym)
            tiles = pack_tiles(X, nr)
            assert len(tiles) == 64 * len(tile_entries(nr)[0])
            z = rng.standard_normal(nr) + 1j * rng.standard_normal(nr)
            zt = np.zeros(8 * ((nr + 7) // 8), dtype=complex)
            zt[:nr] = np.diag(D1) * z
            y = np.diag(D2) * tile_apply(tiles, nr, zt)[:nr]
            ref = np.linalg.solve(S, z)
            assert np.abs(y - ref).max() <= 1e-11 * np.abs(ref).max(), (p, lam)
