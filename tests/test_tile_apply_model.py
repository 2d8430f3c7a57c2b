"""A lane-level model of the tiled Schur-inverse apply of the reduced patch solve (the symmetric
tiles of csrc/tile_layout.h): the pack kernel's map from a stored position to an entry of X, and
the loop a wave runs over the off-diagonal, the pair and diagonal, and the 4x16 sections, with
the lanes' row and column sums, written out in NumPy on the CPU.  It is checked against the dense
product X z for block sizes that cover odd and even numbers of diagonal blocks, the odd blocks'
diagonal list in the free lanes of a last pair tile and in tiles of its own, the 4x16 last block
row, one to four waves per patch and the FP64 / FP32 / BF16 interleavings of P = 1, 2, 4 tiles
per unit.  The positions of the model's pack map must also be those the C layout header gives
(the host readback uses them).  The GPU parity tests compare the kernels themselves with the
oracle; this model is what the layout was checked with before they ran."""
import math

import numpy as np
import pytest

from tests import hostlib

LIB = hostlib.load()


def rup(x, p):
    return (x + p - 1) // p * p


class Layout:
    """Section sizes of one plane of nr rows (the layout header's definitions, restated)."""

    def __init__(self, nr, P):
        self.nr, self.P = nr, P
        self.nbk = (nr + 7) // 8
        self.half = self.nbk >= 2 and self.nbk % 2 == 0 and nr - 8 * (self.nbk - 1) <= 4
        self.nd = self.nbk - 1 if self.half else self.nbk
        self.noff = self.nd * (self.nd - 1) // 2
        self.npair = (self.nd + 1) // 2
        self.ndl = 8 * (self.nd // 2)                    # the odd blocks' diagonal list
        self.ndp = 28 if self.nd % 2 else 0              # of it, in the last pair tile
        self.ndiag = -(-max(self.ndl - self.ndp, 0) // 64)
        self.npd = self.npair + self.ndiag
        self.nh = self.nbk // 2 if self.half else 0
        self.nof2 = rup(self.noff, P)
        self.ntf2 = self.nof2 + rup(self.npd, P)
        self.nsl = self.ntf2 + rup(self.nh, P)

    def list_row(self, s):
        return 16 * (s // 8) + 8 + s % 8


def pack(X, L):
    """The stored plane (positions q of nsl * 64) and the entry (row, col) each holds: slot and
    entry of q, then the section the slot falls in."""
    nr, P = L.nr, L.P
    out = np.zeros(L.nsl * 64, dtype=X.dtype)
    where = {}
    for q in range(L.nsl * 64):
        t, e = q // (64 * P) * P + q % P, q % (64 * P) // P
        r, c = e & 7, e >> 3
        row = col = nr
        s = L.ndl
        if t >= L.ntf2:
            if t - L.ntf2 < L.nh:
                row, col = 8 * (L.nbk - 1) + (e & 3), 16 * (t - L.ntf2) + (e >> 2)
        elif t < L.nof2:
            if t < L.noff:
                I = int((math.sqrt(8.0 * t + 1.0) + 1.0) * 0.5)
                while I * (I - 1) // 2 > t:
                    I -= 1
                while (I + 1) * I // 2 <= t:
                    I += 1
                row, col = 8 * I + r, 8 * (t - I * (I - 1) // 2) + c
        elif t < L.nof2 + L.npair:
            A = 2 * (t - L.nof2)
            B = A + 1
            if r >= c:
                row, col = 8 * A + r, 8 * A + c
            elif B < L.nd:
                row, col = 8 * B + c, 8 * B + r
            else:
                s = c * (c - 1) // 2 + r
        elif t < L.nof2 + L.npd:
            s = L.ndp + 64 * (t - L.nof2 - L.npair) + e
        if s < L.ndl:
            row = col = L.list_row(s)
        if row < nr and col < nr:
            out[q] = 0.5 * (X[row, col] + X[col, row])
            if row >= col:
                where[(row, col)] = q
    return out, where


def wave_apply(st, L, z, w, nw, y):
    """Wave w of nw adds its part of X z into its own y (both of length 8 nbk)."""
    P = L.P
    lane = np.arange(64)
    rr, cc = lane & 7, lane >> 3
    unit = lambda u: [st[(u * 64 + lane) * P + k] for k in range(P)]
    # off-diagonal tiles, batches of 8 tiles; the row partials of block row I flushed on leaving it
    I, J = 1, w * P
    while J >= I:
        J, I = J - I, I + 1
    cur, row = I, np.zeros(64, complex)

    def flush(Ir, row):
        y[8 * Ir:8 * Ir + 8] += row.reshape(8, 8).sum(axis=0)

    u0 = w
    while u0 * P < L.noff:
        xs = []
        for b in range(8 // P):
            u = u0 + b * nw
            xs += unit(u) if u * P < L.noff else [np.zeros(64, complex)] * P
        for k in range(8):
            if (u0 + (k // P) * nw) * P + k % P >= L.noff:
                break
            if I != cur:
                flush(cur, row)
                cur, row = I, np.zeros(64, complex)
            a = xs[k]
            row = row + a * z[8 * J + cc]
            y[8 * J:8 * J + 8] += (a * z[8 * I + rr]).reshape(8, 8).sum(axis=1)
            J += P * nw - (P - 1) if k % P == P - 1 else 1
            while J >= I:
                J, I = J - I, I + 1
        u0 += 8 // P * nw
    if w * P < L.noff:
        flush(cur, row)

    # pair and diagonal tiles, one unit at a time; a pair tile's lanes add their couplings
    def diag_entries(s, a, mask):
        for l in np.nonzero(mask & (s < L.ndl))[0]:
            x = L.list_row(s[l])
            y[x] += a[l] * z[x]

    u0 = w
    while u0 * P < L.npd:
        xs = unit(L.nof2 // P + u0)
        for k in range(P):
            t = u0 * P + k
            if t >= L.npd:
                break
            a = xs[k]
            if t < L.npair:
                A, B = 2 * t, 2 * t + 1
                lo = rr >= cc
                tri = lo | (B < L.nd)
                base = np.where(lo, 8 * A, 8 * B)
                for l in np.nonzero(tri)[0]:
                    i, j = base[l] + rr[l], base[l] + cc[l]
                    y[i] += a[l] * z[j]
                    if i != j:
                        y[j] += a[l] * z[i]
                diag_entries(cc * (cc - 1) // 2 + rr, a, ~tri)
            else:
                diag_entries(L.ndp + 64 * (t - L.npair) + lane, a, np.ones(64, bool))
        u0 += nw

    # 4x16 tiles of the last block row
    if w * P >= L.nh:
        return
    hr, hc, Ih = lane & 3, lane >> 2, 2 * L.nh - 1
    rowh = np.zeros(64, complex)
    u0 = w
    while u0 * P < L.nh:
        xs = []
        for b in range(4 // P):
            u = u0 + b * nw
            xs += unit(L.ntf2 // P + u) if u * P < L.nh else [np.zeros(64, complex)] * P
        for k in range(4):
            q = (u0 + (k // P) * nw) * P + k % P
            if q >= L.nh:
                break
            a, col = xs[k], 16 * q + hc
            rowh += a * z[col]
            if 16 * q < 8 * Ih:
                cs = np.where(col < 8 * Ih, a * z[8 * Ih + hr], 0).reshape(16, 4).sum(axis=1)
                for c in range(16):
                    if 16 * q + c < 8 * Ih:
                        y[16 * q + c] += cs[c]
        u0 += 4 // P * nw
    y[8 * Ih:8 * Ih + 4] += rowh.reshape(16, 4).sum(axis=0)


# nd = 1 .. 12, with and without 4x16 rows; 59 (7 pairs' worth, list in the last pair tile), 89
# (11 blocks: list partly in a tile of its own), 100 and 130 (several list tiles)
SIZES = [1, 5, 8, 9, 12, 16, 20, 27, 36, 50, 59, 60, 61, 64, 89, 100, 130]


@pytest.mark.parametrize("P", [1, 2, 4])
@pytest.mark.parametrize("nr", SIZES)
def test_wave_loop_reproduces_the_product(nr, P):
    rng = np.random.default_rng(nr * 10 + P)
    L = Layout(nr, P)
    X = rng.standard_normal((nr, nr)) + 1j * rng.standard_normal((nr, nr))
    Xs = 0.5 * (X + X.T)
    st, where = pack(X, L)
    # every lower entry held exactly once, at the position of the C layout header
    assert len(where) == nr * (nr + 1) // 2
    for (row, col), q in where.items():
        assert LIB.stgmg_host_sym_slot_elem(nr, P, row, col) == q, (row, col, q)
    z = np.zeros(8 * L.nbk, complex)
    z[:nr] = rng.standard_normal(nr) + 1j * rng.standard_normal(nr)
    ref = Xs @ z[:nr]
    for nw in (1, 2, 4):
        y = np.zeros(8 * L.nbk, complex)
        for w in range(nw):
            yw = np.zeros(8 * L.nbk, complex)
            wave_apply(st, L, z, w, nw, yw)
            y += yw
        assert np.abs(y[:nr] - ref).max() <= 1e-12 * np.abs(ref).max(), (nr, P, nw)
        assert not np.any(y[nr:]), (nr, P, nw)


@pytest.mark.parametrize("nr,stored,full", [(59, 29, 32), (89, 68, 72), (64, 33, 36), (61, 33, 36)])
def test_stored_tiles(nr, stored, full):
    """Tiles per plane (FP64) against those with full 8x8 diagonal tiles: 59 rows = 21
    off-diagonal + 4 pair + 4 half tiles (the list of 3 odd blocks in the last pair tile's free
    lanes); 89 = 55 + 6 + 1 list tile + 6 half tiles; 64 and 61 (8 block rows, no 4x16 row) = 28
    + 4 + 1 list tile."""
    L = Layout(nr, 1)
    assert L.nsl == stored
    assert (L.nbk * (L.nbk - 1) // 2 + L.nbk // 2 if L.half else L.nbk * (L.nbk + 1) // 2) == full
