// Layout of the symmetric tiled storage of an nr x nr Schur inverse X (its lower triangle, in tiles
// of 64 values).  Shared by the pack and apply kernels, the host readback and the footprint.
//
// Block rows of 8: nbk = ceil(nr / 8); the last one holds rem = nr - 8(nbk-1) rows.  When rem <= 4
// and nbk is even, that last block row is stored as nbk/2 "half tiles" of 4x16 (tile q: rows
// 8(nbk-1) + r, r < 4, columns 16q + c, c < 16, entry (r, c) at 4c + r; its diagonal block held in
// full, both triangles), and nd = nbk - 1 block rows remain; otherwise nd = nbk.  The nd block rows
// are held in 8x8 tiles, entry (r, c) at 8c + r, in this order:
//  * off-diagonal tiles (I, J), J < I < nd, I-major: tile I(I-1)/2 + J holds X[8I+r][8J+c];
//  * ceil(nd/2) pair tiles: pair k holds the lower triangle of the diagonal block A = 2k at r >= c
//    (X[8A+r][8A+c]) and the strict lower triangle of the diagonal block B = 2k+1, transposed, at
//    r < c (X[8B+c][8B+r]);
//  * the diagonals of the odd blocks B, as one list: entry s < 8 floor(nd/2) is X[x][x] with
//    x = 16 floor(s/8) + 8 + s mod 8.  When nd is odd the last pair tile has no block B; its lanes
//    r < c hold the list's first 28 entries (s = c(c-1)/2 + r), and the rest fill diagonal tiles
//    at entry 64 m + e of tile m.
// Entries beyond nr, and beyond the list, are zero.
#pragma once

namespace stgmg {

constexpr int sym_nbk(int nr) { return (nr + 7) >> 3; }
constexpr bool sym_half(int nr) {
  return sym_nbk(nr) >= 2 && (sym_nbk(nr) & 1) == 0 && nr - 8 * (sym_nbk(nr) - 1) <= 4;
}
// block rows held in 8x8 tiles
constexpr int sym_nd(int nr) { return sym_half(nr) ? sym_nbk(nr) - 1 : sym_nbk(nr); }
constexpr int sym_off_tiles(int nr) { return sym_nd(nr) * (sym_nd(nr) - 1) / 2; }
constexpr int sym_pair_tiles(int nr) { return (sym_nd(nr) + 1) / 2; }
// entries of the odd blocks' diagonal list, and how many of them the last pair tile holds
constexpr int sym_dlist(int nr) { return 8 * (sym_nd(nr) / 2); }
constexpr int sym_dlist_in_pair(int nr) { return (sym_nd(nr) & 1) ? 28 : 0; }
constexpr int sym_diag_tiles(int nr) {
  return sym_dlist(nr) > sym_dlist_in_pair(nr) ? (sym_dlist(nr) - sym_dlist_in_pair(nr) + 63) / 64 : 0;
}
// 8x8 tiles (they come first)
constexpr int sym_full_tiles(int nr) { return sym_off_tiles(nr) + sym_pair_tiles(nr) + sym_diag_tiles(nr); }
// 4x16 tiles (after the 8x8 ones)
constexpr int sym_half_tiles(int nr) { return sym_half(nr) ? sym_nbk(nr) / 2 : 0; }
constexpr int sym_tiles(int nr) { return sym_full_tiles(nr) + sym_half_tiles(nr); }

// Storage of one plane with P tiles interleaved per unit (P = 1 for FP64 values; P = 2 for FP32
// values and P = 4 for BF16 values, so that one 8-byte load per lane reads entry e of P tiles):
// three sections, the off-diagonal tiles, the pair and diagonal tiles, the 4x16 tiles, each
// rounded up to a multiple of P with zero tiles (slots); entry e of slot t lies at
// (floor(t / P) 64 + e) P + t mod P.  P = 1 is the plain tile order.
constexpr int rup_p(int n, int P) { return (n + P - 1) / P * P; }
constexpr int sym_off_slots(int nr, int P) { return rup_p(sym_off_tiles(nr), P); }
constexpr int sym_full_slots(int nr, int P) {
  return sym_off_slots(nr, P) + rup_p(sym_pair_tiles(nr) + sym_diag_tiles(nr), P);
}
constexpr int sym_half_slots(int nr, int P) { return rup_p(sym_half_tiles(nr), P); }
constexpr int sym_slots(int nr, int P) { return sym_full_slots(nr, P) + sym_half_slots(nr, P); }
// Position of X[row][col], row >= col, within one plane.
constexpr long long sym_slot_elem(int nr, int P, int row, int col) {
  const int I = row >> 3, J = col >> 3, r = row & 7, c = col & 7;
  long long t = 0;
  int e = 0;
  if (sym_half(nr) && I == sym_nbk(nr) - 1) {
    t = sym_full_slots(nr, P) + (col >> 4);
    e = 4 * (col & 15) + r;
  } else if (J < I) {
    t = I * (I - 1) / 2 + J;
    e = 8 * c + r;
  } else if ((I & 1) == 0) {  // block A of pair I/2
    t = sym_off_slots(nr, P) + I / 2;
    e = 8 * c + r;
  } else if (r != c) {  // block B of pair I/2, transposed
    t = sym_off_slots(nr, P) + I / 2;
    e = 8 * r + c;
  } else {  // entry s of the diagonal list
    const int s = 8 * (I / 2) + r;
    if (s < sym_dlist_in_pair(nr)) {
      int cc = 1;
      while ((cc + 1) * cc / 2 <= s) ++cc;
      t = sym_off_slots(nr, P) + sym_pair_tiles(nr) - 1;
      e = 8 * cc + (s - cc * (cc - 1) / 2);
    } else {
      const int s2 = s - sym_dlist_in_pair(nr);
      t = sym_off_slots(nr, P) + sym_pair_tiles(nr) + s2 / 64;
      e = s2 % 64;
    }
  }
  return ((t / P) * 64 + e) * P + t % P;
}

}  // namespace stgmg
