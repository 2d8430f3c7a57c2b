// Layout of the symmetric tiled storage of an nr x nr Schur inverse X (lower triangle in tiles,
// tiles I-major).  Shared by the pack and apply kernels, the host readback and the footprint.
//
// Block rows of 8: nbk = ceil(nr / 8).  Block rows 0 .. nbk-2 are stored as 8x8 tiles (I, J),
// J <= I, at tile index I(I+1)/2 + J, column-major inside (entry (r, c) = X[8I+r][8J+c] at 8c+r).
// The last block row holds rem = nr - 8(nbk-1) rows.  When rem <= 4 and nbk is even it is stored
// as nbk/2 tiles of 4x16 ("half tiles"), tile q covering rows 8(nbk-1) + r, r < 4, and columns
// 16q + c, c < 16, entry (r, c) at 4c + r; the diagonal block is held in full there (both
// triangles).  Otherwise the last block row is stored as 8x8 tiles like the others.  Entries
// beyond nr are zero.  Every tile is 64 values.
#pragma once

namespace stgmg {

constexpr int sym_nbk(int nr) { return (nr + 7) >> 3; }
constexpr bool sym_half(int nr) {
  return sym_nbk(nr) >= 2 && (sym_nbk(nr) & 1) == 0 && nr - 8 * (sym_nbk(nr) - 1) <= 4;
}
// 8x8 tiles (they come first)
constexpr int sym_full_tiles(int nr) {
  return sym_half(nr) ? sym_nbk(nr) * (sym_nbk(nr) - 1) / 2 : sym_nbk(nr) * (sym_nbk(nr) + 1) / 2;
}
// 4x16 tiles (after the 8x8 ones)
constexpr int sym_half_tiles(int nr) { return sym_half(nr) ? sym_nbk(nr) / 2 : 0; }
constexpr int sym_tiles(int nr) { return sym_full_tiles(nr) + sym_half_tiles(nr); }

// Storage of one plane with P tiles interleaved per unit (P = 1 for FP64 values; P = 2 for FP32
// values, so that one 8-byte load per lane reads entry e of two tiles): the 8x8 and the 4x16
// tile counts are each rounded up to a multiple of P with zero tiles (slots), and entry e of slot
// t lies at (floor(t / P) 64 + e) P + t mod P.  P = 1 is the plain tile order.
constexpr int sym_full_slots(int nr, int P) { return (sym_full_tiles(nr) + P - 1) / P * P; }
constexpr int sym_half_slots(int nr, int P) { return (sym_half_tiles(nr) + P - 1) / P * P; }
constexpr int sym_slots(int nr, int P) { return sym_full_slots(nr, P) + sym_half_slots(nr, P); }
// Position of X[row][col], row >= col, within one plane.
constexpr long long sym_slot_elem(int nr, int P, int row, int col) {
  const bool half = sym_half(nr) && (row >> 3) == sym_nbk(nr) - 1;
  const long long t = half ? sym_full_slots(nr, P) + (col >> 4) : (row >> 3) * ((row >> 3) + 1) / 2 + (col >> 3);
  const int e = half ? 4 * (col & 15) + (row & 7) : 8 * (col & 7) + (row & 7);
  return ((t / P) * 64 + e) * P + t % P;
}

}  // namespace stgmg
