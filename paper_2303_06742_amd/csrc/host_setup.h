// Host-side construction of the level hierarchy: time constants, element
// integrals, space-time operators in CSR, patch tables and grid transfers.
// Plain C++17, no HIP; the device side only uploads what is built here.
#pragma once
#include <array>
#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace stgmg {

struct Material {
  double rho, lambda, mu, alpha, c0;
};

// dG(k) on one slab: right Gauss-Radau nodes/weights on [-1,1], Lagrange basis
// at those nodes; Dt[b*(k+1)+a] (row b = test), mt[b] = tau/2 w_b (diagonal
// M^t), e[b] = chi_b(-1).
struct TimeConsts {
  int k = 0;
  double tau = 0;
  std::vector<double> x, w, Dt, mt, e;
};
TimeConsts make_time_consts(int k, double tau);

// Eigen-decomposition of T = (M^t)^{-1} D^t = Q diag(lambda) Q^{-1}, used to split a
// space-time patch solve A_P^{-1} = (Q x I) blockdiag((lambda_a MM_P + KK_P)^{-1})
// (Q^{-1} (M^t)^{-1} x I) into spatial solves.  Kept eigenvalues: every real one and
// the one with positive imaginary part of each complex-conjugate pair (its partner's
// contribution is the complex conjugate).
struct TimeBlocks {
  int nt = 0;       // k + 1
  int nblk = 0;     // kept eigenvalues
  std::vector<std::complex<double>> lam;   // [nblk]
  std::vector<int> is_complex;             // [nblk]
  std::vector<std::complex<double>> tin;   // [nblk][nt]: rows of Q^{-1} (M^t)^{-1}
  std::vector<std::complex<double>> qout;  // [nt][nblk]: columns of Q (a pair counts twice via 2 Re)
};
TimeBlocks make_time_blocks(const TimeConsts& T);

// Broken pressure space P_p^disc on a cell: the monomials prod_ax (xi_ax - 1/2)^alpha_ax in
// the cell-centred reference coordinate, |alpha| <= p, in the lexicographic order of the
// (p+1)^d lattice (x fastest) restricted to total degree <= p.
std::vector<std::array<int, 3>> pdisc_exponents(int p, int d);

// Element and boundary-face matrices of one cell [0,h]^d, indexed [test][trial]
// row-major.  Vector local index = d*a + c (a = lexicographic local node).  The pressure
// basis is Q_{r-1} (Taylor-Hood) or, with disc, P_{r-1}^disc; then the interior faces
// normal to each axis carry the symmetric interior penalty parts of Def:B: for the face
// between K+ (the lower cell, n = +e_axis) and K- (the upper cell), the block of test
// functions on cell b and trial functions on cell a (0 = K+, 1 = K-) is
// K_a BiT1 + K_b BiT2 + BiPen, each stored at [axis][2 * b + a].
struct CellMats {
  int d = 0, r = 0;
  bool disc = false;
  int nls = 0, nlv = 0, nlp = 0;  // local scalar Q_r, vector, pressure counts
  double gamma_a = 0, gamma_b = 0, hF = 0;
  std::vector<double> Mrho, Avol, Cvol, Bvol, Mp;  // Cvol: [p-test][v-trial]
  std::vector<double> Aface[6], Cface[6], BfaceK[6], Bpen[6];  // face = 2*axis + side
  std::vector<double> BiT1[3][4], BiT2[3][4], BiPen[3][4];    // disc only
};
CellMats make_cell_mats(int d, int r, double h, const Material& m, bool disc = false);

struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};

struct LevelHost {
  int d = 0, r = 0, k = 0, N = 0;
  bool disc = false;        // pressure P_{r-1}^disc (cell-major, nlp per cell) instead of Q_{r-1}
  bool dtu = false;         // Problem B.1: -C(d_t u, psi) in the p-equation (MM's p-rows carry -C on U)
  int nlp = 0;              // pressure dofs per cell (disc)
  int64_t n1 = 0, n1p = 0;  // lattice points per axis, Q_r and Q_{r-1}
  int64_t nQ = 0, nP = 0, nv = 0, ns = 0, n = 0;
  std::vector<double> Kcell;
  Csr A;   // space-time operator D^t (x) MM + M^t (x) KK
  Csr MM;  // spatial MM (finest level, and every smoothed level for time-block patch solves)
  Csr KK;  // spatial KK (smoothed levels, time-block patch solves)
  // patches: dofs of patch p are pdof[poff[p] .. poff[p+1]) in increasing order
  int64_t npatch = 0;
  std::vector<int64_t> poff;
  std::vector<int32_t> pdof;
  // dof-major slots: entry t of pdof has slot tpos[t]; the slots of dof mu are
  // [tptr[mu], tptr[mu+1]), in increasing patch order
  std::vector<int64_t> tptr;
  std::vector<int32_t> tpos;
  std::vector<double> winv;  // omega / (number of patches containing mu)
  // Problem B.1: the boundary-face part of C (nP rows, columns = velocity dofs 0..nv-1): the
  // slab right-hand side's jump uses only the volume part of C on u^{n-1}
  Csr Cface;
};

struct BuildOptions {
  int d, r, k, N;
  int patch_kind;  // 0 cell, 1 vertex
  double tau, omega;
  bool need_patches;
  bool need_MM;
  bool need_KK = false;
  bool need_A = true;  // the assembled space-time CSR (otherwise only the spatial MM, KK)
  bool disc = false;   // pressure pair Q_r^d / P_{r-1}^disc with the SIPG form
  bool dtu = false;    // Problem B.1 instead of Problem 3.1
  bool need_Cface = false;  // build LevelHost::Cface (Problem B.1, finest level)
};

// Assemble one level.  Kcell: per-cell K (N^d values).
void build_level(const BuildOptions& o, const Material& m, const std::vector<double>& Kcell, LevelHost& L,
                 int nthreads);

// The velocity rows of a level's spatial matrices by pairs of Q_r nodes.  In the rows of one
// time-node block, ordered (u-equation, v-equation, p-equation) against the columns (V, U, P),
// Problem 3.1 and Problem B.1 both have
//   MM = [[0, rhoM (x) I_d, 0], [rhoM (x) I_d, 0, 0], [...]],  KK = [[-rhoM (x) I_d, 0, 0], [0, A, C^T], [...]],
// so the velocity rows need, per pair of nodes (i, j) that share a cell, the scalar rhoM_ij and
// the d x d block A_ij, and per pair (node i, pressure dof q) the d values C^T_{(i,c), q}.
struct NodeOp {
  int d = 0;
  int64_t nQ = 0;
  std::vector<int64_t> ptr;   // nQ + 1: node pairs of node i
  std::vector<int32_t> col;   // node j
  std::vector<double> m;      // rhoM_ij
  std::vector<double> a;      // A_ij, row-major d x d (row = component of i)
  std::vector<int64_t> cptr;  // nQ + 1: pressure dofs coupled to node i
  std::vector<int32_t> ccol;  // pressure dof q
  std::vector<double> c;      // C^T_{(i,c), q}, d values per pair
};
// Extract the node-pair form from the spatial MM and KK of a level (rows sorted by column or
// not).  Returns false, leaving `out` empty, if the matrices do not have the block structure
// above exactly (the equal rhoM blocks included).
bool build_node_op(const LevelHost& L, NodeOp& out, int nthreads);

// Space-time prolongation from the coarse level to the next finer one.
Csr build_prolongation(const LevelHost& coarse, const LevelHost& fine, int nthreads = 1);
Csr transpose(const Csr& a, int64_t ncols_out);
// Transpose of a block-diagonal matrix: rows [rb[i], rb[i+1]) have their columns in
// [cb[i], cb[i+1]) (checked); the blocks are transposed in parallel.
Csr transpose_block_diag(const Csr& a, int64_t ncols_out, const std::vector<int64_t>& rb,
                         const std::vector<int64_t>& cb, int nthreads);

// Closed-form sizes of one level, without building it (exact structural counts).
struct LevelSizes {
  int64_t n = 0, ns = 0, nnzA = 0, nnzMM = 0, nnzP = 0;  // nnzP: prolongation into this level
  int64_t npatch = 0, sum_np = 0, sum_np_ld = 0;         // sum n_P, sum n_P * inv_ld(n_P)
  int64_t sum_ns_ldh = 0;  // sum over patches of ns * inv_ld(ns), ns = n_P / (k+1)
  int64_t nnzKK = 0;       // spatial KK
  int max_np = 0;
  // reduced time-block solves (per patch: nn nodes, nU = d nn, nP pressure dofs, nr = nU + nP)
  int64_t sum_red_fixed = 0;  // sum of nn * inv_ld(nn) + nU * inv_ld(nP)
  int64_t sum_nr_ldr = 0;     // sum of nr * inv_ld(nr)
  int64_t alg_red_fixed = 0;  // sum of nn^2 + nP nU
  int64_t sum_nr2 = 0;        // sum of nr^2
  int64_t sum_tiles = 0;      // sum of sym_tiles(nr): 64-value tiles of the symmetric storage (FP64)
  int64_t sum_tiles2 = 0;     // sum of sym_slots(nr, 2): the same with the FP32 pairing
  int64_t sum_tiles4 = 0;     // sum of sym_slots(nr, 4): the same with four BF16 tiles per unit
  int max_nr = 0, max_nn = 0;
  int64_t nP = 0;
  int64_t nnzCface = 0;  // Problem B.1: nonzeros of the boundary part of C (LevelHost::Cface)
  int64_t nodeQQ = 0;    // NodeOp pairs of Q_r nodes sharing a cell
  int64_t nodeQP = 0;    // NodeOp pairs (Q_r node, pressure dof) sharing a cell
};
LevelSizes level_sizes(int d, int r, int k, int N, int patch_kind, bool disc = false, bool dtu = false);

// Built-in prescribed solution u_i = S sin t, p = S cos t, S = prod sin(pi x_j):
// source vector S(t) of one time node (u-eq rows zero), and nodal interpolant.
void source_vector(const LevelHost& L, const Material& m, double t, std::vector<double>& out);
// Reference-cell tables for the device source: (r+2)^d Gauss points xq[nq][3] (on [0,1]^d),
// weights wq[nq] (reference cell, summing to 1), basis values bq[(r+1)^d][nq] and
// bp[nlp][nq] of the pressure basis (Q_{r-1}, or P_{r-1}^disc with disc).
void source_tables(int d, int r, std::vector<double>& xq, std::vector<double>& wq, std::vector<double>& bq,
                   std::vector<double>& bp, bool disc = false);
void interpolate_solution(const LevelHost& L, double t, std::vector<double>& out);

}  // namespace stgmg
