// Host-only test exports of the setup code (no HIP): lets CPU tests compare
// the C++ assembly, patch tables, transfers and sources with the oracle.
#include <cstring>
#include <vector>

#include "host_setup.h"
#include "tile_layout.h"

namespace {
stgmg::LevelHost g_level;
stgmg::Csr g_P;
stgmg::NodeOp g_node;
std::vector<double> g_vec;
bool g_disc = false;  // pressure pair of the following builds
bool g_dtu = false;   // Problem B.1 instead of Problem 3.1 in the following builds
}  // namespace

extern "C" {

// Pressure pair of the following builds, prolongations and sizes: 0 = Q_{r-1} (Taylor-Hood),
// 1 = P_{r-1}^disc with the interior penalty form.
void stgmg_host_set_pressure(int disc) { g_disc = disc != 0; }
// Formulation of the following builds and sizes: 0 = Problem 3.1 (v-form), 1 = Problem B.1.
void stgmg_host_set_form(int dtu) { g_dtu = dtu != 0; }

// Build one level; returns n (space-time unknowns) or -1 on error.
long long stgmg_host_build(int d, int r, int k, int N, int patch_kind, double tau, double omega, double rho,
                           double lambda, double mu, double alpha, double c0, const double* Kcell) {
  try {
    long long nc = 1;
    for (int a = 0; a < d; ++a) nc *= N;
    std::vector<double> K(Kcell, Kcell + nc);
    stgmg::BuildOptions o{d, r, k, N, patch_kind, tau, omega, true, true, true, true, g_disc, g_dtu, g_dtu};
    stgmg::Material m{rho, lambda, mu, alpha, c0};
    g_level = stgmg::LevelHost();
    stgmg::build_level(o, m, K, g_level, 4);
    return g_level.n;
  } catch (...) {
    return -1;
  }
}

long long stgmg_host_nnz(int which) {
  const stgmg::Csr& c = which == 0 ? g_level.A : which == 1 ? g_level.MM : which == 3 ? g_level.KK
                       : which == 4 ? g_level.Cface : g_P;
  return (long long)c.col.size();
}

// which: 0 = A, 1 = MM, 2 = last prolongation
void stgmg_host_csr(int which, long long* ptr, int* col, double* val) {
  const stgmg::Csr& c = which == 0 ? g_level.A : which == 1 ? g_level.MM : which == 3 ? g_level.KK
                       : which == 4 ? g_level.Cface : g_P;
  for (size_t i = 0; i < c.ptr.size(); ++i) ptr[i] = c.ptr[i];
  std::memcpy(col, c.col.data(), c.col.size() * sizeof(int));
  std::memcpy(val, c.val.data(), c.val.size() * sizeof(double));
}

long long stgmg_host_npatch(void) { return g_level.npatch; }
long long stgmg_host_patch_total(void) { return (long long)g_level.pdof.size(); }

void stgmg_host_patches(long long* poff, int* pdof, double* winv) {
  for (size_t i = 0; i < g_level.poff.size(); ++i) poff[i] = g_level.poff[i];
  std::memcpy(pdof, g_level.pdof.data(), g_level.pdof.size() * sizeof(int));
  std::memcpy(winv, g_level.winv.data(), g_level.winv.size() * sizeof(double));
}

// Prolongation from an N-cell level to the 2N-cell level (both built here).
long long stgmg_host_prolongation(int d, int r, int k, int Nc) {
  try {
    stgmg::LevelHost C, F;
    std::vector<double> Kc(1, 1.0), Kf(1, 1.0);
    long long ncc = 1, ncf = 1;
    for (int a = 0; a < d; ++a) {
      ncc *= Nc;
      ncf *= 2 * Nc;
    }
    Kc.assign(ncc, 1.0);
    Kf.assign(ncf, 1.0);
    stgmg::Material m{1, 1, 1, 1, 1};
    stgmg::build_level({d, r, k, Nc, 0, 0.1, 0.7, false, false, false, true, g_disc}, m, Kc, C, 4);
    stgmg::build_level({d, r, k, 2 * Nc, 0, 0.1, 0.7, false, false, false, true, g_disc}, m, Kf, F, 4);
    g_P = stgmg::build_prolongation(C, F);
    return (long long)g_P.col.size();
  } catch (...) {
    return -1;
  }
}

void stgmg_host_time(int k, double tau, double* x, double* w, double* Dt, double* mt, double* e) {
  stgmg::TimeConsts T = stgmg::make_time_consts(k, tau);
  for (int i = 0; i <= k; ++i) {
    x[i] = T.x[i];
    w[i] = T.w[i];
    mt[i] = T.mt[i];
    e[i] = T.e[i];
  }
  for (int i = 0; i < (k + 1) * (k + 1); ++i) Dt[i] = T.Dt[i];
}

// Source vector of the built-in solution at time t for the last built level (n_s values).
void stgmg_host_source(double t, double rho, double lambda, double mu, double alpha, double c0, double* out) {
  stgmg::Material m{rho, lambda, mu, alpha, c0};
  stgmg::source_vector(g_level, m, t, g_vec);
  std::memcpy(out, g_vec.data(), g_vec.size() * sizeof(double));
}

void stgmg_host_interpolate(double t, double* out) {
  stgmg::interpolate_solution(g_level, t, g_vec);
  std::memcpy(out, g_vec.data(), g_vec.size() * sizeof(double));
}

// Time-block eigen-decomposition: returns nblk; lam (2*nblk: re, im), cplx (nblk),
// tin (2*nblk*nt), qout (2*nt*nblk), complex values interleaved (re, im).
int stgmg_host_time_blocks(int k, double tau, double* lam, int* cplx, double* tin, double* qout) {
  stgmg::TimeConsts T = stgmg::make_time_consts(k, tau);
  stgmg::TimeBlocks B = stgmg::make_time_blocks(T);
  for (int a = 0; a < B.nblk; ++a) {
    lam[2 * a] = B.lam[a].real();
    lam[2 * a + 1] = B.lam[a].imag();
    cplx[a] = B.is_complex[a];
  }
  for (size_t i = 0; i < B.tin.size(); ++i) {
    tin[2 * i] = B.tin[i].real();
    tin[2 * i + 1] = B.tin[i].imag();
  }
  for (size_t i = 0; i < B.qout.size(); ++i) {
    qout[2 * i] = B.qout[i].real();
    qout[2 * i + 1] = B.qout[i].imag();
  }
  return B.nblk;
}

// KK CSR of the last built level (which = 3 in stgmg_host_csr); which = 4: the boundary part
// of C (Problem B.1 builds), nP rows
// Closed-form sizes: out = {n, nnzA, nnzMM, nnzP, npatch, sum_np, sum_np_ld, max_np, nnzKK,
//                          sum_red_fixed, sum_nr_ldr, max_nr, max_nn, nnzCface}
void stgmg_host_sizes(int d, int r, int k, int N, int patch_kind, long long* out) {
  stgmg::LevelSizes S = stgmg::level_sizes(d, r, k, N, patch_kind, g_disc, g_dtu);
  out[0] = S.n;
  out[1] = S.nnzA;
  out[2] = S.nnzMM;
  out[3] = S.nnzP;
  out[4] = S.npatch;
  out[5] = S.sum_np;
  out[6] = S.sum_np_ld;
  out[7] = S.max_np;
  out[8] = S.nnzKK;
  out[9] = S.sum_red_fixed;
  out[10] = S.sum_nr_ldr;
  out[11] = S.max_nr;
  out[12] = S.max_nn;
  out[13] = S.nnzCface;
  out[14] = S.sum_tiles;
  out[15] = S.sum_tiles2;
  out[16] = S.nodeQQ;
  out[17] = S.nodeQP;
  out[18] = S.sum_tiles4;
}

// Node-pair form of the velocity rows of the last built level (NodeOp): returns the number of
// node pairs, or -1 if the matrices do not have the structure; then the arrays.
long long stgmg_host_node_build(void) {
  if (!stgmg::build_node_op(g_level, g_node, 4)) return -1;
  return (long long)g_node.col.size();
}
long long stgmg_host_node_cnnz(void) { return (long long)g_node.ccol.size(); }
void stgmg_host_node_arrays(long long* ptr, int* col, double* m, double* a, long long* cptr, int* ccol, double* c) {
  for (size_t i = 0; i < g_node.ptr.size(); ++i) ptr[i] = g_node.ptr[i];
  for (size_t i = 0; i < g_node.cptr.size(); ++i) cptr[i] = g_node.cptr[i];
  std::memcpy(col, g_node.col.data(), g_node.col.size() * sizeof(int));
  std::memcpy(m, g_node.m.data(), g_node.m.size() * sizeof(double));
  std::memcpy(a, g_node.a.data(), g_node.a.size() * sizeof(double));
  std::memcpy(ccol, g_node.ccol.data(), g_node.ccol.size() * sizeof(int));
  std::memcpy(c, g_node.c.data(), g_node.c.size() * sizeof(double));
}

// position of X[row][col], row >= col, in one plane of the symmetric tiled storage with P tiles
// interleaved per unit (1: FP64, 2: FP32)
long long stgmg_host_sym_slot_elem(int nr, int P, int row, int col) { return stgmg::sym_slot_elem(nr, P, row, col); }

}  // extern "C"
