// Launch wrappers of the HIP kernels in kernels.hip (all enqueue on `st`).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "tile_layout.h"

namespace stgmg {

// Leading dimension of a stored patch inverse of size n: columns padded to a
// multiple of 4 values so that every column starts 16-byte aligned (FP32) /
// 32-byte aligned (FP64); the padding rows hold zeros.
__host__ __device__ inline int inv_ld(int n) { return (n + 3) & ~3; }

// mode 0: y = A x; 1: y = b - A x; 2: y += A x.  lanes = CSR lanes per row (4..64).
void k_csr(hipStream_t st, int mode, int64_t nrows, const int64_t* ptr, const int32_t* col, const double* val,
           const double* x, const double* b, double* y, int lanes);
void k_fill_zero(hipStream_t st, double* a, int64_t n);
// Level operator in factored form A = D^t (x) MM + M^t (x) KK (spatial CSRs MM, KK of n_s rows):
// mode 0: y = A x; mode 1: y = b - A x.  nt = k + 1 <= 4.
struct TimeOp {
  int nt;
  double D[16], mt[4];
};
void k_kron_spmv(hipStream_t st, int mode, const TimeOp& top, int64_t ns, const int64_t* mptr, const int32_t* mcol,
                 const double* mval, const int64_t* kptr, const int32_t* kcol, const double* kval, const double* x,
                 const double* b, double* y, int lanes);
// The same operator with the velocity rows in node-pair form (host_setup.h NodeOp, uploaded):
// d = 2 or 3, nQ Q_r nodes; the pressure rows [2 d nQ, ns) from the spatial CSRs as above.
struct NodeOpDev {
  int d = 0;
  int64_t nQ = 0;
  int lanes = 0;  // lanes per node, 2, 4, 8 or 16 (0: 4 in 2D, 8 in 3D)
  const int64_t* ptr = nullptr;
  const int32_t* col = nullptr;
  const double* m = nullptr;
  const double* a = nullptr;
  const int64_t* cptr = nullptr;
  const int32_t* ccol = nullptr;
  const double* c = nullptr;
};
// Launch shapes in effect: waves per patch of the tiled patch kernel (waves = 1, 2 or 4 fixes it,
// else by patch count: four below 4,096 patches, 8,192 above 96 Schur rows) and lanes per node of
// the operator kernel (o.lanes, else 4 in 2D and 8 in 3D).
int red_sym_waves(int waves, int64_t npatch, int max_nr);
int node_op_lanes(const NodeOpDev& o);

void k_node_op(hipStream_t st, int mode, const TimeOp& top, const NodeOpDev& o, int64_t ns, const int64_t* mptr,
               const int32_t* mcol, const double* mval, const int64_t* kptr, const int32_t* kcol, const double* kval,
               const double* x, const double* b, double* y);
void k_patch_extract_t(hipStream_t st, int64_t p0, int64_t count, int max_np, const int64_t* poff,
                       const int32_t* pdof, const int64_t* ptr, const int32_t* col, const double* val,
                       const int64_t* woff, double* W);
// One matrix of a batched Gauss-Jordan inversion: size n, row-major input at woff
// (overwritten), output rows i < keep of inv(input) written to out + ooff + i * ld_out,
// with column j placed at j (split == 0) or, for j >= split, at ldh + (j - split); all
// other positions of the kept rows are zero.  status[patch] is set on a zero pivot.
struct GjDesc {
  int32_t n, keep, ld_out, split, ldh, patch;
  int64_t woff, ooff;
};
size_t gj_lds_bytes(int max_np, int nb);
int gj_panel_width(int max_np, size_t lds_limit);
void k_gj_invert_f64(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, double* out,
                     int32_t* status);
void k_gj_invert_f32(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, float* out,
                     int32_t* status);
// Patch kernels: y_P = A_P^{-1} R_P r, entry l of patch p written to y[tpos[poff[p] + l]].
// Time-block patch solves.  Constants: tin [nblk][nt] and qout [nt][nblk] complex
// (re, im interleaved), lam [nblk] complex, cplx [nblk].
struct TimeBlockConsts {
  int nt, nblk;
  double tin[2 * 4 * 4], qout[2 * 4 * 4], lam[2 * 4];
  int cplx[4];
};
// dense spatial MM_P^T and KK_P^T (ns x ns, ns = n_P / nt) of patches [p0, p0 + count) at wmm + i * max_ns^2 etc.
void k_patch_extract_spatial_t(hipStream_t st, int64_t p0, int64_t count, int nt, int max_ns, const int64_t* poff,
                               const int32_t* pdof, const int64_t* mptr, const int32_t* mcol, const double* mval,
                               const int64_t* kptr, const int32_t* kcol, const double* kval, double* wmm,
                               double* wkk);
// block matrices (transposed, row-major) for the Gauss-Jordan work area, one per (patch, kept eigenvalue)
void k_form_time_blocks(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int max_ns, const int32_t* ns_of,
                        const double* wmm, const double* wkk, const GjDesc* desc, double* W);
int patch_apply_tb_threads(int max_ns, bool fp32);
void k_patch_apply_tb_f64(hipStream_t st, int64_t npatch, int max_np, const TimeBlockConsts& tb, const int64_t* poff,
                          const int32_t* pdof, const int32_t* tpos, const int64_t* ioff, const double* inv, const double* r, double* y);
void k_patch_apply_tb_f32(hipStream_t st, int64_t npatch, int max_np, const TimeBlockConsts& tb, const int64_t* poff,
                          const int32_t* pdof, const int32_t* tpos, const int64_t* ioff, const float* inv, const double* r, double* y);
// Reduced time-block patch solves (u-equation rows eliminated): per batch item, the node
// mass block, the Schur complement S(lam_a) of every kept eigenvalue (transposed; if complex,
// real form (cplanes = 0) or real and imaginary planes (cplanes = 1)) into the Gauss-Jordan
// work area via desc (nblk + 1 per patch: mass, blocks), and the
// (p-equation, V) block of KK_P straight into the stored layout (out, after the mass inverse).
// nu_of: velocity dofs nU per patch (per time node).
void k_form_reduced_blocks_f64(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int d, int cplanes, int max_ns,
                               int max_nr, const int32_t* ns_of, const int32_t* nu_of, const double* wmm,
                               const double* wkk, const GjDesc* desc, double* W, double* out);
void k_form_reduced_blocks_f32(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int d, int cplanes, int max_ns,
                               int max_nr, const int32_t* ns_of, const int32_t* nu_of, const double* wmm,
                               const double* wkk, const GjDesc* desc, double* W, float* out);
// after the inversion: G = KK_pV ((rho M)^{-1} (x) I_d) replaces KK_pV in the stored layout;
// desc[i * dstride] is the mass descriptor of batch item i, max_npr the largest nP.
void k_fold_reduced_f64(hipStream_t st, int64_t count, int d, int max_nu, int max_npr, const int32_t* ns_of,
                        const int32_t* nu_of, const GjDesc* desc, int dstride, double* out);
void k_fold_reduced_f32(hipStream_t st, int64_t count, int d, int max_nu, int max_npr, const int32_t* ns_of,
                        const int32_t* nu_of, const GjDesc* desc, int dstride, float* out);
// Gauss-Jordan of matrices held entirely in LDS (one workgroup each, descriptors as for
// k_gj_invert_*; cplx: input = real plane then imaginary plane of an n x n complex matrix,
// output Re at column position j and Im at ldh + j).  LDS bytes per workgroup for size max_n:
size_t gj_lds_kernel_bytes(int max_n, bool cplx);
// Batched Gauss-Jordan of matrices in global memory (W, modified in place), one workgroup per
// descriptor, trailing updates on MFMA; same input planes and output conventions as k_gj_lds_*.
// gj_mfma_bytes: its LDS per workgroup.
size_t gj_mfma_bytes(int max_n, bool cplx);
void k_gj_mfma_f64(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, double* out,
                   int32_t* status);
void k_gj_mfma_f32(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, float* out,
                   int32_t* status);
void k_gj_mfma_bf16(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, __bf16* out,
                    int32_t* status);
void k_gj_lds_f64(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                  double* out, int32_t* status);
void k_gj_lds_f32(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                  float* out, int32_t* status);
int patch_apply_red_threads(int max_nr, bool fp32);
// sym: the Schur inverses stored as the symmetric tiles (tile_layout.h) of X = D2^{-1} S^{-1} D1^{-1}
// (see k_pack_red_sym_*), applied by `waves` waves per patch (1 or 4; 0: four on levels of fewer
// than 4,096 patches -- 8,192 above 96 Schur rows -- else one); else square, column-major, padded.
void k_patch_apply_red_f64(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym,
                           int waves, const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof,
                           const int32_t* tpos, const int32_t* pnu, const int64_t* ioff, const double* inv,
                           const double* r, double* y);
void k_patch_apply_red_f32(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym,
                           int waves, const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof,
                           const int32_t* tpos, const int32_t* pnu, const int64_t* ioff, const float* inv,
                           const double* r, double* y);
// Symmetric tiles from square Schur inverses: one (batch item i, kept eigenvalue a) per block m =
// i * nblk + a: S^{-1} square in sq at soff[m] (as written by k_gj_lds_f64 with ld_out = ldr or
// 2 ldr), tiles of X = D2^{-1} S^{-1} D1^{-1}, (X + X^T)/2, written at out + toff[m]:
// ntl = b(b+1)/2 tiles of 64 values, b = ceil(nr/8), lower tiles I-major, row-major inside,
// complex: Re tiles then Im tiles.  D1 = diag(I_nU, mu1), D2 = diag(I_nU, mu2), mu2 = sqrt(lam),
// mu1 = -1/mu2.  All real kept eigenvalues must be positive.
void k_pack_red_sym_f64(hipStream_t st, int64_t count, const TimeBlockConsts& tb, const int32_t* nu_of,
                        const int32_t* nr_of, const int64_t* soff, const int64_t* toff, const double* sq, double* out);
void k_pack_red_sym_f32(hipStream_t st, int64_t count, const TimeBlockConsts& tb, const int32_t* nu_of,
                        const int32_t* nr_of, const int64_t* soff, const int64_t* toff, const double* sq, float* out);
// BF16 storage (__bf16 values; the reduced solves with symmetric tiles only, four tiles per 8-byte
// unit): the same kernels as the FP32 variants above.
void k_gj_invert_bf16(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, __bf16* out,
                      int32_t* status);
void k_gj_lds_bf16(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                   __bf16* out, int32_t* status);
void k_form_reduced_blocks_bf16(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int d, int cplanes,
                                int max_ns, int max_nr, const int32_t* ns_of, const int32_t* nu_of, const double* wmm,
                                const double* wkk, const GjDesc* desc, double* W, __bf16* out);
void k_fold_reduced_bf16(hipStream_t st, int64_t count, int d, int max_nu, int max_npr, const int32_t* ns_of,
                         const int32_t* nu_of, const GjDesc* desc, int dstride, __bf16* out);
void k_pack_red_sym_bf16(hipStream_t st, int64_t count, const TimeBlockConsts& tb, const int32_t* nu_of,
                         const int32_t* nr_of, const int64_t* soff, const int64_t* toff, const double* sq, __bf16* out);
void k_patch_apply_red_bf16(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym,
                            int waves, const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof,
                            const int32_t* tpos, const int32_t* pnu, const int64_t* ioff, const __bf16* inv,
                            const double* r, double* y);
// Block size used by the patch GEMV for patches of at most max_np rows.
int patch_apply_threads(int max_np, bool fp32);
void k_patch_apply_f64(hipStream_t st, int64_t npatch, int max_np, const int64_t* poff, const int32_t* pdof, const int32_t* tpos,
                       const int64_t* ioff, const double* inv, const double* r, double* y);
void k_patch_apply_f32(hipStream_t st, int64_t npatch, int max_np, const int64_t* poff, const int32_t* pdof, const int32_t* tpos,
                       const int64_t* ioff, const float* inv, const double* r, double* y);
// patch images y stored dof-major (slots [tptr[mu], tptr[mu + 1]) of dof mu): d += winv (sum of the slots)
// assign: d = winv (sum of the slots) instead (the first sweep from d = 0, which needs no zero fill)
void k_vanka_update(hipStream_t st, int64_t n, const int64_t* tptr, const double* winv, const double* y, double* d,
                    bool assign = false);
// y = X b for a dense inverse in the padded column layout; part holds dense_gemv_chunks(n) * n doubles
int dense_gemv_chunks(int n);
void k_dense_gemv_t(hipStream_t st, int n, const double* Xt, const double* b, double* part, double* y);
// Multi-workgroup Gauss-Jordan of one row-major n x n matrix (panels of nb <= 32 columns):
// rowscale once, one step per panel, then the un-permuted, re-scaled output.
void k_gj_large_rowscale(hipStream_t st, int n, double* M, double* scl);
// one panel of nb <= 32 columns at k0; P0 and P1: nb x n scratch (the panel, column-major), Wb: nb x n
void k_gj_large_step(hipStream_t st, int n, int k0, int nb, double* M, int* perm, double* P0, double* P1,
                     double* Wb, int32_t* status);
void k_gj_large_output(hipStream_t st, int n, const double* M, const int* src, const double* scl, double* out);
int dot_blocks(int64_t n);
// out[v] (+)= V_v . w for v < m (V rows of length n, leading dimension ldv); partials >= m * dot_blocks(n)
void k_multi_dot(hipStream_t st, const double* V, int64_t ldv, int m, const double* w, int64_t n, double* partials,
                 double* out, int accumulate);
void k_multi_axpy(hipStream_t st, const double* V, int64_t ldv, int m, const double* h, double sign, double* w,
                  int64_t n);
void k_scale_copy(hipStream_t st, const double* src, const double* nrm2, double* dst, int64_t n);
void k_axpby(hipStream_t st, double a, const double* x, double b, const double* y, double* out, int64_t n);
// Source S(t) of the built-in prescribed solution on one level (one time node, n_s values,
// u-equation rows zero): for every node, the sum over its adjacent cells and their
// (r+2)^d Gauss points of w_q phi_node(x_q) f(x_q, t) (v-equation rows) or g (p-equation
// rows).  Tables (host): reference points xq[nq][3], weights wq[nq] (reference cell),
// basis values bq[nloc_r][nq] of Q_r and bp[nloc_{r-1}][nq] of Q_{r-1}.
// disc: pressure rows are cell-major (cell * nlp + j) with the basis values bp[nlp][nq] of the
// broken P_{r-1}, integrated over their own cell only.
struct SourceArgs {
  int d, r, N, nq, disc, nlp;
  int64_t n1, n1p, nv, ns;
  double h, rho, lam, mu, alpha, c0, t, scale;
  const double* tdev;  // if not NULL the time is tdev[tidx] (device memory, read at run time)
  int tidx;
};
void k_source(hipStream_t st, const SourceArgs& a, const double* xq, const double* wq, const double* bq,
              const double* bp, const double* Kcell, double* out);
void k_slab_rhs(hipStream_t st, int nt, int64_t ns, const double* e, const double* mmx, const double* src,
                double* rhs);

}  // namespace stgmg
