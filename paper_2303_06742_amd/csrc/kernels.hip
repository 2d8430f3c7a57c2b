// HIP kernels for gfx950 (CDNA4, wave64) of the GMRES-GMG slab solver.
//
//   csr_residual       r = b - A x  or  y = A x      (level operator, Eq:DefAn)
//   csr_accumulate     y += A x                       (prolongation, Sec. 4)
//   patch_extract_t    A_P^T into a dense work buffer (Def:VankaOP, A_P = A[Z_P, Z_P])
//   gj_invert          blocked Gauss-Jordan inverse with scaled partial pivoting
//   patch_apply        y_P = A_P^{-1} R_P r           (stored inverses, FP64 or FP32)
//   vanka_update       d += omega/p * sum_P E_P y_P   (Alg. 4.1, atomics-free pull)
//   dense_gemv_t       coarse solve with the stored inverse
//   dot_partials / reduce_partials / multi_axpy / scale_copy: FGMRES BLAS-1, fixed
//                      reduction order (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstdlib>

#include "kernels.h"

namespace stgmg {
namespace dev {

constexpr int WAVE = 64;

// Workgroups are dispatched round-robin over the XCDs, each with its own L2.  xcd_block maps
// the dispatch index b of nb blocks to a logical block index such that every XCD processes
// one contiguous range of logical blocks: neighbouring rows, which read the same vector
// entries, then meet in the same L2.  A bijection on [0, nb).  (Measured on the 256^2 dG(2)
// workload: it helps the gathering Vanka update, and slows the streaming SpMV and patch
// kernels, whose round-robin order keeps the whole chip on one moving address window.)
constexpr int NXCD = 8;
__device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % NXCD, i = b / NXCD, q = nb / NXCD, rem = nb % NXCD;
  return x * q + (x < rem ? x : rem) + i;
}

// Chunked variant: chunks of c consecutive logical blocks go round-robin to the XCDs, so that
// neighbours within a chunk share an L2 while the XCDs stay on one moving address window.
// The blocks past the last whole round of NXCD chunks keep their index.  c <= 0: identity.
// A bijection on [0, nb).
__device__ inline int64_t xcd_chunk(int64_t b, int64_t nb, int64_t c) {
  if (c <= 0) return b;
  const int64_t nfull = nb / (NXCD * c) * (NXCD * c);
  if (b >= nfull) return b;
  const int64_t x = b % NXCD, i = b / NXCD;
  return ((i / c) * NXCD + x) * c + i % c;
}

template <int G>
__device__ inline double group_sum(double v) {
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
  return v;
}

// ---------------------------------------------------------------- CSR
// G lanes per row; BS threads per block.  mode 0: y = A x; mode 1: y = b - A x.
template <int G, int MODE>
__global__ void __launch_bounds__(256) csr_kernel(int64_t nrows, const int64_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ col, const double* __restrict__ val,
                                                  const double* __restrict__ x, const double* __restrict__ b,
                                                  double* __restrict__ y) {
  const int lane = threadIdx.x % G;
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / G;
  if (row >= nrows) return;
  const int64_t s = ptr[row], e = ptr[row + 1];
  double acc = 0.0;
  for (int64_t p = s + lane; p < e; p += G) acc += val[p] * x[col[p]];
  acc = group_sum<G>(acc);
  if (lane == 0) {
    if (MODE == 0) y[row] = acc;
    if (MODE == 1) y[row] = b[row] - acc;
    if (MODE == 2) y[row] += acc;
  }
}

template <int G, int MODE>
static void launch_csr(hipStream_t st, int64_t nrows, const int64_t* ptr, const int32_t* col, const double* val,
                       const double* x, const double* b, double* y) {
  if (nrows == 0) return;
  const int bs = 256;
  const int64_t rows_per_block = bs / G;
  const int64_t grid = (nrows + rows_per_block - 1) / rows_per_block;
  hipLaunchKernelGGL((csr_kernel<G, MODE>), dim3(grid), dim3(bs), 0, st, nrows, ptr, col, val, x, b, y);
}

// Factored level operator: G lanes per spatial row i read the row of MM and of KK once
// and accumulate u_a = MM[i,:] x_a, v_a = KK[i,:] x_a for every time node a; then
// (A x)_b[i] = sum_a D[b][a] u_a + mt[b] v_b.
template <int G, int MODE, int NT>
__device__ inline void kron_row(const TimeOp& top, int64_t ns, int64_t row, int lane, const int64_t* __restrict__ mptr,
                                const int32_t* __restrict__ mcol, const double* __restrict__ mval,
                                const int64_t* __restrict__ kptr, const int32_t* __restrict__ kcol,
                                const double* __restrict__ kval, const double* __restrict__ x,
                                const double* __restrict__ b, double* __restrict__ y) {
  double u[NT], v[NT];
#pragma unroll
  for (int a = 0; a < NT; ++a) u[a] = v[a] = 0.0;
  for (int64_t p = mptr[row] + lane; p < mptr[row + 1]; p += G) {
    const int64_t c = mcol[p];
    const double w = mval[p];
#pragma unroll
    for (int a = 0; a < NT; ++a) u[a] += w * x[a * ns + c];
  }
  for (int64_t p = kptr[row] + lane; p < kptr[row + 1]; p += G) {
    const int64_t c = kcol[p];
    const double w = kval[p];
#pragma unroll
    for (int a = 0; a < NT; ++a) v[a] += w * x[a * ns + c];
  }
#pragma unroll
  for (int a = 0; a < NT; ++a) {
    u[a] = group_sum<G>(u[a]);
    v[a] = group_sum<G>(v[a]);
  }
  if (lane < NT) {
    const int bb = lane;  // this lane writes time node bb (register arrays indexed with constants only)
    double vb = 0.0, s = 0.0;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
      if (a == bb) vb = v[a];
      s += top.D[bb * NT + a] * u[a];
    }
    const double acc = s + top.mt[bb] * vb;
    const int64_t o = bb * ns + row;
    if (MODE == 0) y[o] = acc;
    if (MODE == 1) y[o] = b[o] - acc;
  }
}

template <int G, int MODE, int NT>
__global__ void __launch_bounds__(256) kron_spmv_kernel(TimeOp top, int64_t ns, const int64_t* __restrict__ mptr,
                                                        const int32_t* __restrict__ mcol,
                                                        const double* __restrict__ mval,
                                                        const int64_t* __restrict__ kptr,
                                                        const int32_t* __restrict__ kcol,
                                                        const double* __restrict__ kval,
                                                        const double* __restrict__ x, const double* __restrict__ b,
                                                        double* __restrict__ y) {
  const int lane = threadIdx.x % G;
  const int64_t row = (int64_t(blockIdx.x) * blockDim.x + threadIdx.x) / G;
  if (row >= ns) return;
  kron_row<G, MODE, NT>(top, ns, row, lane, mptr, mcol, mval, kptr, kcol, kval, x, b, y);
}

// Level operator with the velocity rows in node-pair form (NodeOp on the host): blocks
// [0, nb_node) give G lanes to each Q_r node i and produce its 2 d rows (u- and v-equation) at
// every time node from
//   su[a][c] = sum_j rhoM_ij U_a[j][c],  sv[a][c] = sum_j rhoM_ij V_a[j][c],
//   tk[b][c] = sum_j (A_ij U_b[j])[c] + sum_q C^T_{(i,c),q} P_b[q]:
//   (A x)_u,b = sum_a D[b][a] su[a] - mt[b] sv[b],  (A x)_v,b = sum_a D[b][a] sv[a] + mt[b] tk[b];
// the remaining blocks give GP lanes to each pressure row and apply its MM and KK rows as the
// CSR kernel above.  Every value of x at a node is read once per node pair (D consecutive
// values per field and time node), and rhoM, A and C^T are stored once per pair.
template <int G, int MODE, int NT, int D>
__device__ inline void node_rows(const TimeOp& top, int64_t i, int lane, int64_t nv, int64_t ns,
                                 const int64_t* __restrict__ nptr, const int32_t* __restrict__ ncol,
                                 const double* __restrict__ nm, const double* __restrict__ na,
                                 const int64_t* __restrict__ cptr, const int32_t* __restrict__ ccol,
                                 const double* __restrict__ cval, const double* __restrict__ x,
                                 const double* __restrict__ b, double* __restrict__ y) {
  double su[NT][D], sv[NT][D], tk[NT][D];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < D; ++c) su[t][c] = sv[t][c] = tk[t][c] = 0.0;
  const double* xv = x;
  const double* xu = x + nv;
  // the node pairs of node i, G lanes apart, two per lane and round (their loads in flight together)
  auto pair_load = [&](int64_t p, double* A, double (*u)[D], double (*v)[D], double& m) {
    const int64_t j = int64_t(ncol[p]) * D;
    m = nm[p];
#pragma unroll
    for (int e = 0; e < D * D; ++e) A[e] = na[p * (D * D) + e];
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        u[t][c] = xu[t * ns + j + c];
        v[t][c] = xv[t * ns + j + c];
      }
  };
  auto pair_add = [&](const double* A, const double (*u)[D], const double (*v)[D], double m) {
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < D; ++c) {
        su[t][c] += m * u[t][c];
        sv[t][c] += m * v[t][c];
        double s = tk[t][c];
#pragma unroll
        for (int e = 0; e < D; ++e) s += A[c * D + e] * u[t][e];
        tk[t][c] = s;
      }
  };
  const int64_t pe = nptr[i + 1];
  int64_t p = nptr[i] + lane;
  for (; p + G < pe; p += 2 * G) {
    double A0[D * D], A1[D * D], u0[NT][D], v0[NT][D], u1[NT][D], v1[NT][D], m0, m1;
    pair_load(p, A0, u0, v0, m0);
    pair_load(p + G, A1, u1, v1, m1);
    pair_add(A0, u0, v0, m0);
    pair_add(A1, u1, v1, m1);
  }
  if (p < pe) {
    double A0[D * D], u0[NT][D], v0[NT][D], m0;
    pair_load(p, A0, u0, v0, m0);
    pair_add(A0, u0, v0, m0);
  }
  const double* xp = x + 2 * nv;
  for (int64_t p = cptr[i] + lane; p < cptr[i + 1]; p += G) {
    const int64_t q = ccol[p];
    double cv[D];
#pragma unroll
    for (int c = 0; c < D; ++c) cv[c] = cval[p * D + c];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const double pq = xp[t * ns + q];
#pragma unroll
      for (int c = 0; c < D; ++c) tk[t][c] += cv[c] * pq;
    }
  }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      su[t][c] = group_sum<G>(su[t][c]);
      sv[t][c] = group_sum<G>(sv[t][c]);
      tk[t][c] = group_sum<G>(tk[t][c]);
    }
  // every lane holds the sums; the 2 NT D outputs are spread over the lanes
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const int k = 2 * (t * D + c);
      const int64_t ou = int64_t(t) * ns + D * i + c, ov = ou + nv;
      if (lane == k % G) {
        double yu = -top.mt[t] * sv[t][c];
#pragma unroll
        for (int a = 0; a < NT; ++a) yu += top.D[t * NT + a] * su[a][c];
        if (MODE == 0) y[ou] = yu;
        if (MODE == 1) y[ou] = b[ou] - yu;
      }
      if (lane == (k + 1) % G) {
        double yv = top.mt[t] * tk[t][c];
#pragma unroll
        for (int a = 0; a < NT; ++a) yv += top.D[t * NT + a] * sv[a][c];
        if (MODE == 0) y[ov] = yv;
        if (MODE == 1) y[ov] = b[ov] - yv;
      }
    }
}

template <int G, int GP, int MODE, int NT, int D>
__global__ void __launch_bounds__(256) node_op_kernel(
    TimeOp top, int64_t nQ, int64_t nv, int64_t ns, int64_t nb_node, const int64_t* __restrict__ nptr,
    const int32_t* __restrict__ ncol, const double* __restrict__ nm, const double* __restrict__ na,
    const int64_t* __restrict__ cptr, const int32_t* __restrict__ ccol, const double* __restrict__ cval,
    const int64_t* __restrict__ mptr, const int32_t* __restrict__ mcol, const double* __restrict__ mval,
    const int64_t* __restrict__ kptr, const int32_t* __restrict__ kcol, const double* __restrict__ kval,
    const double* __restrict__ x, const double* __restrict__ b, double* __restrict__ y, int64_t xc) {
  if (int64_t(blockIdx.x) < nb_node) {
    const int64_t blk = xcd_chunk(blockIdx.x, nb_node, xc);
    const int64_t i = (blk * blockDim.x + threadIdx.x) / G;
    if (i >= nQ) return;
    node_rows<G, MODE, NT, D>(top, i, int(threadIdx.x % G), nv, ns, nptr, ncol, nm, na, cptr, ccol, cval, x, b, y);
    return;
  }
  const int64_t row = 2 * nv + ((int64_t(blockIdx.x) - nb_node) * blockDim.x + threadIdx.x) / GP;
  if (row >= ns) return;
  kron_row<GP, MODE, NT>(top, ns, row, int(threadIdx.x % GP), mptr, mcol, mval, kptr, kcol, kval, x, b, y);
}

template <int G, int MODE>
static void launch_kron(hipStream_t st, const TimeOp& top, int64_t ns, const int64_t* mptr, const int32_t* mcol,
                        const double* mval, const int64_t* kptr, const int32_t* kcol, const double* kval,
                        const double* x, const double* b, double* y) {
  const int bs = 256;
  const int64_t grid = (ns + bs / G - 1) / (bs / G);
  switch (top.nt) {
    case 1:
      hipLaunchKernelGGL((kron_spmv_kernel<G, MODE, 1>), dim3(grid), dim3(bs), 0, st, top, ns, mptr, mcol, mval, kptr,
                         kcol, kval, x, b, y);
      break;
    case 2:
      hipLaunchKernelGGL((kron_spmv_kernel<G, MODE, 2>), dim3(grid), dim3(bs), 0, st, top, ns, mptr, mcol, mval, kptr,
                         kcol, kval, x, b, y);
      break;
    case 3:
      hipLaunchKernelGGL((kron_spmv_kernel<G, MODE, 3>), dim3(grid), dim3(bs), 0, st, top, ns, mptr, mcol, mval, kptr,
                         kcol, kval, x, b, y);
      break;
    default:
      hipLaunchKernelGGL((kron_spmv_kernel<G, MODE, 4>), dim3(grid), dim3(bs), 0, st, top, ns, mptr, mcol, mval, kptr,
                         kcol, kval, x, b, y);
      break;
  }
}

// ---------------------------------------------------------------- patch extraction
// One block per patch of the batch: W (row-major n x n) receives A_P^T, i.e.
// W[mu * n + nu] = A[dof(nu)][dof(mu)].  W must be zero on entry.
__global__ void __launch_bounds__(256) patch_extract_t_kernel(
    int64_t p0, const int64_t* __restrict__ poff, const int32_t* __restrict__ pdof, const int64_t* __restrict__ ptr,
    const int32_t* __restrict__ col, const double* __restrict__ val, const int64_t* __restrict__ woff,
    double* __restrict__ W) {
  extern __shared__ int32_t sdof[];
  const int64_t p = p0 + blockIdx.x;
  const int64_t o = poff[p];
  const int n = int(poff[p + 1] - o);
  for (int i = threadIdx.x; i < n; i += blockDim.x) sdof[i] = pdof[o + i];
  __syncthreads();
  double* Wp = W + woff[blockIdx.x];
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE, nw = blockDim.x / WAVE;
  for (int nu = wave; nu < n; nu += nw) {
    const int64_t g = sdof[nu];
    for (int64_t q = ptr[g] + lane; q < ptr[g + 1]; q += WAVE) {
      const int32_t c = col[q];
      int lo = 0, hi = n - 1;
      while (lo < hi) {  // first index with sdof >= c
        int mid = (lo + hi) >> 1;
        if (sdof[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (sdof[lo] == c) Wp[int64_t(lo) * n + nu] = val[q];
    }
  }
}

// Dense spatial blocks of a patch (time-block solves): S_P = the first n_P / nt dofs
// of the patch (time node 0, whose global numbers are the spatial numbers);
// wmm[mu * ns + nu] = MM[S(nu)][S(mu)], wkk likewise (transposed).  Zero on entry.
__global__ void __launch_bounds__(256) patch_extract_spatial_t_kernel(
    int64_t p0, int nt, int max_ns, const int64_t* __restrict__ poff, const int32_t* __restrict__ pdof,
    const int64_t* __restrict__ mptr, const int32_t* __restrict__ mcol, const double* __restrict__ mval,
    const int64_t* __restrict__ kptr, const int32_t* __restrict__ kcol, const double* __restrict__ kval,
    double* __restrict__ wmm, double* __restrict__ wkk) {
  extern __shared__ int32_t sdof[];
  const int64_t p = p0 + blockIdx.x;
  const int64_t o = poff[p];
  const int ns = int(poff[p + 1] - o) / nt;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) sdof[i] = pdof[o + i];
  __syncthreads();
  double* Wm = wmm + int64_t(blockIdx.x) * max_ns * max_ns;
  double* Wk = wkk + int64_t(blockIdx.x) * max_ns * max_ns;
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE, nw = blockDim.x / WAVE;
  for (int t = wave; t < 2 * ns; t += nw) {
    const int nu = t % ns;
    const bool is_k = t >= ns;
    const int64_t g = sdof[nu];
    const int64_t* ptr = is_k ? kptr : mptr;
    const int32_t* col = is_k ? kcol : mcol;
    const double* val = is_k ? kval : mval;
    double* Wd = is_k ? Wk : Wm;
    for (int64_t q = ptr[g] + lane; q < ptr[g + 1]; q += WAVE) {
      const int32_t c = col[q];
      int lo = 0, hi = ns - 1;
      while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (sdof[mid] < c)
          lo = mid + 1;
        else
          hi = mid;
      }
      if (sdof[lo] == c) Wd[int64_t(lo) * ns + nu] = val[q];
    }
  }
}

// Block matrix (transposed) of descriptor m = (patch i = m / nblk, eigenvalue a = m % nblk):
// real lambda: lambda MM^T + KK^T; complex lambda = al + i be: the transpose of the real form
// [[al MM + KK, -be MM], [be MM, al MM + KK]].
__global__ void form_time_blocks_kernel(TimeBlockConsts tb, int max_ns, const int32_t* __restrict__ ns_of,
                                        const double* __restrict__ wmm, const double* __restrict__ wkk,
                                        const GjDesc* __restrict__ desc, double* __restrict__ W) {
  const int64_t m = blockIdx.x;
  const int64_t i = m / tb.nblk;
  const int a = int(m % tb.nblk);
  const int ns = ns_of[i];
  const double* Mt = wmm + i * max_ns * max_ns;
  const double* Kt = wkk + i * max_ns * max_ns;
  double* Wd = W + desc[m].woff;
  const double al = tb.lam[2 * a], be = tb.lam[2 * a + 1];
  if (!tb.cplx[a]) {
    for (int64_t q = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; q < int64_t(ns) * ns;
         q += int64_t(gridDim.y) * blockDim.x)
      Wd[q] = al * Mt[q] + Kt[q];
  } else {
    const int n2 = 2 * ns;
    for (int64_t q = int64_t(blockIdx.y) * blockDim.x + threadIdx.x; q < int64_t(ns) * ns;
         q += int64_t(gridDim.y) * blockDim.x) {
      const int mu = int(q / ns), nu = int(q % ns);
      const double d = al * Mt[q] + Kt[q], b = be * Mt[q];
      Wd[int64_t(mu) * n2 + nu] = d;
      Wd[int64_t(mu) * n2 + ns + nu] = b;
      Wd[int64_t(ns + mu) * n2 + nu] = -b;
      Wd[int64_t(ns + mu) * n2 + ns + nu] = d;
    }
  }
}

// Reduced time-block solves: the u-equation rows of every block lam MM_P + KK_P are
// eliminated.  Patch-local order per time node: V [0, nU), U [nU, 2nU), P [2nU, ns) for the
// columns and the u-, v-, p-equation rows alike; nU = d nn (nn patch nodes, components
// interleaved), nP = ns - 2 nU.  Index x of the reduced system (rows: v-, p-equation;
// columns: U, P) is patch index nU + x.  With B = lam MM_P + KK_P, B_uV = -rho M,
// B_uU = lam rho M and the other u-row blocks zero, the Schur complement is
//   S(lam)[x][y] = lam^2 A2 + lam A1 + A0,  A2 = [y < nU] MM[nU+x][y],
//   A1 = MM[nU+x][nU+y] + [y < nU] KK[nU+x][y],  A0 = KK[nU+x][nU+y].
// Work items m = (patch i, slot s) of the batch on blockIdx.x, nslot = nblk + 2:
//   s = 0: the transposed node mass block rho M (component 0 of the u-rows and U columns);
//   s = 1 + a: the transposed S(lam_a); if complex, in the real form [[Re, -Im], [Im, Re]]
//            (cplanes == 0) or as the real plane followed by the imaginary plane (cplanes != 0);
//   s = 1 + nblk: KK[2nU + x][y] (x < nP, y < nU) written to out column-major with leading
//            dimension inv_ld(nP) (zero padding rows), right after the stored mass inverse.
// desc holds nblk + 1 Gauss-Jordan descriptors per patch (mass, then the blocks); wmm, wkk
// are the transposed dense spatial blocks of the patch (stride max_ns^2).
template <typename T>
__global__ void form_reduced_blocks_kernel(TimeBlockConsts tb, int d, int cplanes, int max_ns,
                                           const int32_t* __restrict__ ns_of,
                                           const int32_t* __restrict__ nu_of, const double* __restrict__ wmm,
                                           const double* __restrict__ wkk, const GjDesc* __restrict__ desc,
                                           double* __restrict__ W, T* __restrict__ out) {
  const int nslot = tb.nblk + 2;
  const int64_t m = blockIdx.x;
  const int64_t i = m / nslot;
  const int s = int(m % nslot);
  const int ns = ns_of[i], nU = nu_of[i], nP = ns - 2 * nU, nn = nU / d, nr = nU + nP;
  const double* Mt = wmm + i * max_ns * max_ns;  // Mt[c * ns + r] = MM[r][c]
  const double* Kt = wkk + i * max_ns * max_ns;
  const GjDesc* dp = desc + i * (tb.nblk + 1);
  const int64_t t0 = int64_t(blockIdx.y) * blockDim.x + threadIdx.x, step = int64_t(gridDim.y) * blockDim.x;
  if (s == 0) {
    double* Wd = W + dp[0].woff;
    for (int64_t q = t0; q < int64_t(nn) * nn; q += step) {
      const int b = int(q / nn), a = int(q % nn);
      Wd[q] = Mt[int64_t(nU + b * d) * ns + a * d];
    }
  } else if (s <= tb.nblk) {
    const int a = s - 1;
    const double al = tb.lam[2 * a], be = tb.lam[2 * a + 1];
    double* Wd = W + dp[s].woff;
    for (int64_t q = t0; q < int64_t(nr) * nr; q += step) {
      const int y = int(q / nr), x = int(q % nr);
      const double A2 = y < nU ? Mt[int64_t(y) * ns + nU + x] : 0.0;
      const double A1 = Mt[int64_t(nU + y) * ns + nU + x] + (y < nU ? Kt[int64_t(y) * ns + nU + x] : 0.0);
      const double A0 = Kt[int64_t(nU + y) * ns + nU + x];
      if (!tb.cplx[a]) {
        Wd[q] = (al * al) * A2 + al * A1 + A0;
      } else if (cplanes) {
        Wd[q] = (al * al - be * be) * A2 + al * A1 + A0;
        Wd[int64_t(nr) * nr + q] = (2.0 * al * be) * A2 + be * A1;
      } else {
        const int n2 = 2 * nr;
        const double sr = (al * al - be * be) * A2 + al * A1 + A0, si = (2.0 * al * be) * A2 + be * A1;
        Wd[int64_t(y) * n2 + x] = sr;
        Wd[int64_t(y) * n2 + nr + x] = si;
        Wd[int64_t(nr + y) * n2 + x] = -si;
        Wd[int64_t(nr + y) * n2 + nr + x] = sr;
      }
    }
  } else {
    const int ldp = inv_ld(nP);
    T* o = out + dp[0].ooff + int64_t(nn) * inv_ld(nn);
    for (int64_t q = t0; q < int64_t(nU) * ldp; q += step) {
      const int y = int(q / ldp), x = int(q % ldp);
      o[q] = x < nP ? T(Kt[int64_t(y) * ns + 2 * nU + x]) : T(0);
    }
  }
}

__global__ void fill_zero_kernel(double* __restrict__ a, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    a[i] = 0.0;
}

// ---------------------------------------------------------------- Gauss-Jordan
// In-place blocked Gauss-Jordan inversion of the row-major n x n matrix M of
// this block, with the rows first scaled by powers of two (row equilibration,
// exact in floating point) and partial pivoting on the scaled matrix.  Panels
// of NB columns live in LDS; the rest of the matrix is updated by a rank-NB
// Schur-complement step:  M[:, rest] = [i notin K] M[:, rest] + Pnl[:, K] W,
// with W = the (swapped) pivot rows of M[:, rest].  The result
// inv(M) = inv(S M) S, columns un-permuted, is written row-major to out.
template <typename T, int NB>
__global__ void __launch_bounds__(256) gj_invert_kernel(const GjDesc* __restrict__ desc, double* __restrict__ W,
                                                        T* __restrict__ out, int32_t* __restrict__ status) {
  extern __shared__ double lds[];
  const GjDesc D = desc[blockIdx.x];
  const int n = D.n;
  double* M = W + D.woff;
  double* Pnl = lds;                                   // n * NB
  double* scl = lds + size_t(n) * NB;                  // n
  double* red_v = scl + n;                             // 4 waves
  int* red_i = reinterpret_cast<int*>(red_v + 8);      // 4 waves
  int* perm = red_i + 8;                               // n
  int* src = perm + n;                                 // n
  __shared__ int s_flag;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int wave = tid / WAVE, lane = tid % WAVE, nw = bs / WAVE;
  if (tid == 0) s_flag = 0;
  // row equilibration by powers of two
  for (int i = wave; i < n; i += nw) {
    double m = 0.0;
    for (int j = lane; j < n; j += WAVE) m = fmax(m, fabs(M[int64_t(i) * n + j]));
    for (int off = WAVE / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    const double s = (m > 0.0 && isfinite(m)) ? ldexp(1.0, -ilogb(m)) : 1.0;
    for (int j = lane; j < n; j += WAVE) M[int64_t(i) * n + j] *= s;
    if (lane == 0) scl[i] = s;
  }
  __syncthreads();
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nb = min(NB, n - k0);
    for (int t = tid; t < n * nb; t += bs) {
      const int i = t / nb, c = t % nb;
      Pnl[i * NB + c] = M[int64_t(i) * n + k0 + c];
    }
    __syncthreads();
    for (int c = 0; c < nb; ++c) {
      const int k = k0 + c;
      // pivot search over rows k..n-1 of panel column c (ties: lowest row)
      double bv = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += bs) {
        const double v = fabs(Pnl[i * NB + c]);
        if (v > bv) {
          bv = v;
          bi = i;
        }
      }
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        red_v[wave] = bv;
        red_i[wave] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double v = red_v[0];
        int ii = red_i[0];
        for (int w = 1; w < nw; ++w)
          if (red_v[w] > v || (red_v[w] == v && red_i[w] < ii)) {
            v = red_v[w];
            ii = red_i[w];
          }
        if (!(v > 0.0) || !isfinite(v) || ii >= n) {
          s_flag = 1;
          ii = k;
        }
        perm[k] = ii;
        if (ii != k)
          for (int cc = 0; cc < nb; ++cc) {
            const double tmp = Pnl[k * NB + cc];
            Pnl[k * NB + cc] = Pnl[ii * NB + cc];
            Pnl[ii * NB + cc] = tmp;
          }
        double piv = Pnl[k * NB + c];
        if (piv == 0.0 || !isfinite(piv)) piv = 1.0;
        const double rp = 1.0 / piv;
        Pnl[k * NB + c] = 1.0;
        for (int cc = 0; cc < nb; ++cc) Pnl[k * NB + cc] *= rp;
      }
      __syncthreads();
      for (int i = tid; i < n; i += bs) {
        if (i == k) continue;
        const double f = Pnl[i * NB + c];
        Pnl[i * NB + c] = 0.0;
        for (int cc = 0; cc < nb; ++cc) Pnl[i * NB + cc] -= f * Pnl[k * NB + cc];
      }
      __syncthreads();
    }
    // rest of the matrix: row swaps then the rank-nb update, column-owned by threads
    for (int j = tid; j < n; j += bs) {
      if (j >= k0 && j < k0 + nb) continue;
      double w[NB];
      for (int c = 0; c < nb; ++c) {
        const int k = k0 + c, q = perm[k];
        if (q != k) {
          const double a = M[int64_t(k) * n + j];
          M[int64_t(k) * n + j] = M[int64_t(q) * n + j];
          M[int64_t(q) * n + j] = a;
        }
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) w[c] = c < nb ? M[int64_t(k0 + c) * n + j] : 0.0;
      for (int i = 0; i < n; ++i) {
        double acc = (i >= k0 && i < k0 + nb) ? 0.0 : M[int64_t(i) * n + j];
#pragma unroll
        for (int c = 0; c < NB; ++c) acc += Pnl[i * NB + c] * w[c];
        M[int64_t(i) * n + j] = acc;
      }
    }
    __syncthreads();
    for (int t = tid; t < n * nb; t += bs) {
      const int i = t / nb, c = t % nb;
      M[int64_t(i) * n + k0 + c] = Pnl[i * NB + c];
    }
    __syncthreads();
  }
  // column un-permutation: inv(SM) = M * Pi, source column of each output column
  if (tid == 0) {
    for (int j = 0; j < n; ++j) src[j] = j;
    for (int k = n - 1; k >= 0; --k) {
      const int q = perm[k];
      const int t = src[k];
      src[k] = src[q];
      src[q] = t;
    }
    if (s_flag) status[D.patch] = 1;
  }
  __syncthreads();
  T* o = out + D.ooff;
  for (int i = wave; i < D.keep; i += nw)
    for (int q = lane; q < D.ld_out; q += WAVE) {
      int j = -1;
      if (D.split == 0) {
        j = q < n ? q : -1;
      } else if (q < D.split) {
        j = q;
      } else if (q >= D.ldh && q - D.ldh < n - D.split) {
        j = D.split + (q - D.ldh);
      }
      o[int64_t(i) * D.ld_out + q] = j >= 0 ? T(M[int64_t(i) * n + src[j]] * scl[j]) : T(0);
    }
}

// Gauss-Jordan inversion of a matrix held entirely in LDS, one workgroup per descriptor:
// the same steps and conventions as gj_invert_kernel (power-of-two row equilibration,
// partial pivoting on the scaled matrix with ties to the lowest row, output rows i < keep of
// the inverse with the columns un-permuted and re-scaled), without panels.  CPLX: the input
// at woff holds the real plane (n x n, row-major) followed by the imaginary plane, the pivot
// size is |re| + |im|, and output row i is written as Re of column j at position j and Im at
// ldh + j (all other positions of the row are zero).
template <typename T, bool CPLX>
__global__ void __launch_bounds__(256) gj_lds_kernel(const GjDesc* __restrict__ desc, const double* __restrict__ W,
                                                     T* __restrict__ out, int32_t* __restrict__ status) {
  extern __shared__ double lds[];
  const GjDesc D = desc[blockIdx.x];
  const int n = D.n, nn = n * n;
  double* Ar = lds;                              // n x n
  double* Ai = CPLX ? lds + nn : nullptr;        // n x n
  double* fr = lds + (CPLX ? 2 : 1) * nn;        // column k before the update
  double* fi = CPLX ? fr + n : nullptr;
  double* scl = fr + (CPLX ? 2 : 1) * n;
  int* perm = reinterpret_cast<int*>(scl + n);
  int* src = perm + n;
  __shared__ int s_piv, s_flag;
  const int tid = threadIdx.x, bs = blockDim.x;
  const int wave = tid / WAVE, lane = tid % WAVE, nw = bs / WAVE;
  const double* M = W + D.woff;
  for (int t = tid; t < nn; t += bs) {
    Ar[t] = M[t];
    if constexpr (CPLX) Ai[t] = M[nn + t];
  }
  if (tid == 0) s_flag = 0;
  __syncthreads();
  for (int i = wave; i < n; i += nw) {
    double m = 0.0;
    for (int j = lane; j < n; j += WAVE) {
      m = fmax(m, fabs(Ar[i * n + j]));
      if constexpr (CPLX) m = fmax(m, fabs(Ai[i * n + j]));
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    const double sc = (m > 0.0 && isfinite(m)) ? ldexp(1.0, -ilogb(m)) : 1.0;
    for (int j = lane; j < n; j += WAVE) {
      Ar[i * n + j] *= sc;
      if constexpr (CPLX) Ai[i * n + j] *= sc;
    }
    if (lane == 0) scl[i] = sc;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (wave == 0) {  // pivot: largest scaled entry of column k in rows k..n-1
      double bv = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += WAVE) {
        double v = fabs(Ar[i * n + k]);
        if constexpr (CPLX) v += fabs(Ai[i * n + k]);
        if (v > bv) {
          bv = v;
          bi = i;
        }
      }
      for (int off = WAVE / 2; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off);
        const int oi = __shfl_xor(bi, off);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        if (!(bv > 0.0) || !isfinite(bv) || bi >= n) {
          s_flag = 1;
          bi = k;
        }
        s_piv = bi;
        perm[k] = bi;
      }
    }
    __syncthreads();
    const int pr = s_piv;
    if (pr != k)
      for (int j = tid; j < n; j += bs) {
        const double t = Ar[k * n + j];
        Ar[k * n + j] = Ar[pr * n + j];
        Ar[pr * n + j] = t;
        if constexpr (CPLX) {
          const double u = Ai[k * n + j];
          Ai[k * n + j] = Ai[pr * n + j];
          Ai[pr * n + j] = u;
        }
      }
    __syncthreads();
    // reciprocal of the pivot (every thread), then the pivot row scaled and column k saved
    double pr_r = Ar[k * n + k], pr_i = CPLX ? Ai[k * n + k] : 0.0;
    if (!(fabs(pr_r) + fabs(pr_i) > 0.0) || !isfinite(pr_r) || !isfinite(pr_i)) {
      pr_r = 1.0;
      pr_i = 0.0;
    }
    const double den = pr_r * pr_r + pr_i * pr_i;
    const double rr = CPLX ? pr_r / den : 1.0 / pr_r, ri = CPLX ? -pr_i / den : 0.0;
    __syncthreads();
    for (int j = tid; j < n; j += bs) {
      const double a = j == k ? 1.0 : Ar[k * n + j];
      const double b = CPLX ? (j == k ? 0.0 : Ai[k * n + j]) : 0.0;
      Ar[k * n + j] = a * rr - b * ri;
      if constexpr (CPLX) Ai[k * n + j] = a * ri + b * rr;
    }
    for (int i = tid; i < n; i += bs) {
      fr[i] = i == k ? 0.0 : Ar[i * n + k];
      if constexpr (CPLX) fi[i] = i == k ? 0.0 : Ai[i * n + k];
      if (i != k) {
        Ar[i * n + k] = 0.0;
        if constexpr (CPLX) Ai[i * n + k] = 0.0;
      }
    }
    __syncthreads();
    for (int t = tid; t < nn; t += bs) {
      const int i = t / n, j = t - i * n;
      if (i == k) continue;
      if constexpr (CPLX) {
        const double a = fr[i], b = fi[i], c = Ar[k * n + j], e = Ai[k * n + j];
        Ar[t] -= a * c - b * e;
        Ai[t] -= a * e + b * c;
      } else {
        Ar[t] -= fr[i] * Ar[k * n + j];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    for (int j = 0; j < n; ++j) src[j] = j;
    for (int k = n - 1; k >= 0; --k) {
      const int q = perm[k];
      const int t = src[k];
      src[k] = src[q];
      src[q] = t;
    }
    if (s_flag) status[D.patch] = 1;
  }
  __syncthreads();
  T* o = out + D.ooff;
  for (int i = wave; i < D.keep; i += nw)
    for (int q = lane; q < D.ld_out; q += WAVE) {
      double v = 0.0;
      if constexpr (CPLX) {
        if (q < n)
          v = Ar[i * n + src[q]] * scl[q];
        else if (q >= D.ldh && q - D.ldh < n)
          v = Ai[i * n + src[q - D.ldh]] * scl[q - D.ldh];
      } else {
        if (q < n) v = Ar[i * n + src[q]] * scl[q];
      }
      o[int64_t(i) * D.ld_out + q] = T(v);
    }
}

// ---------------------------------------------------------------- patch apply
// y_P = A_P^{-1} R_P r for every patch.  The inverse of patch p is stored
// column by column, element (i, j) of A_P^{-1} at inv[ioff[p] + j * ld + i]
// with ld = inv_ld(n) (zero padding rows), so one block streams the n*ld
// values of its patch exactly once, front to back.  Each thread owns RPT
// consecutive rows and reads them with one 16-byte load per column.
template <typename T, int RPT>
__global__ void __launch_bounds__(512) patch_apply_kernel(int64_t npatch, const int64_t* __restrict__ poff,
                                                          const int32_t* __restrict__ pdof,
                                                          const int32_t* __restrict__ tpos,
                                                          const int64_t* __restrict__ ioff,
                                                          const T* __restrict__ inv, const double* __restrict__ r,
                                                          double* __restrict__ y) {
  typedef T V __attribute__((ext_vector_type(RPT)));
  extern __shared__ char smem[];
  T* rl = reinterpret_cast<T*>(smem);
  const int64_t p = blockIdx.x;
  const int64_t o = poff[p];
  const int n = int(poff[p + 1] - o);
  const int ld = inv_ld(n);
  for (int i = threadIdx.x; i < n; i += blockDim.x) rl[i] = T(r[pdof[o + i]]);
  __syncthreads();
  const int i0 = RPT * int(threadIdx.x);
  if (i0 >= n) return;
  const V* X = reinterpret_cast<const V*>(inv + ioff[p] + i0);
  const int ldv = ld / RPT;
  V a = V(0), b = V(0);
  int j = 0;
  for (; j + 7 < n; j += 8) {
    const V v0 = __builtin_nontemporal_load(X + int64_t(j) * ldv);
    const V v1 = __builtin_nontemporal_load(X + int64_t(j + 1) * ldv);
    const V v2 = __builtin_nontemporal_load(X + int64_t(j + 2) * ldv);
    const V v3 = __builtin_nontemporal_load(X + int64_t(j + 3) * ldv);
    const V v4 = __builtin_nontemporal_load(X + int64_t(j + 4) * ldv);
    const V v5 = __builtin_nontemporal_load(X + int64_t(j + 5) * ldv);
    const V v6 = __builtin_nontemporal_load(X + int64_t(j + 6) * ldv);
    const V v7 = __builtin_nontemporal_load(X + int64_t(j + 7) * ldv);
    a += v0 * rl[j];
    b += v1 * rl[j + 1];
    a += v2 * rl[j + 2];
    b += v3 * rl[j + 3];
    a += v4 * rl[j + 4];
    b += v5 * rl[j + 5];
    a += v6 * rl[j + 6];
    b += v7 * rl[j + 7];
  }
  for (; j < n; ++j) a += __builtin_nontemporal_load(X + int64_t(j) * ldv) * rl[j];
  a += b;
#pragma unroll
  for (int q = 0; q < RPT; ++q)
    if (i0 + q < n) y[tpos[o + i0 + q]] = double(a[q]);
}

// Time-block patch solve: y_P = (Q x I) blockdiag(X_a) (Q^{-1} (M^t)^{-1} x I) r_P with the
// spatial block inverses X_a stored per patch one after another: a real block as ns
// columns of stride inv_ld(ns); a complex block as ns columns of stride 2 inv_ld(ns)
// holding Re X_a in rows [0, ns) and Im X_a in rows [inv_ld(ns), inv_ld(ns) + ns).
// Each thread owns R consecutive rows (one 16-byte load per column); W waves split the
// columns of every block into W contiguous ranges and their partial images are summed
// in LDS; NTL selects streaming (non-temporal) loads for the stored inverses.
template <typename T>
struct NV16;
template <>
struct NV16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int R = 2;
};
template <>
struct NV16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int R = 4;
};

template <bool NTL, typename V>
__device__ inline V ld16(const V* p) {
  if constexpr (NTL)
    return __builtin_nontemporal_load(p);
  else
    return *p;
}

template <typename T, int W, bool NTL>
__global__ void __launch_bounds__(512) patch_apply_tb_kernel(TimeBlockConsts tb, const int64_t* __restrict__ poff,
                                                             const int32_t* __restrict__ pdof,
                                                             const int32_t* __restrict__ tpos,
                                                             const int64_t* __restrict__ ioff,
                                                             const T* __restrict__ inv, const double* __restrict__ r,
                                                             double* __restrict__ y) {
  using V = typename NV16<T>::type;
  constexpr int R = NV16<T>::R;
  extern __shared__ double sm[];
  const int64_t p = blockIdx.x;
  const int64_t o = poff[p];
  const int n = int(poff[p + 1] - o);
  const int nt = tb.nt, nblk = tb.nblk;
  const int ns = n / nt, ldh = inv_ld(ns);
  const int per_w = blockDim.x / W;  // threads per column range
  const int w = threadIdx.x / per_w, tl = threadIdx.x % per_w;
  double* rl = sm;                          // n
  T* sv = reinterpret_cast<T*>(sm + n);     // nblk * 2 * ldh (re, im) as T
  double* tv = sm + n + 2 * nblk * ldh;     // W partial images, nblk * 2 * ldh each
  for (int i = threadIdx.x; i < n; i += blockDim.x) rl[i] = r[pdof[o + i]];
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += blockDim.x)
    for (int a = 0; a < nblk; ++a) {
      double sr = 0.0, si = 0.0;
      for (int b = 0; b < nt; ++b) {
        const double x = rl[b * ns + i];
        sr += tb.tin[2 * (a * nt + b)] * x;
        si += tb.tin[2 * (a * nt + b) + 1] * x;
      }
      sv[(2 * a) * ldh + i] = T(sr);
      sv[(2 * a + 1) * ldh + i] = T(si);
    }
  __syncthreads();
  const int i0 = R * tl;
  const int jc = (ns + W - 1) / W, j0 = w * jc, j1 = min(ns, j0 + jc);
  double* tw = tv + int64_t(w) * nblk * 2 * ldh;
  int64_t off = ioff[p];
  for (int a = 0; a < nblk; ++a) {
    const T* sr = sv + (2 * a) * ldh;
    const T* si = sv + (2 * a + 1) * ldh;
    if (!tb.cplx[a]) {
      if (i0 < ns) {
        const V* X = reinterpret_cast<const V*>(inv + off + i0);
        const int ldv = ldh / R;
        V acc = V(0), acc2 = V(0);
        int j = j0;
        for (; j + 3 < j1; j += 4) {
          const V v0 = ld16<NTL>(X + int64_t(j) * ldv), v1 = ld16<NTL>(X + int64_t(j + 1) * ldv);
          const V v2 = ld16<NTL>(X + int64_t(j + 2) * ldv), v3 = ld16<NTL>(X + int64_t(j + 3) * ldv);
          acc += v0 * sr[j];
          acc2 += v1 * sr[j + 1];
          acc += v2 * sr[j + 2];
          acc2 += v3 * sr[j + 3];
        }
        for (; j < j1; ++j) acc += ld16<NTL>(X + int64_t(j) * ldv) * sr[j];
        acc += acc2;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          tw[(2 * a) * ldh + i0 + q] = double(acc[q]);
          tw[(2 * a + 1) * ldh + i0 + q] = 0.0;
        }
      }
      off += int64_t(ns) * ldh;
    } else {
      if (i0 < ns) {
        const V* Xr = reinterpret_cast<const V*>(inv + off + i0);
        const V* Xi = reinterpret_cast<const V*>(inv + off + ldh + i0);
        const int ldv = 2 * ldh / R;
        V tr = V(0), ti = V(0), tr2 = V(0), ti2 = V(0);
        int j = j0;
        for (; j + 1 < j1; j += 2) {
          const V a0 = ld16<NTL>(Xr + int64_t(j) * ldv), b0 = ld16<NTL>(Xi + int64_t(j) * ldv);
          const V a1 = ld16<NTL>(Xr + int64_t(j + 1) * ldv), b1 = ld16<NTL>(Xi + int64_t(j + 1) * ldv);
          tr += a0 * sr[j] - b0 * si[j];
          ti += b0 * sr[j] + a0 * si[j];
          tr2 += a1 * sr[j + 1] - b1 * si[j + 1];
          ti2 += b1 * sr[j + 1] + a1 * si[j + 1];
        }
        for (; j < j1; ++j) {
          const V a0 = ld16<NTL>(Xr + int64_t(j) * ldv), b0 = ld16<NTL>(Xi + int64_t(j) * ldv);
          tr += a0 * sr[j] - b0 * si[j];
          ti += b0 * sr[j] + a0 * si[j];
        }
        tr += tr2;
        ti += ti2;
#pragma unroll
        for (int q = 0; q < R; ++q) {
          tw[(2 * a) * ldh + i0 + q] = double(tr[q]);
          tw[(2 * a + 1) * ldh + i0 + q] = double(ti[q]);
        }
      }
      off += int64_t(ns) * 2 * ldh;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < ns; i += blockDim.x)
    for (int b = 0; b < nt; ++b) {
      double acc = 0.0;
      for (int a = 0; a < nblk; ++a) {
        const double qr = tb.qout[2 * (b * nblk + a)], qi = tb.qout[2 * (b * nblk + a) + 1];
        double t_r = 0.0, t_i = 0.0;
        for (int ww = 0; ww < W; ++ww) {
          t_r += tv[int64_t(ww) * nblk * 2 * ldh + (2 * a) * ldh + i];
          t_i += tv[int64_t(ww) * nblk * 2 * ldh + (2 * a + 1) * ldh + i];
        }
        acc += tb.cplx[a] ? 2.0 * (qr * t_r - qi * t_i) : qr * t_r;
      }
      y[tpos[o + b * ns + i]] = acc;
    }
}

// Reduced time-block patch solve.  Per kept eigenvalue lam of (M^t)^{-1} D^t and the
// transformed right-hand side (r_u, r_v, r_p) of the patch:
//   w = (rho M)^{-1} r_u,  [U; P] = S(lam)^{-1} [r_v + lam r_u; r_p + G r_u],  V = lam U - w,
// with G = KK_pV (rho M)^{-1}: the exact solution of (lam MM_P + KK_P) [V; U; P] = [r_u; r_v; r_p]
// (S as in form_reduced_blocks_kernel).  Stored per patch at ioff[p]: (rho M)^{-1} (nn columns,
// stride inv_ld(nn), applied per velocity component), G (nU columns, stride inv_ld(nP)), then
// one S^{-1} per kept eigenvalue (nr = nU + nP columns: stride inv_ld(nr) if real, 2 inv_ld(nr)
// with Re in rows [0, nr) and Im in rows [inv_ld(nr), inv_ld(nr) + nr) if complex).  All sums
// are in FP64 whatever the storage type T.  At most RED_MAXB kept eigenvalues (k <= 3).
//
// One block per patch.  The stored values are read with buffer loads: the patch's region is
// the buffer (range-checked), the lane's rows a 32-bit vector offset and the column a scalar
// offset, so that no 64-bit address is held per load (the start of a lane's column range is
// part of its vector offset: the scalar offset has to be the same on all lanes of a wave, and
// a wave can hold two ranges).  The S^{-1} stream runs in batches of 8 columns per lane (16
// loads for a complex block; the compiler pipelines two batches of a real block).
// Thread layout of the S^{-1} product: W column ranges of blockDim / W threads, R consecutive
// rows per thread (one 16-byte load per column).
constexpr int RED_MAXB = 2;
// LDS planes of the kept eigenvalues in the reduced solve: Re of block a at plane red_pl(tb, a),
// its Im in the next plane if the eigenvalue is complex (a real one has none); red_npl in all.
__host__ __device__ inline int red_pl(const TimeBlockConsts& tb, int a) {
  int p = 0;
  for (int b = 0; b < a; ++b) p += tb.cplx[b] ? 2 : 1;
  return p;
}
__host__ __device__ inline int red_npl(const TimeBlockConsts& tb) { return red_pl(tb, tb.nblk); }

// Balanced symmetrising factors of a Schur complement S(lam) = [[lam^2 rho M + A, C^T],
// [-lam C, lam c0 M_p + B]]: with mu2 = sqrt(lam) (principal root) and mu1 = -1/mu2,
// D1 S D2 is (complex) symmetric for D1 = diag(I_nU, mu1 I_nP), D2 = diag(I_nU, mu2 I_nP)
// (mu2 C^T is the transpose of -lam mu1 C, and mu1 mu2 = -1 leaves the pressure block symmetric).
__device__ inline void sym_factors(double al, double be, double* m1r, double* m1i, double* m2r, double* m2i) {
  const double mod = sqrt(al * al + be * be);
  const double sr = sqrt(0.5 * (mod + al)), si = copysign(sqrt(0.5 * fmax(mod - al, 0.0)), be);
  const double q = sr * sr + si * si;
  *m2r = sr;
  *m2i = si;
  *m1r = -sr / q;
  *m1i = si / q;
}

// Symmetric tiled storage of the Schur inverses: X = (D1 S D2)^{-1} = D2^{-1} S^{-1} D1^{-1} is
// symmetric; its lower triangle is stored in the tiles of tile_layout.h (off-diagonal 8x8 tiles
// I-major, the diagonal blocks as triangles paired two to a tile, the last block row possibly as
// 4x16 tiles); a complex X as the Re tiles followed by the Im tiles.  One block per (batch item, kept eigenvalue); S^{-1} is read
// from the square scratch (column j of Re at soff + j * ldc, Im rows after ldr) and
// symmetrised as (X + X^T) / 2.
template <typename T>
__global__ void __launch_bounds__(256) pack_red_sym_kernel(TimeBlockConsts tb, const int32_t* __restrict__ nu_of,
                                                           const int32_t* __restrict__ nr_of,
                                                           const int64_t* __restrict__ soff,
                                                           const int64_t* __restrict__ toff,
                                                           const double* __restrict__ sq, T* __restrict__ out) {
  const int nblk = tb.nblk;
  const int64_t m = blockIdx.x;
  const int64_t i = m / nblk;
  const int a = int(m % nblk);
  const int nU = nu_of[i], nr = nr_of[i], ldr = inv_ld(nr);
  const bool cp = tb.cplx[a] != 0;
  const int ldc = cp ? 2 * ldr : ldr;
  constexpr int P = 8 / int(sizeof(T));  // tiles interleaved per unit (tile_layout.h)
  const int nh = sym_half_tiles(nr), ntf2 = sym_full_slots(nr, P);
  const int nsl = sym_slots(nr, P), Ilast = sym_nbk(nr) - 1;
  const int nd = sym_nd(nr), noff = sym_off_tiles(nr), npair = sym_pair_tiles(nr), nof2 = sym_off_slots(nr, P);
  const int ndl = sym_dlist(nr), ndp = sym_dlist_in_pair(nr), npd = npair + sym_diag_tiles(nr);
  double m1r, m1i, m2r, m2i;
  sym_factors(tb.lam[2 * a], tb.lam[2 * a + 1], &m1r, &m1i, &m2r, &m2i);
  // 1/mu2 and 1/mu1 = -mu2
  const double q2 = m2r * m2r + m2i * m2i;
  const double f2r = m2r / q2, f2i = -m2i / q2, g1r = -m2r, g1i = -m2i;
  const double* S = sq + soff[m];
  T* o = out + toff[m];
  auto X = [&](int row, int col, double* xr, double* xi) {  // S^{-1}(row, col) / (d2_row d1_col)
    double vr = S[int64_t(col) * ldc + row], vi = cp ? S[int64_t(col) * ldc + ldr + row] : 0.0;
    if (row >= nU) {
      const double tr = vr * f2r - vi * f2i, ti = vr * f2i + vi * f2r;
      vr = tr;
      vi = ti;
    }
    if (col >= nU) {
      const double tr = vr * g1r - vi * g1i, ti = vr * g1i + vi * g1r;
      vr = tr;
      vi = ti;
    }
    *xr = vr;
    *xi = vi;
  };
  for (int q = threadIdx.x; q < nsl * 64; q += blockDim.x) {
    const int t = q / (64 * P) * P + q % P, e = q % (64 * P) / P;  // slot and entry of position q
    int row = nr, col = nr;  // zero slots
    const int r = e & 7, c = e >> 3;
    int s = ndl;  // entry of the odd blocks' diagonal list held here, if below ndl
    if (t >= ntf2) {  // 4x16 tile of the last block row
      if (t - ntf2 < nh) {
        row = 8 * Ilast + (e & 3);
        col = 16 * (t - ntf2) + (e >> 2);
      }
    } else if (t < nof2) {  // off-diagonal tile (I, J), J < I
      if (t < noff) {
        int I = int((sqrt(8.0 * t + 1.0) + 1.0) * 0.5);
        while (I * (I - 1) / 2 > t) --I;
        while ((I + 1) * I / 2 <= t) ++I;
        const int J = t - I * (I - 1) / 2;
        row = 8 * I + r;
        col = 8 * J + c;
      }
    } else if (t < nof2 + npair) {  // pair tile: block A at r >= c, block B transposed at r < c
      const int A = 2 * (t - nof2), B = A + 1;
      if (r >= c) {
        row = 8 * A + r;
        col = 8 * A + c;
      } else if (B < nd) {
        row = 8 * B + c;
        col = 8 * B + r;
      } else {
        s = c * (c - 1) / 2 + r;
      }
    } else if (t < nof2 + npd) {  // diagonal tile
      s = ndp + 64 * (t - nof2 - npair) + e;
    }
    if (s < ndl) row = col = 16 * (s >> 3) + 8 + (s & 7);
    double vr = 0.0, vi = 0.0;
    if (row < nr && col < nr) {
      double ar, ai, br, bi;
      X(row, col, &ar, &ai);
      X(col, row, &br, &bi);
      vr = 0.5 * (ar + br);
      vi = 0.5 * (ai + bi);
    }
    o[q] = T(vr);
    if (cp) o[int64_t(nsl) * 64 + q] = T(vi);
  }
}


template <typename T, bool NTL>
__device__ inline T bld1(__amdgpu_buffer_rsrc_t rs, int voff) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0, NTL ? 2 : 0));
  else if constexpr (sizeof(T) == 4)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, voff, 0, NTL ? 2 : 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b16(rs, voff, 0, NTL ? 2 : 0));
}

template <typename V, bool NTL>
__device__ inline V bld16(__amdgpu_buffer_rsrc_t rs, int voff, int soff) {
  static_assert(sizeof(V) == 16 || sizeof(V) == 8, "16- or 8-byte loads");
  if constexpr (sizeof(V) == 16)
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b128(rs, voff, soff, NTL ? 2 : 0));
  else
    return __builtin_bit_cast(V, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, soff, NTL ? 2 : 0));
}

template <typename T>
__device__ inline __amdgpu_buffer_rsrc_t patch_rsrc(const T* p, int64_t count) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<T*>(p), 0, int(count * int64_t(sizeof(T))), 0x00020000);
}

// One step of a DPP butterfly sum of a double: ctrl 0 adds the value of lane xor 1 (quad_perm
// [1,0,3,2]), ctrl 1 that of lane xor 2 (quad_perm [2,3,0,1]), ctrl 2 the mirrored lane within
// each group of 8 (row_half_mirror).
__device__ inline double dpp_sum_step(double x, int ctrl) {
  const int2 b = __builtin_bit_cast(int2, x);
  int2 o;
  switch (ctrl) {
    case 0:
      o.x = __builtin_amdgcn_update_dpp(0, b.x, 0xB1, 0xF, 0xF, false);
      o.y = __builtin_amdgcn_update_dpp(0, b.y, 0xB1, 0xF, 0xF, false);
      break;
    case 1:
      o.x = __builtin_amdgcn_update_dpp(0, b.x, 0x4E, 0xF, 0xF, false);
      o.y = __builtin_amdgcn_update_dpp(0, b.y, 0x4E, 0xF, 0xF, false);
      break;
    default:
      o.x = __builtin_amdgcn_update_dpp(0, b.x, 0x141, 0xF, 0xF, false);
      o.y = __builtin_amdgcn_update_dpp(0, b.y, 0x141, 0xF, 0xF, false);
      break;
  }
  return x + __builtin_bit_cast(double, o);
}
// Sum over the 8 consecutive lanes of each group (lanes 8g .. 8g+7); every lane of the group
// ends with the sum.
__device__ inline double dpp_sum8(double v) { return dpp_sum_step(dpp_sum_step(dpp_sum_step(v, 0), 1), 2); }
// The same over the 4 lanes of each quad.
__device__ inline double dpp_sum4(double v) { return dpp_sum_step(dpp_sum_step(v, 0), 1); }

// *p += v in LDS as one atomic add (ds_add_f64), for lanes of a wave that share an address.
__device__ inline void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// P values of one unit of tiles (tile_layout.h) at byte offset voff: one 8-byte load per lane.
template <typename T, bool NTL>
__device__ inline void bld_unit(__amdgpu_buffer_rsrc_t rs, int voff, T* out) {
  if constexpr (sizeof(T) == 8) {
    out[0] = bld1<T, NTL>(rs, voff);
  } else if constexpr (sizeof(T) == 4) {
    typedef float F2 __attribute__((ext_vector_type(2)));
    const F2 v = __builtin_bit_cast(F2, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0, NTL ? 2 : 0));
    out[0] = v.x;
    out[1] = v.y;
  } else {
    typedef __bf16 B4 __attribute__((ext_vector_type(4)));
    const B4 v = __builtin_bit_cast(B4, __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0, NTL ? 2 : 0));
    out[0] = v.x;
    out[1] = v.y;
    out[2] = v.z;
    out[3] = v.w;
  }
}

// y += X zt for one plane of symmetric tiles (layout and the interleaving of P tiles per unit in
// tile_layout.h), by wave w of nw: it takes the units w, w + nw, ... of each of the three
// sections.  Lane (r, c) = (lane % 8, lane / 8) of the off-diagonal tile (I, J) adds
// X[8I+r][8J+c] zt[8J+c] to its row partial (summed over c when the wave leaves block row I) and
// X[8I+r][8J+c] zt[8I+r] to column 8J+c (summed over r at once).  A pair tile's lanes add the
// same two terms for the entry of their own diagonal block with LDS atomic adds (lanes of one row
// or column share an address); the lanes that hold the diagonal list add x_ii zt_i to row i
// alone.  Lane (r, c) = (lane % 4,
// lane / 4) of 4x16 tile q adds row 8I+r, column 16q+c of the last block row I, the transposed
// entry only left of the diagonal block (which the 4x16 tiles hold in full).  The pair and
// diagonal tiles have a loop of their own after the off-diagonal stream, so that the stream keeps
// its registers.  zt and y are LDS vectors (re at [0, ldt), im at [ldt, 2 ldt), ldt =
// 8 ceil(nr / 8)); y is this wave's own buffer and must start at zero.
template <typename T, bool NTL, bool CP>
__device__ inline void sym_tiles_apply(__amdgpu_buffer_rsrc_t rs, int nr, const double* zt, int ldt, double* y, int w,
                                       int nw) {
  constexpr int P = 8 / int(sizeof(T));  // tiles per unit: one 8-byte load per lane
  constexpr int UB = 8 / P;                  // units per batch of 8 tiles
  const int lane = threadIdx.x & 63, rr = lane & 7, cc = lane >> 3;
  const double* zr = zt;
  const double* zi = zt + ldt;
  double* yr = y;
  double* yi = y + ldt;
  const int nd = sym_nd(nr), noff = sym_off_tiles(nr), npair = sym_pair_tiles(nr);
  const int npd = npair + sym_diag_tiles(nr), ndl = sym_dlist(nr), ndp = sym_dlist_in_pair(nr);
  const int nh = sym_half_tiles(nr);
  const int nof2 = sym_off_slots(nr, P), ntf2 = sym_full_slots(nr, P);
  const int im = sym_slots(nr, P) * 64 * int(sizeof(T));
  // off-diagonal tiles
  int I = 1, J = w * P;  // the wave's first tile I(I-1)/2 + J, J < I
  while (J >= I) {
    J -= I;
    ++I;
  }
  int curI = I;
  double rowr = 0.0, rowi = 0.0;
  auto flush = [&](int Ir) {  // sum the row partials of block row Ir over c
#pragma unroll
    for (int sh = 8; sh < 64; sh <<= 1) {
      rowr += __shfl_xor(rowr, sh);
      if constexpr (CP) rowi += __shfl_xor(rowi, sh);
    }
    if (cc == 0) {
      yr[8 * Ir + rr] += rowr;
      if constexpr (CP) yi[8 * Ir + rr] += rowi;
    }
    rowr = rowi = 0.0;
  };
  for (int u0 = w; u0 * P < noff; u0 += UB * nw) {
    T xr[8], xi[8];
#pragma unroll
    for (int b = 0; b < UB; ++b) {
      const int u = u0 + b * nw;
      const int e = (u * 64 + lane) * P * int(sizeof(T));
      if (u * P < noff) {
        bld_unit<T, NTL>(rs, e, xr + b * P);
        if constexpr (CP) bld_unit<T, NTL>(rs, e + im, xi + b * P);
      } else {
#pragma unroll
        for (int s = 0; s < P; ++s) xr[b * P + s] = xi[b * P + s] = T(0);
      }
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((u0 + (k / P) * nw) * P + k % P >= noff) break;
      if (I != curI) {
        flush(curI);
        curI = I;
      }
      const double ar = double(xr[k]);
      const double zjr = zr[8 * J + cc];
      const double zir = zr[8 * I + rr];
      if constexpr (CP) {
        const double ai = double(xi[k]);
        const double zji = zi[8 * J + cc], zii = zi[8 * I + rr];
        rowr += ar * zjr - ai * zji;
        rowi += ar * zji + ai * zjr;
        const double cr = dpp_sum8(ar * zir - ai * zii), ci = dpp_sum8(ar * zii + ai * zir);
        if (rr == 0) {
          yr[8 * J + cc] += cr;
          yi[8 * J + cc] += ci;
        }
      } else {
        rowr += ar * zjr;
        const double cr = dpp_sum8(ar * zir);
        if (rr == 0) yr[8 * J + cc] += cr;
      }
      J += k % P == P - 1 ? P * nw - (P - 1) : 1;  // the next tile of this wave
      while (J >= I) {
        J -= I;
        ++I;
      }
    }
  }
  if (w * P < noff) flush(curI);
  // pair and diagonal tiles (units after the nof2 / P units of the off-diagonal section)
  auto diag_entry = [&](int s, double ar, double ai) {  // x_ii of the list (s < ndl): y_i += x_ii zt_i
    if (s < ndl) {
      const int x = 16 * (s >> 3) + 8 + (s & 7);
      if constexpr (CP) {
        const double vr = zr[x], vi = zi[x];
        yr[x] += ar * vr - ai * vi;
        yi[x] += ar * vi + ai * vr;
      } else {
        yr[x] += ar * zr[x];
      }
    }
  };
  for (int u0 = w; u0 * P < npd; u0 += nw) {
    T xr[P], xi[P];
    const int e = ((nof2 / P + u0) * 64 + lane) * P * int(sizeof(T));
    bld_unit<T, NTL>(rs, e, xr);
    if constexpr (CP) bld_unit<T, NTL>(rs, e + im, xi);
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const int t = u0 * P + k;
      if (t >= npd) break;
      const double ar = double(xr[k]);
      const double ai = CP ? double(xi[k]) : 0.0;
      if (t < npair) {  // pair tile: block A at r >= c, block B transposed at r < c
        const int A = 2 * t, B = A + 1;
        const bool lo = rr >= cc;
        if (lo || B < nd) {
          // the entry couples i = base + r and j = base + c of the lane's block (block B's is
          // stored transposed, which the symmetric coupling does not see): y_i += v zt_j and, off
          // the diagonal, y_j += v zt_i, as LDS atomic adds (several lanes share each row)
          const int base = lo ? 8 * A : 8 * B, i = base + rr, j = base + cc;
          if constexpr (CP) {
            const double zjr = zr[j], zji = zi[j];
            lds_add(yr + i, ar * zjr - ai * zji);
            lds_add(yi + i, ar * zji + ai * zjr);
            if (rr != cc) {
              const double zir = zr[i], zii = zi[i];
              lds_add(yr + j, ar * zir - ai * zii);
              lds_add(yi + j, ar * zii + ai * zir);
            }
          } else {
            lds_add(yr + i, ar * zr[j]);
            if (rr != cc) lds_add(yr + j, ar * zr[i]);
          }
        } else {  // no block B: the lanes r < c hold the diagonal list
          diag_entry(cc * (cc - 1) / 2 + rr, ar, ai);
        }
      } else {  // diagonal tile
        diag_entry(ndp + 64 * (t - npair) + lane, ar, ai);
      }
    }
  }
  if (w * P >= nh) return;
  // 4x16 tiles of the last block row Ih = 2 nh - 1 (units after the ntf2 / P units of 8x8 tiles)
  constexpr int UH = 4 / P;  // units per batch of 4 tiles
  const int hr = lane & 3, hc = lane >> 2, Ih = 2 * nh - 1;
  const double zhr = zr[8 * Ih + hr];
  const double zhi = CP ? zi[8 * Ih + hr] : 0.0;
  rowr = rowi = 0.0;
  for (int u0 = w; u0 * P < nh; u0 += UH * nw) {
    T xr[4], xi[4];
#pragma unroll
    for (int b = 0; b < UH; ++b) {
      const int u = u0 + b * nw;
      const int e = ((ntf2 / P + u) * 64 + lane) * P * int(sizeof(T));
      if (u * P < nh) {
        bld_unit<T, NTL>(rs, e, xr + b * P);
        if constexpr (CP) bld_unit<T, NTL>(rs, e + im, xi + b * P);
      } else {
#pragma unroll
        for (int s = 0; s < P; ++s) xr[b * P + s] = xi[b * P + s] = T(0);
      }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = (u0 + (k / P) * nw) * P + k % P;
      if (q >= nh) break;
      const int col = 16 * q + hc;
      const double ar = double(xr[k]);
      const double ai = CP ? double(xi[k]) : 0.0;
      const double zjr = zr[col];
      if constexpr (CP) {
        const double zji = zi[col];
        rowr += ar * zjr - ai * zji;
        rowi += ar * zji + ai * zjr;
      } else {
        rowr += ar * zjr;
      }
      if (16 * q < 8 * Ih) {  // the tile has columns left of the diagonal block
        const bool below = col < 8 * Ih;
        if constexpr (CP) {
          const double cr = dpp_sum4(below ? ar * zhr - ai * zhi : 0.0);
          const double ci = dpp_sum4(below ? ar * zhi + ai * zhr : 0.0);
          if (hr == 0 && below) {
            yr[col] += cr;
            yi[col] += ci;
          }
        } else {
          const double cr = dpp_sum4(below ? ar * zhr : 0.0);
          if (hr == 0 && below) yr[col] += cr;
        }
      }
    }
  }
#pragma unroll
  for (int sh = 4; sh < 64; sh <<= 1) {  // row sums over c
    rowr += __shfl_xor(rowr, sh);
    if constexpr (CP) rowi += __shfl_xor(rowi, sh);
  }
  if (hc == 0) {
    yr[8 * Ih + hr] += rowr;
    if constexpr (CP) yi[8 * Ih + hr] += rowi;
  }
}

// The sizes and offsets of one patch's reduced solve.
struct RedPatch {
  int64_t o, base, nsmall;
  int n, ns, nU, nP, nn, nr, ldn, ldp, ldr;
};
__device__ inline RedPatch red_patch(const TimeBlockConsts& tb, int d, int64_t p, const int64_t* __restrict__ poff,
                                     const int32_t* __restrict__ pnu, const int64_t* __restrict__ ioff) {
  RedPatch P;
  P.o = poff[p];
  P.n = int(poff[p + 1] - P.o);
  P.ns = P.n / tb.nt;
  P.nU = pnu[p];
  P.nP = P.ns - 2 * P.nU;
  P.nn = P.nU / d;
  P.nr = P.nU + P.nP;
  P.ldn = inv_ld(P.nn);
  P.ldp = inv_ld(P.nP);
  P.ldr = inv_ld(P.nr);
  P.base = ioff[p];
  P.nsmall = int64_t(P.nn) * P.ldn + int64_t(P.nU) * P.ldp;  // (rho M)^{-1} and G
  return P;
}

// Front of the reduced solve, threads t0, t0 + nth, ... of the patch's thread set, sync() between
// phases: r_P gathered into rl (n), transformed to the eigenvalue blocks in sv ([a][re, im][ns]),
// then w = (rho M)^{-1} r_u per component into wv (planes of nU, red_pl) and z = [r_v + lam r_u;
// r_p + G r_u] into z (planes of ldr).  rl may share memory with wv and z (it is dead once sv
// is formed); the caller synchronises after the last phase.
template <typename T, bool NTL, typename Sync>
__device__ inline void red_front(const TimeBlockConsts& tb, int d, const RedPatch& P, const int32_t* __restrict__ pdof,
                                 const T* __restrict__ inv, const double* __restrict__ r, double* rl, double* sv,
                                 double* wv, double* z, int t0, int nth, Sync sync) {
  const int nt = tb.nt, nblk = tb.nblk, n = P.n, ns = P.ns, nU = P.nU, nn = P.nn, nr = P.nr, ldr = P.ldr;
  // gather r_P: batches of independent index and value loads
  for (int ib = t0; ib < n; ib += 8 * nth) {
    int32_t g[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = ib + u * nth;
      g[u] = i < n ? pdof[P.o + i] : 0;
    }
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = ib + u * nth < n ? r[g[u]] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (ib + u * nth < n) rl[ib + u * nth] = v[u];
  }
  sync();
  for (int i = t0; i < ns; i += nth)
    for (int a = 0; a < nblk; ++a) {
      double sr = 0.0, si = 0.0;
      for (int b = 0; b < nt; ++b) {
        const double x = rl[b * ns + i];
        sr += tb.tin[2 * (a * nt + b)] * x;
        si += tb.tin[2 * (a * nt + b) + 1] * x;
      }
      sv[(2 * a) * ns + i] = sr;
      sv[(2 * a + 1) * ns + i] = si;
    }
  sync();
  // items [0, nU): w = (rho M)^{-1} r_u per component and z_U = r_v + lam r_u;
  // items [nU, nr): z_P = r_p + G r_u
  const __amdgpu_buffer_rsrc_t rs = patch_rsrc(inv + P.base, P.nsmall);
  int pl[RED_MAXB];
#pragma unroll
  for (int a = 0; a < RED_MAXB; ++a) pl[a] = red_pl(tb, a);
  for (int it = t0; it < nr; it += nth) {
    double ar[RED_MAXB] = {0, 0}, ai[RED_MAXB] = {0, 0};
    const bool vel = it < nU;
    // element j of the row: byte offset e0 + j * es (column-major: adjacent lanes read
    // adjacent entries)
    const int e0 = int(sizeof(T)) * (vel ? it / d : nn * P.ldn + (it - nU));
    const int es = int(sizeof(T)) * (vel ? P.ldn : P.ldp);
    const int m = vel ? nn : nU;
    const int sstep = vel ? d : 1, s0 = vel ? it % d : 0;  // r_u entries: j * d + c (mass) or j (G)
    int j = 0;
    for (; j + 7 < m; j += 8) {
      T mv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) mv[u] = bld1<T, NTL>(rs, e0 + (j + u) * es);
#pragma unroll
      for (int u = 0; u < 8; ++u)
#pragma unroll
        for (int a = 0; a < RED_MAXB; ++a)
          if (a < nblk) {
            ar[a] += double(mv[u]) * sv[(2 * a) * ns + (j + u) * sstep + s0];
            ai[a] += double(mv[u]) * sv[(2 * a + 1) * ns + (j + u) * sstep + s0];
          }
    }
    for (; j < m; ++j) {
      const double mv = double(bld1<T, NTL>(rs, e0 + j * es));
#pragma unroll
      for (int a = 0; a < RED_MAXB; ++a)
        if (a < nblk) {
          ar[a] += mv * sv[(2 * a) * ns + j * sstep + s0];
          ai[a] += mv * sv[(2 * a + 1) * ns + j * sstep + s0];
        }
    }
#pragma unroll
    for (int a = 0; a < RED_MAXB; ++a)
      if (a < nblk) {
        if (vel) {
          const double al = tb.lam[2 * a], be = tb.lam[2 * a + 1];
          const bool c = tb.cplx[a] != 0;
          const double ur = sv[(2 * a) * ns + it], ui = sv[(2 * a + 1) * ns + it];
          wv[pl[a] * nU + it] = ar[a];
          z[pl[a] * ldr + it] = sv[(2 * a) * ns + nU + it] + al * ur - be * ui;
          if (c) {
            wv[(pl[a] + 1) * nU + it] = ai[a];
            z[(pl[a] + 1) * ldr + it] = sv[(2 * a + 1) * ns + nU + it] + al * ui + be * ur;
          }
        } else {
          z[pl[a] * ldr + it] = sv[(2 * a) * ns + nU + it] + ar[a];
          if (tb.cplx[a]) z[(pl[a] + 1) * ldr + it] = sv[(2 * a + 1) * ns + nU + it] + ai[a];
        }
      }
  }
}

// Symmetric tiles: zt = D1 z (planes of LDT, zero padded beyond nr).
__device__ inline void sym_scale_z(const TimeBlockConsts& tb, const RedPatch& P, int LDT, const double* z, double* zt,
                                   int t0, int nth) {
  const int nblk = tb.nblk, nr = P.nr, nU = P.nU, ldr = P.ldr;
  for (int x = t0; x < LDT; x += nth)
#pragma unroll
    for (int a = 0; a < RED_MAXB; ++a)
      if (a < nblk) {
        double m1r, m1i, m2r, m2i;
        sym_factors(tb.lam[2 * a], tb.lam[2 * a + 1], &m1r, &m1i, &m2r, &m2i);
        const int pa = red_pl(tb, a);
        const bool c = tb.cplx[a] != 0;
        double vr = x < nr ? z[pa * ldr + x] : 0.0, vi = x < nr && c ? z[(pa + 1) * ldr + x] : 0.0;
        if (x >= nU) {
          const double ur = vr * m1r - vi * m1i, ui = vr * m1i + vi * m1r;
          vr = ur;
          vi = ui;
        }
        zt[pa * LDT + x] = vr;
        if (c) zt[(pa + 1) * LDT + x] = vi;
      }
}

// Symmetric tiles: wave w of W adds X D1 z of every kept eigenvalue into its own partial
// products tt + w * npl LDT (planes of LDT, zeroed by the caller).
template <typename T, bool NTL>
__device__ inline void sym_apply_blocks(const TimeBlockConsts& tb, const RedPatch& P, int LDT,
                                        const T* __restrict__ inv, const double* zt, double* tt, int w, int W) {
  const int nblk = tb.nblk, nr = P.nr;
  const int nsl = sym_slots(nr, 8 / int(sizeof(T)));  // stored tiles per plane
  int64_t off = P.base + P.nsmall;
  for (int a = 0; a < nblk; ++a) {
    const bool cp = tb.cplx[a] != 0;
    const int64_t cnt = int64_t(cp ? 2 : 1) * nsl * 64;
    const __amdgpu_buffer_rsrc_t rs = patch_rsrc(inv + off, cnt);
    const int pa = red_pl(tb, a);
    double* yw = tt + (int64_t(w) * red_npl(tb) + pa) * LDT;
    if (cp)
      sym_tiles_apply<T, NTL, true>(rs, nr, zt + pa * LDT, LDT, yw, w, W);
    else
      sym_tiles_apply<T, NTL, false>(rs, nr, zt + pa * LDT, LDT, yw, w, W);
    off += cnt;
  }
}

// Symmetric tiles: t_P = mu2 (X D1 z)_P in each of the W partial products.
__device__ inline void sym_scale_t(const TimeBlockConsts& tb, const RedPatch& P, int LDT, int W, double* tt, int t0,
                                   int nth) {
  const int nblk = tb.nblk, nU = P.nU, nP = P.nP;
  for (int q = t0; q < W * nP; q += nth)
#pragma unroll
    for (int a = 0; a < RED_MAXB; ++a)
      if (a < nblk) {
        const int ww = q / nP, x = nU + q % nP;
        double m1r, m1i, m2r, m2i;
        sym_factors(tb.lam[2 * a], tb.lam[2 * a + 1], &m1r, &m1i, &m2r, &m2i);
        const bool c = tb.cplx[a] != 0;
        double* yb = tt + (int64_t(ww) * red_npl(tb) + red_pl(tb, a)) * LDT;
        const double vr = yb[x], vi = c ? yb[LDT + x] : 0.0;
        yb[x] = vr * m2r - vi * m2i;
        if (c) yb[LDT + x] = vr * m2i + vi * m2r;
      }
}

// Back of the reduced solve: the spatial images [lam U - w; U; P] (the sum of the W partial
// products at stride LDT, and w) transformed back to the time nodes and written to the image
// slots y[tpos[o + l]].
__device__ inline void red_back(const TimeBlockConsts& tb, const RedPatch& P, int LDT, int W, const double* tv,
                                const double* wv, const int32_t* __restrict__ tpos, double* __restrict__ y, int t0,
                                int nth) {
  const int nt = tb.nt, nblk = tb.nblk, ns = P.ns, nU = P.nU;
  for (int i = t0; i < ns; i += nth) {
    const int ii = i < nU ? i : i - nU;
    double hr[RED_MAXB], hi[RED_MAXB];
#pragma unroll
    for (int a = 0; a < RED_MAXB; ++a)
      if (a < nblk) {
        const bool c = tb.cplx[a] != 0;
        const int pa = red_pl(tb, a), npl = red_npl(tb);
        double t_r = 0.0, t_i = 0.0;
        for (int ww = 0; ww < W; ++ww) {
          t_r += tv[(int64_t(ww) * npl + pa) * LDT + ii];
          if (c) t_i += tv[(int64_t(ww) * npl + pa + 1) * LDT + ii];
        }
        if (i < nU) {
          const double al = tb.lam[2 * a], be = tb.lam[2 * a + 1];
          hr[a] = al * t_r - be * t_i - wv[pa * nU + i];
          hi[a] = c ? al * t_i + be * t_r - wv[(pa + 1) * nU + i] : 0.0;
        } else {
          hr[a] = t_r;
          hi[a] = t_i;
        }
      }
    for (int b = 0; b < nt; ++b) {
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < RED_MAXB; ++a)
        if (a < nblk) {
          const double qr = tb.qout[2 * (b * nblk + a)], qi = tb.qout[2 * (b * nblk + a) + 1];
          acc += tb.cplx[a] ? 2.0 * (qr * hr[a] - qi * hi[a]) : qr * hr[a];
        }
      y[tpos[P.o + b * ns + i]] = acc;
    }
  }
}

struct BlockSync {
  __device__ void operator()() const { __syncthreads(); }
};

template <typename T, int R, bool NTL, bool SYM>
__device__ __forceinline__ void patch_apply_red_body(TimeBlockConsts tb, int d, int W, int xc,
                                                     const int64_t* __restrict__ poff, const int32_t* __restrict__ pdof,
                                                     const int32_t* __restrict__ tpos, const int32_t* __restrict__ pnu,
                                                     const int64_t* __restrict__ ioff, const T* __restrict__ inv,
                                                     const double* __restrict__ r, double* __restrict__ y) {
  typedef T V __attribute__((ext_vector_type(R)));
  extern __shared__ double sm[];
  const int64_t p = xcd_chunk(blockIdx.x, gridDim.x, xc);
  const RedPatch P = red_patch(tb, d, p, poff, pnu, ioff);
  const int nblk = tb.nblk;
  const int n = P.n, ns = P.ns, nU = P.nU, nr = P.nr, ldr = P.ldr;
  // region A: r_P, later w (npl planes of nU) and z (npl planes of ldr);
  // region B: transformed right-hand sides [a][re, im][ns], later W partial images (W npl planes)
  const int npl = red_npl(tb);
  const int szA = max(n, npl * (nU + ldr));
  double* rl = sm;
  double* wv = sm;
  double* z = sm + npl * nU;
  double* sv = sm + szA;
  double* tv = sm + szA;
  red_front<T, NTL>(tb, d, P, pdof, inv, r, rl, sv, wv, z, int(threadIdx.x), int(blockDim.x), BlockSync());
  __syncthreads();
  // symmetric tiles (one wave): t = D2 X D1 z per kept eigenvalue into region B, stride LDT
  const int LDT = SYM ? 8 * ((nr + 7) >> 3) : ldr;
  if constexpr (SYM) {
    // W waves: wave w's products at tv + w * npl LDT (planes of LDT, the partial images the
    // back-transform sums), then D1 z shared by all waves
    double* tt = tv;
    double* zt = tv + int64_t(W) * npl * LDT;  // planes of LDT: D1 z, zero padded
    for (int x = threadIdx.x; x < int64_t(W) * npl * LDT; x += blockDim.x) tt[x] = 0.0;
    sym_scale_z(tb, P, LDT, z, zt, int(threadIdx.x), int(blockDim.x));
    __syncthreads();
    sym_apply_blocks<T, NTL>(tb, P, LDT, inv, zt, tt, int(threadIdx.x >> 6), W);
    __syncthreads();
    sym_scale_t(tb, P, LDT, W, tt, int(threadIdx.x), int(blockDim.x));  // every wave's part
  } else {
    const int per_w = blockDim.x / W;
    const int w = threadIdx.x / per_w, tl = threadIdx.x % per_w;
    const int i0 = R * tl;
    const int jc = (nr + W - 1) / W, j0 = w * jc, j1 = min(nr, j0 + jc);
    const int voff = i0 * int(sizeof(T));
    int64_t off = P.base + P.nsmall;
    for (int a = 0; a < nblk; ++a) {
      const double* zr = z + red_pl(tb, a) * ldr;
      const double* zi = zr + ldr;  // complex blocks only
      double* twr = tv + (int64_t(w) * npl + red_pl(tb, a)) * ldr;
      double* twi = twr + ldr;  // complex blocks only
      const bool cp = tb.cplx[a] != 0;
      const int64_t cnt = int64_t(nr) * (cp ? 2 * ldr : ldr);
      if (w < W && i0 < ldr) {
        const __amdgpu_buffer_rsrc_t rs = patch_rsrc(inv + off, cnt);
        double accr[R], acci[R];
#pragma unroll
        for (int q = 0; q < R; ++q) accr[q] = acci[q] = 0.0;
        if (!cp) {
          const int cb = ldr * int(sizeof(T));  // bytes per column
          const int vo = voff + j0 * cb;
          V A[8];
          auto load = [&](V* buf, int jr) {  // columns j0 + jr + u
#pragma unroll
            for (int u = 0; u < 8; ++u) buf[u] = bld16<V, NTL>(rs, vo, (jr + u) * cb);
          };
          auto sum = [&](const V* buf, int jj) {
#pragma unroll
            for (int u = 0; u < 8; u += 2)
#pragma unroll
              for (int q = 0; q < R; ++q) {
                accr[q] += double(buf[u][q]) * zr[jj + u];
                acci[q] += double(buf[u + 1][q]) * zr[jj + u + 1];
              }
          };
          const int nb = (j1 - j0) / 8;
          for (int b = 0; b < nb; ++b) {
            load(A, 8 * b);
            sum(A, j0 + 8 * b);
          }
          const int jt = j0 + 8 * nb, vt = voff + jt * cb;
          for (int t = 0; t < j1 - jt; ++t) {
            const V v0 = bld16<V, NTL>(rs, vt, t * cb);
#pragma unroll
            for (int q = 0; q < R; ++q) accr[q] += double(v0[q]) * zr[jt + t];
          }
#pragma unroll
          for (int q = 0; q < R; ++q) twr[i0 + q] = accr[q] + acci[q];
        } else {
          const int cb = 2 * ldr * int(sizeof(T)), ib = ldr * int(sizeof(T));  // column, Im offset
          const int vo = voff + j0 * cb;
          V Ar[8], Ai[8];
          const int nb = (j1 - j0) / 8;
          for (int b = 0; b < nb; ++b) {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              Ar[u] = bld16<V, NTL>(rs, vo, (8 * b + u) * cb);
              Ai[u] = bld16<V, NTL>(rs, vo + ib, (8 * b + u) * cb);
            }
            const int jj = j0 + 8 * b;
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
              for (int q = 0; q < R; ++q) {
                accr[q] += double(Ar[u][q]) * zr[jj + u] - double(Ai[u][q]) * zi[jj + u];
                acci[q] += double(Ai[u][q]) * zr[jj + u] + double(Ar[u][q]) * zi[jj + u];
              }
          }
          const int jt = j0 + 8 * nb, vt = voff + jt * cb;
          for (int t = 0; t < j1 - jt; ++t) {
            const V a0 = bld16<V, NTL>(rs, vt, t * cb), b0 = bld16<V, NTL>(rs, vt + ib, t * cb);
#pragma unroll
            for (int q = 0; q < R; ++q) {
              accr[q] += double(a0[q]) * zr[jt + t] - double(b0[q]) * zi[jt + t];
              acci[q] += double(b0[q]) * zr[jt + t] + double(a0[q]) * zi[jt + t];
            }
          }
#pragma unroll
          for (int q = 0; q < R; ++q) {
            twr[i0 + q] = accr[q];
            twi[i0 + q] = acci[q];
          }
        }
      }
      off += cnt;
    }
  }
  __syncthreads();
  // spatial images [lam U - w; U; P], transformed back to the time nodes (products at stride
  // LDT: the square path's W partial images, or the tiled path's single result)
  red_back(tb, P, LDT, W, tv, wv, tpos, y, int(threadIdx.x), int(blockDim.x));
}

// Square Schur inverses: W column ranges per block of up to 512 threads.
template <typename T, int R, bool NTL>
__global__ void __launch_bounds__(512) patch_apply_red_kernel(TimeBlockConsts tb, int d, int W, int xc,
                                                              const int64_t* __restrict__ poff,
                                                              const int32_t* __restrict__ pdof,
                                                              const int32_t* __restrict__ tpos,
                                                              const int32_t* __restrict__ pnu,
                                                              const int64_t* __restrict__ ioff,
                                                              const T* __restrict__ inv, const double* __restrict__ r,
                                                              double* __restrict__ y) {
  patch_apply_red_body<T, R, NTL, false>(tb, d, W, xc, poff, pdof, tpos, pnu, ioff, inv, r, y);
}

// Symmetric tiles: NW waves per patch (one on large levels, several where the level has too
// few patches to fill the chip and a patch's serial chain sets the time).  The register budget
// is held to 6 waves per SIMD (80 VGPRs) for the one-wave kernels: the kernel is bound by the
// HBM loads in flight, and the LDS of a 59-row dG(2) patch (6.1 KB) allows 26 waves per CU.
// The several-wave kernels of the small levels do not fit in 80 VGPRs without spilling; they
// get 5 waves (96 VGPRs).
template <typename T, int NW>
constexpr int sym_waves_per_eu() { return NW == 1 ? 6 : 5; }
template <typename T, bool NTL, int NW>
__global__ void __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(sym_waves_per_eu<T, NW>())))
patch_apply_red_sym_kernel(TimeBlockConsts tb, int d, int xc, const int64_t* __restrict__ poff,
                           const int32_t* __restrict__ pdof, const int32_t* __restrict__ tpos,
                           const int32_t* __restrict__ pnu, const int64_t* __restrict__ ioff,
                           const T* __restrict__ inv, const double* __restrict__ r, double* __restrict__ y) {
  patch_apply_red_body<T, 2, NTL, true>(tb, d, NW, xc, poff, pdof, tpos, pnu, ioff, inv, r, y);
}

// G = KK_pV ((rho M)^{-1} (x) I_d) in place of KK_pV in the stored layout of the reduced
// solves (column-major, leading dimension inv_ld(nP)), one block per patch of the batch:
// G[x][m d + c] = sum_b KK_pV[x][b d + c] Minv[b][m].
template <typename T>
__global__ void __launch_bounds__(256) fold_reduced_kernel(int d, const int32_t* __restrict__ ns_of,
                                                           const int32_t* __restrict__ nu_of,
                                                           const GjDesc* __restrict__ desc, int dstride,
                                                           T* __restrict__ out) {
  extern __shared__ double kl[];  // KK_pV, nU x ldp (column-major, as stored)
  const int64_t i = blockIdx.x;
  const int ns = ns_of[i], nU = nu_of[i], nP = ns - 2 * nU, nn = nU / d;
  const int ldn = inv_ld(nn), ldp = inv_ld(nP);
  const T* Minv = out + desc[i * dstride].ooff;
  T* Gp = out + desc[i * dstride].ooff + int64_t(nn) * ldn;
  for (int q = threadIdx.x; q < nU * ldp; q += blockDim.x) kl[q] = double(Gp[q]);
  __syncthreads();
  for (int q = threadIdx.x; q < nU * ldp; q += blockDim.x) {
    const int col = q / ldp, x = q % ldp;  // G[x][col], col = m d + c
    if (x >= nP) continue;                 // padding rows stay zero
    const int m = col / d, c = col % d;
    double acc = 0.0;
    for (int b = 0; b < nn; ++b) acc += kl[(b * d + c) * ldp + x] * double(Minv[int64_t(m) * ldn + b]);
    Gp[q] = T(acc);
  }
}

// d[mu] += winv[mu] * sum of the patch images of mu, stored dof-major: the patch kernels write
// the image of patch entry (p, l) at tpos[poff[p] + l], and the slots of mu are
// [tptr[mu], tptr[mu + 1]) in patch order.
template <bool ASSIGN>  // ASSIGN: d = winv (sum of the slots), for a sweep from d = 0
__global__ void vanka_update_kernel(int64_t n, const int64_t* __restrict__ tptr, const double* __restrict__ winv,
                                    const double* __restrict__ y, double* __restrict__ d) {
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t t = tptr[i]; t < tptr[i + 1]; ++t) s += y[t];
  if (ASSIGN)
    d[i] = winv[i] * s;
  else
    d[i] += winv[i] * s;
}

// ---------------------------------------------------------------- dense coarse solve
// y = X b with X stored column by column (X[i][j] at j*ld + i, ld = inv_ld(n)).
// Block (bx, by) sums columns [by*GEMV_COLS, ...) for rows [bx*256, ...) into
// part[by][i]; dense_gemv_reduce adds the column chunks in order.
constexpr int GEMV_COLS = 64;  // column chunk per workgroup: about 85 workgroups for 1,047 unknowns
__global__ void __launch_bounds__(256) dense_gemv_part_kernel(int n, const double* __restrict__ Xt,
                                                              const double* __restrict__ b,
                                                              double* __restrict__ part) {
  __shared__ double sb[GEMV_COLS];
  const int j0 = blockIdx.y * GEMV_COLS, j1 = min(n, j0 + GEMV_COLS);
  for (int j = j0 + threadIdx.x; j < j1; j += blockDim.x) sb[j - j0] = b[j];
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int ld = inv_ld(n);
  double a0 = 0, a1 = 0;
  int j = j0;
  for (; j + 1 < j1; j += 2) {
    a0 += Xt[int64_t(j) * ld + i] * sb[j - j0];
    a1 += Xt[int64_t(j + 1) * ld + i] * sb[j + 1 - j0];
  }
  if (j < j1) a0 += Xt[int64_t(j) * ld + i] * sb[j - j0];
  part[int64_t(blockIdx.y) * n + i] = a0 + a1;
}

__global__ void dense_gemv_reduce_kernel(int n, int nchunk, const double* __restrict__ part, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[int64_t(c) * n + i];
  y[i] = s;
}

// ---------------------------------------------------------------- large Gauss-Jordan
// The same blocked Gauss-Jordan as gj_invert_kernel for one matrix too large
// for a workgroup (M row-major n x n).  Per panel of nb columns: the panel is
// copied column-major into a scratch buffer, gj_large_column eliminates it one
// pivot column per launch over as many workgroups as the rows need (two
// ping-pong buffers), gj_large_swap applies the panel's row swaps to the other
// columns and copies the pivot rows to Wb, gj_large_update performs the rank-nb
// update over 2D tiles, and the eliminated panel is copied back.
__global__ void __launch_bounds__(1024) gj_large_rowscale_kernel(int n, double* __restrict__ M,
                                                                 double* __restrict__ scl) {
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int i = blockIdx.x * (blockDim.x / WAVE) + wave;
  if (i >= n) return;
  double m = 0.0;
  for (int j = lane; j < n; j += WAVE) m = fmax(m, fabs(M[int64_t(i) * n + j]));
  for (int off = WAVE / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  const double s = (m > 0.0 && isfinite(m)) ? ldexp(1.0, -ilogb(m)) : 1.0;
  for (int j = lane; j < n; j += WAVE) M[int64_t(i) * n + j] *= s;
  if (lane == 0) scl[i] = s;
}

// One pivot column of the panel, over many workgroups.  The panel is held column-major
// (P[c * n + i] = M[i][k0 + c]) in two buffers: every workgroup reads Pin only and writes its own
// rows of Pout, so no workgroup can see a half-updated column.  Each workgroup repeats the pivot
// search of column c over rows k..n-1 (the same rows and tie rule in every workgroup: the largest
// scaled entry, ties to the lowest row), forms the new pivot row (the old row p divided by the
// pivot, with 1/pivot in column c) and writes, for its rows i != k, the old row (row k's values
// for i = p, the row swap) minus its column-c entry times the new pivot row (column c: 0 minus
// it).  These are the same operations, in the same order per element, as one step of the
// workgroup Gauss-Jordan kernels.
__global__ void __launch_bounds__(256) gj_large_column_kernel(int n, int k0, int c, int nb,
                                                              const double* __restrict__ Pin,
                                                              double* __restrict__ Pout, int* __restrict__ perm,
                                                              int32_t* __restrict__ status) {
  __shared__ double rv[256 / WAVE];
  __shared__ int ri[256 / WAVE];
  __shared__ double prow[32];
  __shared__ int s_piv;
  const int tid = threadIdx.x, wave = tid / WAVE, lane = tid % WAVE, nw = blockDim.x / WAVE;
  const int k = k0 + c;
  const double* col = Pin + int64_t(c) * n;
  double bv = -1.0;
  int bi = n;
  for (int i = k + tid; i < n; i += blockDim.x) {
    const double v = fabs(col[i]);
    if (v > bv) {
      bv = v;
      bi = i;
    }
  }
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    const double ov = __shfl_xor(bv, off);
    const int oi = __shfl_xor(bi, off);
    if (ov > bv || (ov == bv && oi < bi)) {
      bv = ov;
      bi = oi;
    }
  }
  if (lane == 0) {
    rv[wave] = bv;
    ri[wave] = bi;
  }
  __syncthreads();
  if (tid == 0) {
    double v = rv[0];
    int ii = ri[0];
    for (int w = 1; w < nw; ++w)
      if (rv[w] > v || (rv[w] == v && ri[w] < ii)) {
        v = rv[w];
        ii = ri[w];
      }
    const bool bad = !(v > 0.0) || !isfinite(v) || ii >= n;
    if (bad) ii = k;
    if (blockIdx.x == 0) {
      perm[k] = ii;
      if (bad) status[0] = 1;
    }
    s_piv = ii;
  }
  __syncthreads();
  const int p = s_piv;
  double piv = col[p];
  if (piv == 0.0 || !isfinite(piv)) piv = 1.0;
  const double rp = 1.0 / piv;
  if (tid < nb) prow[tid] = (tid == c ? 1.0 : Pin[int64_t(tid) * n + p]) * rp;
  __syncthreads();
  const int i = blockIdx.x * blockDim.x + tid;
  if (i >= n) return;
  if (i == k) {
    for (int cc = 0; cc < nb; ++cc) Pout[int64_t(cc) * n + i] = prow[cc];
    return;
  }
  const int s = i == p ? k : i;
  const double f = Pin[int64_t(c) * n + s];
  for (int cc = 0; cc < nb; ++cc)
    Pout[int64_t(cc) * n + i] = (cc == c ? 0.0 : Pin[int64_t(cc) * n + s]) - f * prow[cc];
}

// P[c * n + i] = M[i][k0 + c] (to_panel) or back
__global__ void gj_large_panel_copy_kernel(int n, int k0, int nb, double* __restrict__ M, double* __restrict__ P,
                                           int to_panel) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (i >= n || c >= nb) return;
  if (to_panel)
    P[int64_t(c) * n + i] = M[int64_t(i) * n + k0 + c];
  else
    M[int64_t(i) * n + k0 + c] = P[int64_t(c) * n + i];
}

// columns outside the panel: apply the row swaps of this panel, copy the pivot rows to Wb[c][j]
__global__ void gj_large_swap_kernel(int n, int k0, int nb, double* __restrict__ M, const int* __restrict__ perm,
                                     double* __restrict__ Wb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= k0 && j < k0 + nb)) return;
  for (int c = 0; c < nb; ++c) {
    const int k = k0 + c, q = perm[k];
    if (q != k) {
      const double a = M[int64_t(k) * n + j];
      M[int64_t(k) * n + j] = M[int64_t(q) * n + j];
      M[int64_t(q) * n + j] = a;
    }
  }
  for (int c = 0; c < nb; ++c) Wb[int64_t(c) * n + j] = M[int64_t(k0 + c) * n + j];
}

// M[i][j] = [i not in panel rows] M[i][j] + sum_c P[c][i] Wb[c][j], j outside the panel
constexpr int GJL_ROWS = 128;
__global__ void __launch_bounds__(256) gj_large_update_kernel(int n, int k0, int nb, double* __restrict__ M,
                                                              const double* __restrict__ P,
                                                              const double* __restrict__ Wb) {
  __shared__ double pn[GJL_ROWS * 32];
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i0 = blockIdx.y * GJL_ROWS, i1 = min(n, i0 + GJL_ROWS);
  for (int t = threadIdx.x; t < (i1 - i0) * nb; t += blockDim.x) {
    const int c = t / (i1 - i0), i = t % (i1 - i0);
    pn[i * 32 + c] = P[int64_t(c) * n + i0 + i];
  }
  __syncthreads();
  if (j >= n || (j >= k0 && j < k0 + nb)) return;
  double w[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) w[c] = c < nb ? Wb[int64_t(c) * n + j] : 0.0;
  for (int i = i0; i < i1; ++i) {
    double acc = (i >= k0 && i < k0 + nb) ? 0.0 : M[int64_t(i) * n + j];
#pragma unroll
    for (int c = 0; c < 32; ++c) acc += pn[(i - i0) * 32 + c] * w[c];
    M[int64_t(i) * n + j] = acc;
  }
}

// out[i * ld + j] = M[i][src[j]] * scl[j] (zero padding for j >= n)
__global__ void gj_large_output_kernel(int n, const double* __restrict__ M, const int* __restrict__ src,
                                       const double* __restrict__ scl, double* __restrict__ out) {
  const int ld = inv_ld(n);
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= ld) return;
  out[int64_t(i) * ld + j] = j < n ? M[int64_t(i) * n + src[j]] * scl[j] : 0.0;
}

// ---------------------------------------------------------------- BLAS-1 (FGMRES)
// partials[v * nblk + blk] = sum over block blk's chunk of V_v . w
__global__ void __launch_bounds__(256) dot_partials_kernel(const double* __restrict__ V, int64_t ldv,
                                                           const double* __restrict__ w, int64_t n, int64_t chunk,
                                                           double* __restrict__ partials) {
  __shared__ double red[256 / WAVE];
  const int v = blockIdx.y;
  const int64_t lo = int64_t(blockIdx.x) * chunk, hi = min(n, lo + chunk);
  const double* Vv = V + int64_t(v) * ldv;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) acc += Vv[i] * w[i];
  for (int off = WAVE / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < int(blockDim.x / WAVE); ++q) s += red[q];
    partials[int64_t(v) * gridDim.x + blockIdx.x] = s;
  }
}

// out[v] = sum_b partials[v * nblk + b] (+ out[v] if accumulate)
__global__ void __launch_bounds__(256) reduce_partials_kernel(const double* __restrict__ partials, int nblk,
                                                              double* __restrict__ out, int accumulate) {
  __shared__ double red[256 / WAVE];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partials[int64_t(v) * nblk + b];
  for (int off = WAVE / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (threadIdx.x % WAVE == 0) red[threadIdx.x / WAVE] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int q = 0; q < int(blockDim.x / WAVE); ++q) s += red[q];
    out[v] = accumulate ? out[v] + s : s;
  }
}

// w += sign * sum_v h[v] V_v
__global__ void multi_axpy_kernel(const double* __restrict__ V, int64_t ldv, int m, const double* __restrict__ h,
                                  double sign, double* __restrict__ w, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < m; ++v) s += h[v] * V[int64_t(v) * ldv + i];
  w[i] += sign * s;
}

// dst = src * (1 / sqrt(*nrm2))  (nrm2 = squared norm on the device)
__global__ void scale_copy_kernel(const double* __restrict__ src, const double* __restrict__ nrm2,
                                  double* __restrict__ dst, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double nr = sqrt(*nrm2);
  dst[i] = nr > 0.0 ? src[i] / nr : 0.0;
}

// out = a*x + b*y elementwise
__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                             double* __restrict__ out, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// rhs[b*ns + i] = e_b * mmx[i] + src[b*ns + i]
// rhs may be src itself (each thread reads its entry before writing it)
__global__ void slab_rhs_kernel(int nt, int64_t ns, const double* __restrict__ e, const double* __restrict__ mmx,
                                const double* src, double* rhs) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= int64_t(nt) * ns) return;
  const int b = int(i / ns);
  rhs[i] = e[b] * mmx[i % ns] + src[i];
}

}  // namespace dev

// ================================================================= launchers
static inline int64_t blocks_for(int64_t n, int bs) { return (n + bs - 1) / bs; }

void k_csr(hipStream_t st, int mode, int64_t nrows, const int64_t* ptr, const int32_t* col, const double* val,
           const double* x, const double* b, double* y, int lanes) {
#define STGMG_CSR(G)                                                                  \
  if (mode == 0) dev::launch_csr<G, 0>(st, nrows, ptr, col, val, x, b, y);            \
  else if (mode == 1) dev::launch_csr<G, 1>(st, nrows, ptr, col, val, x, b, y);       \
  else dev::launch_csr<G, 2>(st, nrows, ptr, col, val, x, b, y);
  if (lanes <= 4) {
    STGMG_CSR(4)
  } else if (lanes <= 8) {
    STGMG_CSR(8)
  } else if (lanes <= 16) {
    STGMG_CSR(16)
  } else if (lanes <= 32) {
    STGMG_CSR(32)
  } else {
    STGMG_CSR(64)
  }
#undef STGMG_CSR
}

void k_kron_spmv(hipStream_t st, int mode, const TimeOp& top, int64_t ns, const int64_t* mptr, const int32_t* mcol,
                 const double* mval, const int64_t* kptr, const int32_t* kcol, const double* kval, const double* x,
                 const double* b, double* y, int lanes) {
  if (ns == 0) return;
  // at least nt lanes per row: lane b writes time node b
#define STGMG_KRON(G)                                                                              \
  if (mode == 0) dev::launch_kron<G, 0>(st, top, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y); \
  else dev::launch_kron<G, 1>(st, top, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y);
  if (lanes <= 4) {
    STGMG_KRON(4)
  } else if (lanes <= 8) {
    STGMG_KRON(8)
  } else if (lanes <= 16) {
    STGMG_KRON(16)
  } else {
    STGMG_KRON(32)
  }
#undef STGMG_KRON
}

template <int G, int MODE, int NT, int D>
static void launch_node_op(hipStream_t st, const TimeOp& top, const NodeOpDev& o, int64_t ns, const int64_t* mptr,
                           const int32_t* mcol, const double* mval, const int64_t* kptr, const int32_t* kcol,
                           const double* kval, const double* x, const double* b, double* y) {
  // lanes per pressure row as for the CSR kernel
  constexpr int GP = D == 2 ? 16 : 32;
  const int64_t nv = int64_t(D) * o.nQ, np = ns - 2 * nv;
  const int64_t nb_node = (o.nQ * G + 255) / 256, nb_p = (np * GP + 255) / 256;
  // each XCD takes chunks of xc consecutive node blocks, so that the x values of neighbouring
  // nodes are fetched into one XCD's L2 rather than into all eight: measured best of round-robin /
  // 16 / 64 / 256 / one range per XCD (256^2 dG(2): 0.136 -> 0.124 ms at 64; 32^3 dG(1):
  // 0.576 -> 0.532 ms at 16).  Tuning: STGMG_OP_XCD_CHUNK (0 round-robin, -1 one range per XCD).
  int64_t xc = D == 2 ? 64 : 16;
  if (const char* e = std::getenv("STGMG_OP_XCD_CHUNK")) xc = std::atoll(e);
  if (xc < 0) xc = std::max<int64_t>(1, nb_node / 8);
  hipLaunchKernelGGL((dev::node_op_kernel<G, GP, MODE, NT, D>), dim3(nb_node + nb_p), dim3(256), 0, st, top, o.nQ, nv,
                     ns, nb_node, o.ptr, o.col, o.m, o.a, o.cptr, o.ccol, o.c, mptr, mcol, mval, kptr, kcol, kval, x, b,
                     y, xc);
}

template <int MODE, int D>
static void node_op_nt(hipStream_t st, const TimeOp& top, const NodeOpDev& o, int64_t ns, const int64_t* mptr,
                       const int32_t* mcol, const double* mval, const int64_t* kptr, const int32_t* kcol,
                       const double* kval, const double* x, const double* b, double* y) {
  // lanes per node (a power of two): by default 4 for the ~16 node pairs of a 2D Q2 node, 8 for
  // the ~64 of a 3D one
  const int lanes = node_op_lanes(o);
#define STGMG_NODE(G)                                                                                    \
  switch (top.nt) {                                                                                      \
    case 1: launch_node_op<G, MODE, 1, D>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y); break; \
    case 2: launch_node_op<G, MODE, 2, D>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y); break; \
    case 3: launch_node_op<G, MODE, 3, D>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y); break; \
    default: launch_node_op<G, MODE, 4, D>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y); break; \
  }
  if (lanes <= 2) {
    STGMG_NODE(2)
  } else if (lanes <= 4) {
    STGMG_NODE(4)
  } else if (lanes <= 8) {
    STGMG_NODE(8)
  } else {
    STGMG_NODE(16)
  }
#undef STGMG_NODE
}

void k_node_op(hipStream_t st, int mode, const TimeOp& top, const NodeOpDev& o, int64_t ns, const int64_t* mptr,
               const int32_t* mcol, const double* mval, const int64_t* kptr, const int32_t* kcol, const double* kval,
               const double* x, const double* b, double* y) {
  if (ns == 0) return;
  if (o.d == 2) {
    if (mode == 0) node_op_nt<0, 2>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y);
    else node_op_nt<1, 2>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y);
  } else {
    if (mode == 0) node_op_nt<0, 3>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y);
    else node_op_nt<1, 3>(st, top, o, ns, mptr, mcol, mval, kptr, kcol, kval, x, b, y);
  }
}

void k_fill_zero(hipStream_t st, double* a, int64_t n) {
  if (n == 0) return;
  int64_t g = blocks_for(n, 256);
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(dev::fill_zero_kernel, dim3(g), dim3(256), 0, st, a, n);
}

void k_patch_extract_t(hipStream_t st, int64_t p0, int64_t count, int max_np, const int64_t* poff,
                       const int32_t* pdof, const int64_t* ptr, const int32_t* col, const double* val,
                       const int64_t* woff, double* W) {
  if (count == 0) return;
  hipLaunchKernelGGL(dev::patch_extract_t_kernel, dim3(count), dim3(256), size_t(max_np) * sizeof(int32_t), st, p0,
                     poff, pdof, ptr, col, val, woff, W);
}

size_t gj_lds_bytes(int max_np, int nb) {
  return (size_t(max_np) * nb + max_np + 16) * sizeof(double) + 2 * size_t(max_np) * sizeof(int);
}

int gj_panel_width(int max_np, size_t lds_limit) {
  for (int nb : {32, 16, 8, 4})
    if (gj_lds_bytes(max_np, nb) <= lds_limit) return nb;
  return 0;
}

template <typename T>
static void gj_launch(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, T* out,
                      int32_t* status) {
  const size_t lds = gj_lds_bytes(max_n, nb);
  switch (nb) {
    case 32:
      hipLaunchKernelGGL((dev::gj_invert_kernel<T, 32>), dim3(count), dim3(256), lds, st, desc, W, out, status);
      break;
    case 16:
      hipLaunchKernelGGL((dev::gj_invert_kernel<T, 16>), dim3(count), dim3(256), lds, st, desc, W, out, status);
      break;
    case 8:
      hipLaunchKernelGGL((dev::gj_invert_kernel<T, 8>), dim3(count), dim3(256), lds, st, desc, W, out, status);
      break;
    default:
      hipLaunchKernelGGL((dev::gj_invert_kernel<T, 4>), dim3(count), dim3(256), lds, st, desc, W, out, status);
      break;
  }
}

void k_gj_invert_f64(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, double* out,
                     int32_t* status) {
  if (count) gj_launch<double>(st, nb, count, max_n, desc, W, out, status);
}
void k_gj_invert_f32(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, float* out,
                     int32_t* status) {
  if (count) gj_launch<float>(st, nb, count, max_n, desc, W, out, status);
}
void k_gj_invert_bf16(hipStream_t st, int nb, int64_t count, int max_n, const GjDesc* desc, double* W, __bf16* out,
                      int32_t* status) {
  if (count) gj_launch<__bf16>(st, nb, count, max_n, desc, W, out, status);
}

int patch_apply_threads(int max_np, bool fp32) {
  const int rpt = fp32 ? 4 : 2;
  const int t = (inv_ld(max_np) / rpt + 63) / 64 * 64;
  return t < 64 ? 64 : t;
}

void k_patch_apply_f64(hipStream_t st, int64_t npatch, int max_np, const int64_t* poff, const int32_t* pdof, const int32_t* tpos,
                       const int64_t* ioff, const double* inv, const double* r, double* y) {
  if (npatch == 0) return;
  hipLaunchKernelGGL((dev::patch_apply_kernel<double, 2>), dim3(npatch), dim3(patch_apply_threads(max_np, false)),
                     size_t(max_np) * sizeof(double), st, npatch, poff, pdof, tpos, ioff, inv, r, y);
}
void k_patch_apply_f32(hipStream_t st, int64_t npatch, int max_np, const int64_t* poff, const int32_t* pdof, const int32_t* tpos,
                       const int64_t* ioff, const float* inv, const double* r, double* y) {
  if (npatch == 0) return;
  hipLaunchKernelGGL((dev::patch_apply_kernel<float, 4>), dim3(npatch), dim3(patch_apply_threads(max_np, true)),
                     size_t(max_np) * sizeof(float), st, npatch, poff, pdof, tpos, ioff, inv, r, y);
}

void k_patch_extract_spatial_t(hipStream_t st, int64_t p0, int64_t count, int nt, int max_ns, const int64_t* poff,
                               const int32_t* pdof, const int64_t* mptr, const int32_t* mcol, const double* mval,
                               const int64_t* kptr, const int32_t* kcol, const double* kval, double* wmm,
                               double* wkk) {
  if (count == 0) return;
  hipLaunchKernelGGL(dev::patch_extract_spatial_t_kernel, dim3(count), dim3(256), size_t(max_ns) * sizeof(int32_t),
                     st, p0, nt, max_ns, poff, pdof, mptr, mcol, mval, kptr, kcol, kval, wmm, wkk);
}

void k_form_time_blocks(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int max_ns, const int32_t* ns_of,
                        const double* wmm, const double* wkk, const GjDesc* desc, double* W) {
  if (count == 0) return;
  const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(16, (int64_t(max_ns) * max_ns + 255) / 256));
  hipLaunchKernelGGL(dev::form_time_blocks_kernel, dim3(count * tb.nblk, gx), dim3(256), 0, st, tb, max_ns, ns_of,
                     wmm, wkk, desc, W);
}

// r_P (n_P values), the transformed right-hand sides (2 * ldh per kept eigenvalue) and W
// partial block images (2 * ldh per kept eigenvalue each), ldh = inv_ld(n_P / nt).
static size_t tb_lds(int max_np, int nt, int nblk, int W) {
  const int ldh = inv_ld(max_np / nt);
  return (size_t(max_np) + 2 * size_t(nblk) * ldh * (1 + W)) * sizeof(double);
}

int patch_apply_tb_threads(int max_ns, bool fp32) {
  const int rpt = fp32 ? 4 : 2;
  const int t = (inv_ld(max_ns) / rpt + 63) / 64 * 64;
  return t < 64 ? 64 : t;
}

// tuning: STGMG_TB_WAVES (1 or 2 column ranges per patch), STGMG_TB_NT (1: streaming loads)
static void tb_variant(int* W, bool* ntl) {
  *W = 1;       // measured on the 256^2 dG(2) workload: a second wave per patch does not help,
  *ntl = true;  // streaming loads do (+9% FP64, +6% FP32)
  if (const char* e = std::getenv("STGMG_TB_WAVES")) *W = std::atoi(e) == 2 ? 2 : 1;
  if (const char* e = std::getenv("STGMG_TB_NT")) *ntl = std::atoi(e) != 0;
}

template <typename T>
static void launch_tb(hipStream_t st, int64_t npatch, int max_np, const TimeBlockConsts& tb, const int64_t* poff,
                      const int32_t* pdof, const int32_t* tpos, const int64_t* ioff, const T* inv, const double* r, double* y) {
  if (npatch == 0) return;
  int W;
  bool ntl;
  tb_variant(&W, &ntl);
  const int th = patch_apply_tb_threads(max_np / tb.nt, sizeof(T) == 4) * W;
  const size_t lds = tb_lds(max_np, tb.nt, tb.nblk, W);
#define STGMG_TB(WW, NN)                                                                                      \
  hipLaunchKernelGGL((dev::patch_apply_tb_kernel<T, WW, NN>), dim3(npatch), dim3(th), lds, st, tb, poff, pdof, tpos, \
                     ioff, inv, r, y)
  if (W == 1 && !ntl) STGMG_TB(1, false);
  else if (W == 1) STGMG_TB(1, true);
  else if (!ntl) STGMG_TB(2, false);
  else STGMG_TB(2, true);
#undef STGMG_TB
}

void k_patch_apply_tb_f64(hipStream_t st, int64_t npatch, int max_np, const TimeBlockConsts& tb, const int64_t* poff,
                          const int32_t* pdof, const int32_t* tpos, const int64_t* ioff, const double* inv, const double* r, double* y) {
  launch_tb<double>(st, npatch, max_np, tb, poff, pdof, tpos, ioff, inv, r, y);
}
void k_patch_apply_tb_f32(hipStream_t st, int64_t npatch, int max_np, const TimeBlockConsts& tb, const int64_t* poff,
                          const int32_t* pdof, const int32_t* tpos, const int64_t* ioff, const float* inv, const double* r, double* y) {
  launch_tb<float>(st, npatch, max_np, tb, poff, pdof, tpos, ioff, inv, r, y);
}

// Reduced time-block solves: LDS regions A = max(n_P, 2 nblk (nU + ldr)) and
// B = max(2 nblk ns, W 2 nblk ldr) doubles (bounds from the maxima over the patches).
static size_t red_lds(int max_np, int max_nu, int max_nr, int nt, int nblk, int npl, int W) {
  const size_t ldr = inv_ld(max_nr), ns = max_np / nt;
  const size_t a = std::max<size_t>(max_np, size_t(npl) * (max_nu + ldr));
  const size_t b = std::max<size_t>(2 * size_t(nblk) * ns, size_t(W) * npl * ldr);
  return (a + b) * sizeof(double);
}

// Rows per thread R (one 16-byte load per column for FP64 R = 2 / FP32 R = 4), threads per
// column range = ceil(inv_ld(max_nr) / R), blocks of whole waves holding W >= 1 such ranges.
static void red_layout(int max_nr, int R, int* th, int* W) {
  const int per_w = (inv_ld(max_nr) + R - 1) / R;
  *th = std::max(64, (per_w + 63) / 64 * 64);
  if (const char* e = std::getenv("STGMG_RED_WAVES")) {  // tuning: waves per block
    const int v = std::atoi(e);
    if (v >= 1 && v <= 8 && 64 * v >= *th) *th = 64 * v;
  }
  *W = std::max(1, *th / per_w);
  if (const char* e = std::getenv("STGMG_RED_RANGES")) {  // tuning: column ranges per block
    const int v = std::atoi(e);
    if (v >= 1 && v <= *W) *W = v;
  }
}

// rows per thread of the reduced patch GEMV: two for FP64 (16-byte loads); for FP32 two
// (8-byte loads) on short columns and four (16-byte loads) on columns of more than 64
// values.  Measured per finest-level launch: 256^2 dG(2) vertex patches (Schur blocks of 59
// rows) 0.834 ms with two against 0.884 ms with four; 32^3 dG(1) cell patches (89 rows)
// 0.616 ms with two against 0.560 ms with four; 32^3 dG(1) vertex patches (402 rows)
// 11.06 ms with two against 10.30 ms with four.  STGMG_RED_R=2|4 overrides for FP32.
static int red_rows(bool fp32, int max_nr) {
  if (!fp32) return 2;
  if (const char* e = std::getenv("STGMG_RED_R")) {
    const int v = std::atoi(e);
    if (v == 2 || v == 4) return v;
  }
  return inv_ld(max_nr) > 64 ? 4 : 2;
}

int patch_apply_red_threads(int max_nr, bool fp32) {
  int th, W;
  red_layout(max_nr, red_rows(fp32, max_nr), &th, &W);
  return th;
}

// levels with fewer patches than this run the tiled solve with 4 waves per patch (256^2 dG(2)
// solves/s with the threshold at 0 / 256 / 1,024 / 4,096 / 8,192 / 20,000 patches: 18.0 / 18.1 /
// 18.3 / 18.4 / 18.1 / 17.2; the 64^2 level's 4,225 patches run faster with one wave each);
// larger Schur blocks (more tiles per patch) keep 4 waves up to twice as many patches (122 and
// 402 rows: 2-3% faster with 8,192 than with 4,096)
constexpr int64_t SYM_MULTI_BELOW = 4096;
constexpr int SYM_LARGE_NR = 96;

int red_sym_waves(int waves, int64_t npatch, int max_nr) {
  if (waves == 1 || waves == 2 || waves == 4) return waves;
  int64_t multi = max_nr > SYM_LARGE_NR ? 2 * SYM_MULTI_BELOW : SYM_MULTI_BELOW;
  if (const char* e = std::getenv("STGMG_SYM_MULTI_BELOW")) multi = std::atoll(e);  // tuning
  return npatch < multi ? 4 : 1;
}

int node_op_lanes(const NodeOpDev& o) { return o.lanes > 0 ? o.lanes : (o.d == 2 ? 4 : 8); }

// tuning: STGMG_RED_NT (0: ordinary loads instead of streaming loads), STGMG_XCD_CHUNK
template <typename T>
static void launch_red(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym, int waves,
                       const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof, const int32_t* tpos,
                       const int32_t* pnu, const int64_t* ioff, const T* inv, const double* r, double* y) {
  if (npatch == 0) return;
  const int rr = red_rows(sizeof(T) == 4, max_nr);
  int th, W;
  red_layout(max_nr, rr, &th, &W);
  const int npl = dev::red_npl(tb);
  size_t lds = red_lds(max_np, max_nu, max_nr, tb.nt, tb.nblk, npl, W);
  if (sym) {  // W waves per patch; region B holds W partial products and D1 z at stride 8 ceil(nr / 8)
    W = red_sym_waves(waves, npatch, max_nr);
    th = 64 * W;
    const size_t ldr = inv_ld(max_nr), ns = max_np / tb.nt, ldt = 8 * ((max_nr + 7) / 8);
    const size_t a = std::max<size_t>(max_np, size_t(npl) * (max_nu + ldr));
    const size_t b = std::max<size_t>(2 * size_t(tb.nblk) * ns, size_t(W + 1) * npl * ldt);
    lds = (a + b) * sizeof(double);
  }
  bool ntl = true;
  if (const char* e = std::getenv("STGMG_RED_NT")) ntl = std::atoi(e) != 0;
  // chunks of 16 patches per XCD: measured best of {off, 16, 64, 256, 1024, contiguous} on the
  // 256^2 dG(2) workload (the dof-major image writes of neighbouring patches share lines)
  int xc = 16;
  if (const char* e = std::getenv("STGMG_XCD_CHUNK")) xc = std::atoi(e);  // tuning: 0 = round-robin
#define STGMG_RED(RR, NT)                                                                                       \
  hipLaunchKernelGGL((dev::patch_apply_red_kernel<T, RR, NT>), dim3(npatch), dim3(th), lds, st, tb, d, W, xc, poff, \
                     pdof, tpos, pnu, ioff, inv, r, y)
  if (sym) {
#define STGMG_SYM(NT, NW)                                                                                           \
  hipLaunchKernelGGL((dev::patch_apply_red_sym_kernel<T, NT, NW>), dim3(npatch), dim3(64 * NW), lds, st, tb, d, xc, \
                     poff, pdof, tpos, pnu, ioff, inv, r, y)
    if (W == 4) {
      if (ntl) STGMG_SYM(true, 4);
      else STGMG_SYM(false, 4);
    } else if (W == 2) {
      if (ntl) STGMG_SYM(true, 2);
      else STGMG_SYM(false, 2);
    } else {
      if (ntl) STGMG_SYM(true, 1);
      else STGMG_SYM(false, 1);
    }
#undef STGMG_SYM
    return;
  }
  if constexpr (sizeof(T) == 2) {
    return;  // BF16 storage uses the symmetric tiles only (the setup makes sure of it)
  } else {
    if constexpr (sizeof(T) == 4) {
      if (rr == 4) {
        if (ntl) STGMG_RED(4, true);
        else STGMG_RED(4, false);
        return;
      }
    }
    if (ntl) STGMG_RED(2, true);
    else STGMG_RED(2, false);
  }
#undef STGMG_RED
}

void k_patch_apply_red_f64(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym,
                           int waves, const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof,
                           const int32_t* tpos, const int32_t* pnu, const int64_t* ioff, const double* inv,
                           const double* r, double* y) {
  launch_red<double>(st, npatch, max_np, max_nu, max_nr, sym, waves, tb, d, poff, pdof, tpos, pnu, ioff, inv, r, y);
}
void k_patch_apply_red_f32(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym,
                           int waves, const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof,
                           const int32_t* tpos, const int32_t* pnu, const int64_t* ioff, const float* inv,
                           const double* r, double* y) {
  launch_red<float>(st, npatch, max_np, max_nu, max_nr, sym, waves, tb, d, poff, pdof, tpos, pnu, ioff, inv, r, y);
}
void k_patch_apply_red_bf16(hipStream_t st, int64_t npatch, int max_np, int max_nu, int max_nr, bool sym,
                            int waves, const TimeBlockConsts& tb, int d, const int64_t* poff, const int32_t* pdof,
                            const int32_t* tpos, const int32_t* pnu, const int64_t* ioff, const __bf16* inv,
                            const double* r, double* y) {
  launch_red<__bf16>(st, npatch, max_np, max_nu, max_nr, sym, waves, tb, d, poff, pdof, tpos, pnu, ioff, inv, r, y);
}

void k_pack_red_sym_f64(hipStream_t st, int64_t count, const TimeBlockConsts& tb, const int32_t* nu_of,
                        const int32_t* nr_of, const int64_t* soff, const int64_t* toff, const double* sq, double* out) {
  if (count == 0) return;
  hipLaunchKernelGGL(dev::pack_red_sym_kernel<double>, dim3(count * tb.nblk), dim3(256), 0, st, tb, nu_of, nr_of, soff,
                     toff, sq, out);
}
void k_pack_red_sym_f32(hipStream_t st, int64_t count, const TimeBlockConsts& tb, const int32_t* nu_of,
                        const int32_t* nr_of, const int64_t* soff, const int64_t* toff, const double* sq, float* out) {
  if (count == 0) return;
  hipLaunchKernelGGL(dev::pack_red_sym_kernel<float>, dim3(count * tb.nblk), dim3(256), 0, st, tb, nu_of, nr_of, soff,
                     toff, sq, out);
}
void k_pack_red_sym_bf16(hipStream_t st, int64_t count, const TimeBlockConsts& tb, const int32_t* nu_of,
                         const int32_t* nr_of, const int64_t* soff, const int64_t* toff, const double* sq, __bf16* out) {
  if (count == 0) return;
  hipLaunchKernelGGL(dev::pack_red_sym_kernel<__bf16>, dim3(count * tb.nblk), dim3(256), 0, st, tb, nu_of, nr_of, soff,
                     toff, sq, out);
}

template <typename T>
static void launch_fold(hipStream_t st, int64_t count, int d, int max_nu, int max_np_sp, const int32_t* ns_of,
                        const int32_t* nu_of, const GjDesc* desc, int dstride, T* out) {
  if (count == 0) return;
  const size_t lds = size_t(max_nu) * inv_ld(max_np_sp) * sizeof(double);
  hipLaunchKernelGGL(dev::fold_reduced_kernel<T>, dim3(count), dim3(256), lds, st, d, ns_of, nu_of, desc, dstride,
                     out);
}
void k_fold_reduced_f64(hipStream_t st, int64_t count, int d, int max_nu, int max_npr, const int32_t* ns_of,
                        const int32_t* nu_of, const GjDesc* desc, int dstride, double* out) {
  launch_fold<double>(st, count, d, max_nu, max_npr, ns_of, nu_of, desc, dstride, out);
}
void k_fold_reduced_f32(hipStream_t st, int64_t count, int d, int max_nu, int max_npr, const int32_t* ns_of,
                        const int32_t* nu_of, const GjDesc* desc, int dstride, float* out) {
  launch_fold<float>(st, count, d, max_nu, max_npr, ns_of, nu_of, desc, dstride, out);
}
void k_fold_reduced_bf16(hipStream_t st, int64_t count, int d, int max_nu, int max_npr, const int32_t* ns_of,
                         const int32_t* nu_of, const GjDesc* desc, int dstride, __bf16* out) {
  launch_fold<__bf16>(st, count, d, max_nu, max_npr, ns_of, nu_of, desc, dstride, out);
}

size_t gj_lds_kernel_bytes(int max_n, bool cplx) {
  const size_t nn = size_t(max_n) * max_n;
  return ((cplx ? 2 : 1) * (nn + max_n) + max_n) * sizeof(double) + 2 * size_t(max_n) * sizeof(int);
}

template <typename T>
static void gj_lds_launch(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                          T* out, int32_t* status) {
  if (count == 0) return;
  const size_t lds = gj_lds_kernel_bytes(max_n, cplx);
  if (cplx) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::gj_lds_kernel<T, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL((dev::gj_lds_kernel<T, true>), dim3(count), dim3(256), lds, st, desc, W, out, status);
  } else {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dev::gj_lds_kernel<T, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, int(lds));
    hipLaunchKernelGGL((dev::gj_lds_kernel<T, false>), dim3(count), dim3(256), lds, st, desc, W, out, status);
  }
}
void k_gj_lds_f64(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                  double* out, int32_t* status) {
  gj_lds_launch<double>(st, cplx, count, max_n, desc, W, out, status);
}
void k_gj_lds_f32(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                  float* out, int32_t* status) {
  gj_lds_launch<float>(st, cplx, count, max_n, desc, W, out, status);
}
void k_gj_lds_bf16(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, const double* W,
                   __bf16* out, int32_t* status) {
  gj_lds_launch<__bf16>(st, cplx, count, max_n, desc, W, out, status);
}

void k_form_reduced_blocks_f64(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int d, int cplanes, int max_ns,
                               int max_nr, const int32_t* ns_of, const int32_t* nu_of, const double* wmm,
                               const double* wkk, const GjDesc* desc, double* W, double* out) {
  if (count == 0) return;
  const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(16, (4 * int64_t(max_nr) * max_nr + 255) / 256));
  hipLaunchKernelGGL(dev::form_reduced_blocks_kernel<double>, dim3(count * (tb.nblk + 2), gx), dim3(256), 0, st, tb,
                     d, cplanes, max_ns, ns_of, nu_of, wmm, wkk, desc, W, out);
}
void k_form_reduced_blocks_f32(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int d, int cplanes, int max_ns,
                               int max_nr, const int32_t* ns_of, const int32_t* nu_of, const double* wmm,
                               const double* wkk, const GjDesc* desc, double* W, float* out) {
  if (count == 0) return;
  const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(16, (4 * int64_t(max_nr) * max_nr + 255) / 256));
  hipLaunchKernelGGL(dev::form_reduced_blocks_kernel<float>, dim3(count * (tb.nblk + 2), gx), dim3(256), 0, st, tb, d,
                     cplanes, max_ns, ns_of, nu_of, wmm, wkk, desc, W, out);
}
void k_form_reduced_blocks_bf16(hipStream_t st, int64_t count, const TimeBlockConsts& tb, int d, int cplanes,
                                int max_ns, int max_nr, const int32_t* ns_of, const int32_t* nu_of, const double* wmm,
                                const double* wkk, const GjDesc* desc, double* W, __bf16* out) {
  if (count == 0) return;
  const int64_t gx = std::max<int64_t>(1, std::min<int64_t>(16, (4 * int64_t(max_nr) * max_nr + 255) / 256));
  hipLaunchKernelGGL(dev::form_reduced_blocks_kernel<__bf16>, dim3(count * (tb.nblk + 2), gx), dim3(256), 0, st, tb,
                     d, cplanes, max_ns, ns_of, nu_of, wmm, wkk, desc, W, out);
}

void k_vanka_update(hipStream_t st, int64_t n, const int64_t* tptr, const double* winv, const double* y, double* d,
                    bool assign) {
  if (n == 0) return;
  if (assign)
    hipLaunchKernelGGL(dev::vanka_update_kernel<true>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, tptr, winv, y, d);
  else
    hipLaunchKernelGGL(dev::vanka_update_kernel<false>, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, tptr, winv, y,
                       d);
}

int dense_gemv_chunks(int n) { return (n + dev::GEMV_COLS - 1) / dev::GEMV_COLS; }

void k_dense_gemv_t(hipStream_t st, int n, const double* Xt, const double* b, double* part, double* y) {
  const int nc = dense_gemv_chunks(n);
  hipLaunchKernelGGL(dev::dense_gemv_part_kernel, dim3(blocks_for(n, 256), nc), dim3(256), 0, st, n, Xt, b, part);
  hipLaunchKernelGGL(dev::dense_gemv_reduce_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, nc, part, y);
}

void k_gj_large_rowscale(hipStream_t st, int n, double* M, double* scl) {
  hipLaunchKernelGGL(dev::gj_large_rowscale_kernel, dim3(blocks_for(n, 16)), dim3(1024), 0, st, n, M, scl);
}
void k_gj_large_step(hipStream_t st, int n, int k0, int nb, double* M, int* perm, double* P0, double* P1,
                     double* Wb, int32_t* status) {
  const dim3 cgrid(blocks_for(n, 256), nb);
  hipLaunchKernelGGL(dev::gj_large_panel_copy_kernel, cgrid, dim3(256), 0, st, n, k0, nb, M, P0, 1);
  double* pin = P0;
  double* pout = P1;
  for (int c = 0; c < nb; ++c) {
    hipLaunchKernelGGL(dev::gj_large_column_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, k0, c, nb, pin,
                       pout, perm, status);
    std::swap(pin, pout);
  }
  hipLaunchKernelGGL(dev::gj_large_swap_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, k0, nb, M, perm, Wb);
  hipLaunchKernelGGL(dev::gj_large_update_kernel, dim3(blocks_for(n, 256), blocks_for(n, dev::GJL_ROWS)), dim3(256),
                     0, st, n, k0, nb, M, pin, Wb);
  hipLaunchKernelGGL(dev::gj_large_panel_copy_kernel, cgrid, dim3(256), 0, st, n, k0, nb, M, pin, 0);
}
void k_gj_large_output(hipStream_t st, int n, const double* M, const int* src, const double* scl, double* out) {
  hipLaunchKernelGGL(dev::gj_large_output_kernel, dim3(blocks_for(inv_ld(n), 256), n), dim3(256), 0, st, n, M, src,
                     scl, out);
}

int dot_blocks(int64_t n) {
  int64_t b = (n + 8191) / 8192;
  if (b < 1) b = 1;
  if (b > 1024) b = 1024;
  return int(b);
}

void k_multi_dot(hipStream_t st, const double* V, int64_t ldv, int m, const double* w, int64_t n, double* partials,
                 double* out, int accumulate) {
  const int nblk = dot_blocks(n);
  const int64_t chunk = (n + nblk - 1) / nblk;
  hipLaunchKernelGGL(dev::dot_partials_kernel, dim3(nblk, m), dim3(256), 0, st, V, ldv, w, n, chunk, partials);
  hipLaunchKernelGGL(dev::reduce_partials_kernel, dim3(m), dim3(256), 0, st, partials, nblk, out, accumulate);
}

void k_multi_axpy(hipStream_t st, const double* V, int64_t ldv, int m, const double* h, double sign, double* w,
                  int64_t n) {
  if (n == 0 || m == 0) return;
  hipLaunchKernelGGL(dev::multi_axpy_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, V, ldv, m, h, sign, w, n);
}

void k_scale_copy(hipStream_t st, const double* src, const double* nrm2, double* dst, int64_t n) {
  hipLaunchKernelGGL(dev::scale_copy_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, src, nrm2, dst, n);
}

void k_axpby(hipStream_t st, double a, const double* x, double b, const double* y, double* out, int64_t n) {
  if (n == 0) return;
  hipLaunchKernelGGL(dev::axpby_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, st, a, x, b, y, out, n);
}

void k_slab_rhs(hipStream_t st, int nt, int64_t ns, const double* e, const double* mmx, const double* src,
                double* rhs) {
  hipLaunchKernelGGL(dev::slab_rhs_kernel, dim3(blocks_for(int64_t(nt) * ns, 256)), dim3(256), 0, st, nt, ns, e, mmx,
                     src, rhs);
}

}  // namespace stgmg
