// Batched Gauss-Jordan inversion of the larger patch blocks (above 64 Schur rows, in particular
// those that do not fit in LDS), with the rank-16 updates of the trailing matrix on the matrix
// cores (v_mfma_f64_16x16x4f64).
//
// The operation is the exact inverse of each local block (the patch solve of Def. 4.2 and the
// local operator of Alg. 4.1, inverted once at setup).  One workgroup inverts one matrix, held in
// global memory; per panel of 16 columns:
//   1. the panel (n x 16, complex: two planes) is loaded into LDS and eliminated column by column
//      with partial pivoting (the largest scaled entry, |re| + |im| for complex blocks, ties to the
//      lowest row, searched with wavefront shuffles), as in the workgroup kernels in kernels.hip;
//   2. the panel's row swaps are applied to the other columns, one 16-column tile per wavefront;
//   3. those columns get the rank-16 update  M[:, J] = [i not in panel rows] M[:, J] + Pnl W,
//      W = the panel's (swapped) pivot rows of M[:, J]: a 16 x 16 output tile per MFMA chain,
//      four k-steps of 4 (complex: four real products per k-step);
//   4. the eliminated panel is written back.
// Inputs and outputs follow the conventions of the workgroup kernels: power-of-two row
// equilibration before the elimination, the inverse of the scaled matrix re-scaled by columns and
// un-permuted on output, rows i < keep written with ld_out per row (complex: Re of column j at j,
// Im at ldh + j).  A zero or non-finite pivot sets status[patch] = 1 (the step then uses 1).
//
// Lane layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[l / 16 + 4 r][l % 16] in accumulator element r.
#include <hip/hip_runtime.h>
#include <cstdint>
#include "kernels.h"

namespace stgmg {
namespace dev {
namespace {

constexpr int MW = 64;        // wavefront
constexpr int GB = 16;        // panel width (the MFMA tile)
constexpr int PS = GB + 1;    // LDS row stride of the panel (odd: the A-operand rows fall on distinct banks)
constexpr int GT = 512;       // threads per workgroup
typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma(double a, double b, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

template <typename T, bool CPLX>
__global__ void __launch_bounds__(GT) gj_mfma_kernel(const GjDesc* __restrict__ desc, double* __restrict__ W,
                                                     T* __restrict__ out, int32_t* __restrict__ status) {
  extern __shared__ double lds[];
  const GjDesc D = desc[blockIdx.x];
  const int n = D.n;
  const int64_t nn = int64_t(n) * n;
  double* Mr = W + D.woff;
  double* Mi = CPLX ? Mr + nn : nullptr;
  double* Pr = lds;                                   // n x PS
  double* Pi = CPLX ? lds + n * PS : nullptr;         // n x PS
  double* scl = lds + (CPLX ? 2 : 1) * n * PS;        // n
  double* red_v = scl + n;                            // GT / MW
  int* perm = reinterpret_cast<int*>(red_v + GT / MW);  // n
  int* src = perm + n;                                // n
  int* red_i = src + n;                               // GT / MW
  int* mv = red_i + GT / MW;                          // rows written by the panel's swaps (<= 2 GB)
  int* ms = mv + 2 * GB;                              // the row each takes its values from
  __shared__ int s_piv, s_flag, s_nm;
  const int tid = threadIdx.x, wave = tid / MW, lane = tid % MW, nw = GT / MW;
  if (tid == 0) s_flag = 0;
  // row equilibration by powers of two
  for (int i = wave; i < n; i += nw) {
    double m = 0.0;
    for (int j = lane; j < n; j += MW) {
      m = fmax(m, fabs(Mr[int64_t(i) * n + j]));
      if constexpr (CPLX) m = fmax(m, fabs(Mi[int64_t(i) * n + j]));
    }
    for (int off = MW / 2; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
    const double s = (m > 0.0 && isfinite(m)) ? ldexp(1.0, -ilogb(m)) : 1.0;
    for (int j = lane; j < n; j += MW) {
      Mr[int64_t(i) * n + j] *= s;
      if constexpr (CPLX) Mi[int64_t(i) * n + j] *= s;
    }
    if (lane == 0) scl[i] = s;
  }
  __syncthreads();
  const int ntile = (n + GB - 1) / GB;
  for (int k0 = 0; k0 < n; k0 += GB) {
    const int nb = min(GB, n - k0);
    for (int t = tid; t < n * GB; t += GT) {
      const int i = t / GB, c = t % GB;
      Pr[i * PS + c] = c < nb ? Mr[int64_t(i) * n + k0 + c] : 0.0;
      if constexpr (CPLX) Pi[i * PS + c] = c < nb ? Mi[int64_t(i) * n + k0 + c] : 0.0;
    }
    __syncthreads();
    // 1. the panel, column by column
    for (int c = 0; c < nb; ++c) {
      const int k = k0 + c;
      double bv = -1.0;
      int bi = n;
      for (int i = k + tid; i < n; i += GT) {
        double v = fabs(Pr[i * PS + c]);
        if constexpr (CPLX) v += fabs(Pi[i * PS + c]);
        if (v > bv) {
          bv = v;
          bi = i;
        }
      }
      for (int off = MW / 2; off > 0; off >>= 1) {
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
        s_piv = ii;
      }
      __syncthreads();
      const int p = s_piv;
      // rows k and p swapped and the new pivot row divided by the pivot: lanes 0..15 of wave 0,
      // every value read before any is written
      if (tid < GB) {
        const int cc = tid;
        double pvr = Pr[p * PS + c], pvi = CPLX ? Pi[p * PS + c] : 0.0;
        const double ar = Pr[p * PS + cc], ai = CPLX ? Pi[p * PS + cc] : 0.0;
        const double kr = Pr[k * PS + cc], ki = CPLX ? Pi[k * PS + cc] : 0.0;
        if (!(fabs(pvr) + fabs(pvi) > 0.0) || !isfinite(pvr) || !isfinite(pvi)) {
          pvr = 1.0;
          pvi = 0.0;
        }
        double rr, ri;
        if constexpr (CPLX) {
          const double den = pvr * pvr + pvi * pvi;
          rr = pvr / den;
          ri = -pvi / den;
        } else {
          rr = 1.0 / pvr;
          ri = 0.0;
        }
        const double xr = cc == c ? 1.0 : ar, xi = cc == c ? 0.0 : ai;
        if (p != k) {
          Pr[p * PS + cc] = kr;
          if constexpr (CPLX) Pi[p * PS + cc] = ki;
        }
        Pr[k * PS + cc] = CPLX ? xr * rr - xi * ri : xr * rr;
        if constexpr (CPLX) Pi[k * PS + cc] = xr * ri + xi * rr;
      }
      __syncthreads();
      for (int i = tid; i < n; i += GT) {
        if (i == k) continue;
        const double fr = Pr[i * PS + c], fi = CPLX ? Pi[i * PS + c] : 0.0;
        Pr[i * PS + c] = 0.0;
        if constexpr (CPLX) Pi[i * PS + c] = 0.0;
#pragma unroll
        for (int cc = 0; cc < GB; ++cc) {
          if constexpr (CPLX) {
            const double xr = Pr[k * PS + cc], xi = Pi[k * PS + cc];
            Pr[i * PS + cc] -= fr * xr - fi * xi;
            Pi[i * PS + cc] -= fr * xi + fi * xr;
          } else {
            Pr[i * PS + cc] -= fr * Pr[k * PS + cc];
          }
        }
      }
      __syncthreads();
    }
    // the panel's swaps as one permutation of at most 2 GB rows: new row mv[t] = old row ms[t].
    // Wave 0: lane c < nb holds row k0 + c, lane GB + c the pivot row perm[k0 + c] when it lies
    // below the panel rows (the first lane with that row only); the swaps are replayed in order
    // by exchanging the source rows of the two lanes that hold their rows.
    if (wave == 0) {
      int row = -1;
      if (lane < nb) {
        row = k0 + lane;
      } else if (lane >= GB && lane < GB + nb) {
        const int q = perm[k0 + lane - GB];
        row = q >= k0 + nb ? q : -1;
      }
      for (int o = GB; o < 2 * GB; ++o) {
        const int ro = __shfl(row, o);
        if (lane > o && row == ro) row = -1;
      }
      int from = row;
      for (int c = 0; c < nb; ++c) {
        const int ra = k0 + c, rb = perm[k0 + c];
        if (ra == rb) continue;
        const int la = __ffsll(static_cast<unsigned long long>(__ballot(row == ra))) - 1;
        const int lb = __ffsll(static_cast<unsigned long long>(__ballot(row == rb))) - 1;
        const int fa = __shfl(from, la), fb = __shfl(from, lb);
        if (row == ra) from = fb;
        else if (row == rb) from = fa;
      }
      const unsigned long long live = __ballot(row >= 0);
      if (row >= 0) {
        const int t = __popcll(live & ((1ull << lane) - 1ull));
        mv[t] = row;
        ms[t] = from;
      }
      if (lane == 0) s_nm = __popcll(live);
    }
    __syncthreads();
    const int nm = s_nm;
    // 2. + 3. the other columns, one 16-column tile per wavefront at a time
    const int jp = k0 / GB;
    for (int jt = wave; jt < ntile; jt += nw) {
      if (jt == jp) continue;
      const int j = jt * GB + (lane % 16);
      const bool jok = j < n;
      const int g = lane / 16;
      double sr[2 * GB / 4], si[2 * GB / 4];
#pragma unroll
      for (int q = 0; q < 2 * GB / 4; ++q) {
        const int t = g + 4 * q;
        const bool mvd = jok && t < nm && ms[t] != mv[t];
        sr[q] = mvd ? Mr[int64_t(ms[t]) * n + j] : 0.0;
        if constexpr (CPLX) si[q] = mvd ? Mi[int64_t(ms[t]) * n + j] : 0.0;
      }
#pragma unroll
      for (int q = 0; q < 2 * GB / 4; ++q) {
        const int t = g + 4 * q;
        if (jok && t < nm && ms[t] != mv[t]) {
          Mr[int64_t(mv[t]) * n + j] = sr[q];
          if constexpr (CPLX) Mi[int64_t(mv[t]) * n + j] = si[q];
        }
      }
      __threadfence_block();
      // B operand: the pivot rows of these columns, k-step s holds W[4 s + l / 16][l % 16]
      double br[4], bi[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const int c = 4 * s + g;
        br[s] = jok && c < nb ? Mr[int64_t(k0 + c) * n + j] : 0.0;
        bi[s] = CPLX && jok && c < nb ? Mi[int64_t(k0 + c) * n + j] : 0.0;
      }
      // C tile of row tile it: element r at row 16 it + l / 16 + 4 r; pivot rows start from zero
      auto load_c = [&](int it, d4& cr, d4& ci) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = it * GB + g + 4 * r;
          const bool in = jok && row < n && (row < k0 || row >= k0 + nb);
          cr[r] = in ? Mr[int64_t(row) * n + j] : 0.0;
          if constexpr (CPLX) ci[r] = in ? Mi[int64_t(row) * n + j] : 0.0;
        }
      };
      // two row tiles in flight ahead of the one being updated (rows disjoint from it)
      d4 cr, ci = {0.0, 0.0, 0.0, 0.0}, c1r = {0.0, 0.0, 0.0, 0.0}, c1i = {0.0, 0.0, 0.0, 0.0};
      load_c(0, cr, ci);
      if (ntile > 1) load_c(1, c1r, c1i);
      for (int it = 0; it < ntile; ++it) {
        d4 c2r = {0.0, 0.0, 0.0, 0.0}, c2i = {0.0, 0.0, 0.0, 0.0};
        if (it + 2 < ntile) load_c(it + 2, c2r, c2i);
        const int arow = it * GB + (lane % 16);
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          const int acol = 4 * s + g;
          const double ar = arow < n ? Pr[arow * PS + acol] : 0.0;
          cr = mfma(ar, br[s], cr);
          if constexpr (CPLX) {
            const double ai = arow < n ? Pi[arow * PS + acol] : 0.0;
            cr = mfma(-ai, bi[s], cr);
            ci = mfma(ar, bi[s], ci);
            ci = mfma(ai, br[s], ci);
          }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = it * GB + g + 4 * r;
          if (jok && row < n) {
            Mr[int64_t(row) * n + j] = cr[r];
            if constexpr (CPLX) Mi[int64_t(row) * n + j] = ci[r];
          }
        }
        cr = c1r;
        ci = c1i;
        c1r = c2r;
        c1i = c2i;
      }
    }
    __syncthreads();
    // 4. the eliminated panel back into its columns
    for (int t = tid; t < n * nb; t += GT) {
      const int i = t / nb, c = t % nb;
      Mr[int64_t(i) * n + k0 + c] = Pr[i * PS + c];
      if constexpr (CPLX) Mi[int64_t(i) * n + k0 + c] = Pi[i * PS + c];
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
    for (int q = lane; q < D.ld_out; q += MW) {
      double v = 0.0;
      if (q < n) {
        v = Mr[int64_t(i) * n + src[q]] * scl[q];
      } else if (CPLX && q >= D.ldh && q - D.ldh < n) {
        v = Mi[int64_t(i) * n + src[q - D.ldh]] * scl[q - D.ldh];
      }
      o[int64_t(i) * D.ld_out + q] = T(v);
    }
}

}  // namespace
}  // namespace dev

size_t gj_mfma_bytes(int max_n, bool cplx) {
  return ((cplx ? 2 : 1) * size_t(max_n) * dev::PS + max_n + dev::GT / dev::MW) * sizeof(double) +
         (2 * size_t(max_n) + dev::GT / dev::MW + 4 * dev::GB) * sizeof(int);
}

template <typename T>
static void gj_mfma_launch(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, T* out,
                           int32_t* status) {
  if (count <= 0) return;
  const size_t lds = gj_mfma_bytes(max_n, cplx);
  if (cplx)
    hipLaunchKernelGGL((dev::gj_mfma_kernel<T, true>), dim3(count), dim3(dev::GT), lds, st, desc, W, out, status);
  else
    hipLaunchKernelGGL((dev::gj_mfma_kernel<T, false>), dim3(count), dim3(dev::GT), lds, st, desc, W, out, status);
}

void k_gj_mfma_f64(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, double* out,
                   int32_t* status) {
  gj_mfma_launch<double>(st, cplx, count, max_n, desc, W, out, status);
}
void k_gj_mfma_f32(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, float* out,
                   int32_t* status) {
  gj_mfma_launch<float>(st, cplx, count, max_n, desc, W, out, status);
}
void k_gj_mfma_bf16(hipStream_t st, bool cplx, int64_t count, int max_n, const GjDesc* desc, double* W, __bf16* out,
                    int32_t* status) {
  gj_mfma_launch<__bf16>(st, cplx, count, max_n, desc, W, out, status);
}

}  // namespace stgmg
