// Source vector of the built-in prescribed solution on one level (device assembly of the
// time-node source S(t) of the slab right-hand side, Def:LG).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace stgmg {
namespace dev {

// f (d components) and g of the built-in solution u_i = S sin t, p = S cos t, S = prod sin(pi x_j)
__device__ inline void builtin_fg(const SourceArgs& a, const double* x, double K, double* f, double* g) {
  const double pi = 3.14159265358979323846;
  double sn[3] = {1, 1, 1}, cs[3] = {0, 0, 0};
  for (int ax = 0; ax < a.d; ++ax) {
    sn[ax] = sin(pi * x[ax]);
    cs[ax] = cos(pi * x[ax]);
  }
  double S = 1.0, dS[3];
  for (int ax = 0; ax < a.d; ++ax) S *= sn[ax];
  const double st = sin(a.t), ct = cos(a.t);
  double divS = 0.0;
  for (int i = 0; i < a.d; ++i) {
    dS[i] = pi * cs[i];
    for (int j = 0; j < a.d; ++j)
      if (j != i) dS[i] *= sn[j];
    divS += dS[i];
  }
  for (int i = 0; i < a.d; ++i) {
    double sum = 0.0;  // sum_c d_i d_c S
    for (int c = 0; c < a.d; ++c) {
      if (c == i) {
        sum += -pi * pi * S;
      } else {
        double v = pi * pi * cs[i] * cs[c];
        for (int l = 0; l < a.d; ++l)
          if (l != i && l != c) v *= sn[l];
        sum += v;
      }
    }
    f[i] = (-a.rho * S + a.mu * a.d * pi * pi * S - (a.mu + a.lam) * sum) * st + a.alpha * dS[i] * ct;
  }
  *g = -a.c0 * S * st + a.alpha * divS * ct + K * a.d * pi * pi * S * ct;
}

// one thread per Q_r node (v-equation rows, all components) or pressure function (p-equation
// rows: a Q_{r-1} node, or one broken P_{r-1} function of one cell)
__global__ void source_kernel(SourceArgs a, const double* __restrict__ xq, const double* __restrict__ wq,
                              const double* __restrict__ bq, const double* __restrict__ bp,
                              const double* __restrict__ Kcell, double* __restrict__ out) {
  if (a.tdev) a.t = a.tdev[a.tidx];  // a time set on the device (replays of a captured graph)
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t nQ = a.nv / a.d, nP = a.ns - 2 * a.nv;
  if (t >= nQ + nP) return;
  const bool isP = t >= nQ;
  if (isP && a.disc) {
    // broken pressure: function j of one cell, integrated over that cell
    const int64_t jj = t - nQ, cell = jj / a.nlp;
    const int s = int(jj % a.nlp);
    int cc[3] = {0, 0, 0};
    int64_t rem = cell;
    for (int ax = 0; ax < a.d; ++ax) {
      cc[ax] = int(rem % a.N);
      rem /= a.N;
    }
    const double K = Kcell[cell];
    const double vol = a.d == 2 ? a.h * a.h : a.h * a.h * a.h;
    const double* bt = bp + int64_t(s) * a.nq;
    double accg = 0.0;
    for (int q = 0; q < a.nq; ++q) {
      double x[3];
      for (int ax = 0; ax < a.d; ++ax) x[ax] = (cc[ax] + xq[3 * q + ax]) * a.h;
      double f[3], gg;
      builtin_fg(a, x, K, f, &gg);
      accg += wq[q] * vol * bt[q] * gg;
    }
    out[2 * a.nv + jj] = a.scale * accg;
    return;
  }
  const int p = isP ? a.r - 1 : a.r;
  const int64_t node = isP ? t - nQ : t;
  const int64_t n1 = isP ? a.n1p : a.n1;
  int64_t g[3] = {0, 0, 0};
  int64_t rem = node;
  for (int ax = 0; ax < a.d; ++ax) {
    g[ax] = rem % n1;
    rem /= n1;
  }
  int cl[3][2], ll[3][2], cn[3] = {1, 1, 1};
  for (int ax = 0; ax < a.d; ++ax) {
    cn[ax] = 0;
    if (g[ax] % p == 0) {
      const int64_t c = g[ax] / p;
      if (c - 1 >= 0) {
        cl[ax][cn[ax]] = int(c - 1);
        ll[ax][cn[ax]++] = p;
      }
      if (c < a.N) {
        cl[ax][cn[ax]] = int(c);
        ll[ax][cn[ax]++] = 0;
      }
    } else {
      cl[ax][0] = int(g[ax] / p);
      ll[ax][0] = int(g[ax] % p);
      cn[ax] = 1;
    }
  }
  int combos = 1;
  for (int ax = 0; ax < a.d; ++ax) combos *= cn[ax];
  double acc[3] = {0, 0, 0}, accg = 0.0;
  const double vol = a.d == 2 ? a.h * a.h : a.h * a.h * a.h;
  for (int cb = 0; cb < combos; ++cb) {
    int cc[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, tt = cb;
    for (int ax = 0; ax < a.d; ++ax) {
      cc[ax] = cl[ax][tt % cn[ax]];
      lo[ax] = ll[ax][tt % cn[ax]];
      tt /= cn[ax];
    }
    int loc = 0;
    for (int ax = a.d - 1; ax >= 0; --ax) loc = loc * (p + 1) + lo[ax];
    int64_t cell = 0;
    for (int ax = a.d - 1; ax >= 0; --ax) cell = cell * a.N + cc[ax];
    const double K = Kcell[cell];
    const double* bt = (isP ? bp : bq) + int64_t(loc) * a.nq;
    for (int q = 0; q < a.nq; ++q) {
      double x[3];
      for (int ax = 0; ax < a.d; ++ax) x[ax] = (cc[ax] + xq[3 * q + ax]) * a.h;
      double f[3], gg;
      builtin_fg(a, x, K, f, &gg);
      const double w = wq[q] * vol * bt[q];
      if (isP) {
        accg += w * gg;
      } else {
        for (int c = 0; c < a.d; ++c) acc[c] += w * f[c];
      }
    }
  }
  if (isP) {
    out[2 * a.nv + node] = a.scale * accg;
  } else {
    for (int c = 0; c < a.d; ++c) {
      out[a.nv + a.d * node + c] = a.scale * acc[c];
      out[a.d * node + c] = 0.0;
    }
  }
}

}  // namespace dev

static inline int64_t blocks_for(int64_t n, int bs) { return (n + bs - 1) / bs; }

void k_source(hipStream_t st, const SourceArgs& a, const double* xq, const double* wq, const double* bq,
              const double* bp, const double* Kcell, double* out) {
  const int64_t nthreads = a.nv / a.d + (a.ns - 2 * a.nv);
  hipLaunchKernelGGL(dev::source_kernel, dim3(blocks_for(nthreads, 256)), dim3(256), 0, st, a, xq, wq, bq, bp, Kcell,
                     out);
}

}  // namespace stgmg
