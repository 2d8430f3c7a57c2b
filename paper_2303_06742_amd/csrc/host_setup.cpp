// Host construction of the slab operators, patch tables and transfers.
//
// Discretisation (paper Sec. 2-4): dG(k) in time with the Lagrange basis at the
// right Gauss-Radau points (Eq:GF, Eq:TimeExp), Taylor-Hood Q_r^d / Q_{r-1} or
// Q_r^d / P_{r-1}^disc with the symmetric interior penalty form of Def:B in
// space on axis-parallel square/cube cells (Def:VhQh), Nitsche boundary terms
// (Def:ACB, Def:ab) with gamma_a = 5e4 r(r+1), gamma_b = r(r-1)/2 and
// h_F = |K|_d on boundary faces.  The slab matrix of Problem 4.1 (v-form of
// Problem 3.1) is
//     A_n = D^t (x) MM + M^t (x) KK,
//     MM = [[0, Mrho, 0], [Mrho, 0, 0], [0, 0, c0 Mp]],
//     KK = [[-Mrho, 0, 0], [0, A_gamma, C^T], [-C, 0, B_gamma]]
// with rows (u-eq, v-eq, p-eq) and columns (V, U, P).
#include "host_setup.h"
#include "tile_layout.h"

#include <algorithm>
#include <atomic>
#include <array>
#include <cmath>
#include <functional>
#include <stdexcept>
#include <thread>

namespace stgmg {

std::vector<std::array<int, 3>> pdisc_exponents(int p, int d) {
  std::vector<std::array<int, 3>> out;
  int n = 1;
  for (int a = 0; a < d; ++a) n *= p + 1;
  for (int i = 0; i < n; ++i) {
    std::array<int, 3> e = {0, 0, 0};
    int rem = i, deg = 0;
    for (int ax = 0; ax < d; ++ax) {
      e[ax] = rem % (p + 1);
      rem /= p + 1;
      deg += e[ax];
    }
    if (deg <= p) out.push_back(e);
  }
  return out;
}

namespace {

// ---------------------------------------------------------------- 1D tools
double legendre(int n, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int j = 2; j <= n; ++j) {
    double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Gauss-Legendre points/weights on [0,1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p = legendre(n, z), pm = legendre(n - 1, z);
      double dp = n * (z * p - pm) / (z * z - 1.0);
      double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p = legendre(n, z), pm = legendre(n - 1, z);
    double dp = n * (z * p - pm) / (z * z - 1.0);
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 0.5 * 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Degree-p Lagrange basis on the equispaced nodes j/p of [0,1]: values and derivatives at xi.
void lagrange01(int p, double xi, double* v, double* dv) {
  for (int a = 0; a <= p; ++a) {
    double xa = double(a) / p, val = 1.0, der = 0.0;
    for (int b = 0; b <= p; ++b) {
      if (b == a) continue;
      double xb = double(b) / p;
      // product rule: der = der*(xi-xb)/(xa-xb) + val/(xa-xb)
      der = der * (xi - xb) / (xa - xb) + val / (xa - xb);
      val = val * (xi - xb) / (xa - xb);
    }
    v[a] = val;
    if (dv) dv[a] = der;
  }
}

// Tensor-product basis of Q_p on [0,h]^d at a reference point: values and physical gradients.
struct Tab {
  int nl;
  std::vector<double> v;  // [nl]
  std::vector<double> g;  // [nl][3]
};
void tabulate(int p, int d, const double* xi, double h, Tab& t) {
  int n1 = p + 1;
  t.nl = 1;
  for (int a = 0; a < d; ++a) t.nl *= n1;
  t.v.assign(t.nl, 1.0);
  t.g.assign(size_t(t.nl) * 3, 1.0);
  double v1[3][8], d1[3][8];
  for (int ax = 0; ax < d; ++ax) lagrange01(p, xi[ax], v1[ax], d1[ax]);
  for (int a = 0; a < t.nl; ++a) {
    int idx[3] = {0, 0, 0}, rem = a;
    for (int ax = 0; ax < d; ++ax) {
      idx[ax] = rem % n1;
      rem /= n1;
    }
    for (int ax = 0; ax < d; ++ax) t.v[a] *= v1[ax][idx[ax]];
    for (int g = 0; g < d; ++g)
      for (int ax = 0; ax < d; ++ax)
        t.g[a * 3 + g] *= (g == ax) ? d1[ax][idx[ax]] / h : v1[ax][idx[ax]];
  }
}

// P_p^disc basis (pdisc_exponents) on [0,h]^d at a reference point: values and physical gradients.
void tabulate_pdisc(int p, int d, const double* xi, double h, Tab& t) {
  const auto ex = pdisc_exponents(p, d);
  t.nl = int(ex.size());
  t.v.assign(t.nl, 1.0);
  t.g.assign(size_t(t.nl) * 3, 1.0);
  for (int a = 0; a < t.nl; ++a) {
    for (int ax = 0; ax < d; ++ax) {
      const double z = xi[ax] - 0.5;
      const int e = ex[a][ax];
      const double pw = std::pow(z, e), dpw = e > 0 ? e * std::pow(z, e - 1) / h : 0.0;
      t.v[a] *= pw;
      for (int g = 0; g < d; ++g) t.g[a * 3 + g] *= (g == ax) ? dpw : pw;
    }
  }
}

// pressure basis of the pair: Q_{r-1} or P_{r-1}^disc
void tabulate_p(bool disc, int r, int d, const double* xi, double h, Tab& t) {
  if (disc)
    tabulate_pdisc(r - 1, d, xi, h, t);
  else
    tabulate(r - 1, d, xi, h, t);
}

template <class F>
void parallel_for(int64_t n, int nthreads, F&& f) {
  if (nthreads <= 1 || n < 4096) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nthreads - 1) / nthreads;
  for (int t = 0; t < nthreads; ++t) {
    int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&f, lo, hi] { f(lo, hi); });
  }
  for (auto& x : th) x.join();
}

}  // namespace

// ------------------------------------------------------------- time constants
TimeConsts make_time_consts(int k, double tau) {
  TimeConsts T;
  T.k = k;
  T.tau = tau;
  int n = k + 1;
  // right Radau: roots of P_k - P_{k+1}; x = +1 is one of them.  The interior
  // roots are found by sign changes of (P_k - P_{k+1})/(1-x) and bisection.
  std::vector<double> xs;
  if (k > 0) {
    auto f = [k](double x) { return (legendre(k, x) - legendre(k + 1, x)) / (1.0 - x); };
    const int M = 20000;
    double xl = -1.0, fl = f(xl);
    for (int i = 1; i <= M; ++i) {
      double xr = -1.0 + 2.0 * i / M * (1.0 - 1e-12), fr = f(xr);
      if (fl == 0.0) {
        xs.push_back(xl);
      } else if ((fl < 0) != (fr < 0)) {
        double a = xl, b = xr, fa = fl;
        for (int it = 0; it < 200; ++it) {
          double m = 0.5 * (a + b), fm = f(m);
          if ((fm < 0) == (fa < 0)) {
            a = m;
            fa = fm;
          } else {
            b = m;
          }
        }
        xs.push_back(0.5 * (a + b));
      }
      xl = xr;
      fl = fr;
    }
  }
  if (int(xs.size()) != k) throw std::runtime_error("Gauss-Radau node search failed");
  xs.push_back(1.0);
  T.x = xs;
  T.w.resize(n);
  // weights of the right Radau rule: 2/n^2 at +1, (1 + x_j) / (n^2 P_{n-1}(x_j)^2) inside
  for (int j = 0; j < n; ++j) {
    if (j == n - 1) {
      T.w[j] = 2.0 / (double(n) * n);
    } else {
      double pk = legendre(n - 1, xs[j]);
      T.w[j] = (1.0 + xs[j]) / (double(n) * n * pk * pk);
    }
  }
  auto chi = [&](int a, double t) {
    double v = 1.0;
    for (int b = 0; b < n; ++b)
      if (b != a) v *= (t - xs[b]) / (xs[a] - xs[b]);
    return v;
  };
  auto dchi = [&](int a, double t) {
    double s = 0.0;
    for (int c = 0; c < n; ++c) {
      if (c == a) continue;
      double v = 1.0 / (xs[a] - xs[c]);
      for (int b = 0; b < n; ++b)
        if (b != a && b != c) v *= (t - xs[b]) / (xs[a] - xs[b]);
      s += v;
    }
    return s;
  };
  T.Dt.assign(n * n, 0.0);
  T.e.resize(n);
  T.mt.resize(n);
  for (int b = 0; b < n; ++b) {
    T.e[b] = chi(b, -1.0);
    T.mt[b] = 0.5 * tau * T.w[b];
  }
  // D^t[b][a] = w_b chi_a'(x_b) + chi_a(-1) chi_b(-1)  (the rule is exact, chi_b(x_m) = delta)
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) T.Dt[b * n + a] = T.w[b] * dchi(a, xs[b]) + T.e[a] * T.e[b];
  return T;
}

// ------------------------------------------------------------- time blocks
namespace {
using cd = std::complex<double>;

// x = A^{-1} b for a small complex matrix (Gaussian elimination, partial pivoting)
std::vector<cd> csolve(std::vector<cd> A, std::vector<cd> b, int n) {
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[r * n + c]) > std::abs(A[piv * n + c])) piv = r;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(b[c], b[piv]);
    }
    for (int r = c + 1; r < n; ++r) {
      const cd f = A[r * n + c] / A[c * n + c];
      for (int j = c; j < n; ++j) A[r * n + j] -= f * A[c * n + j];
      b[r] -= f * b[c];
    }
  }
  std::vector<cd> x(n);
  for (int r = n - 1; r >= 0; --r) {
    cd sum = b[r];
    for (int j = r + 1; j < n; ++j) sum -= A[r * n + j] * x[j];
    x[r] = sum / A[r * n + r];
  }
  return x;
}
}  // namespace

TimeBlocks make_time_blocks(const TimeConsts& Tc) {
  const int n = Tc.k + 1;
  TimeBlocks B;
  B.nt = n;
  std::vector<double> T(n * n);
  for (int b = 0; b < n; ++b)
    for (int a = 0; a < n; ++a) T[b * n + a] = Tc.Dt[b * n + a] / Tc.mt[b];
  // characteristic polynomial by Faddeev-LeVerrier: p(x) = x^n + c[n-1] x^{n-1} + ... + c[0]
  std::vector<double> c(n + 1, 0.0), Mk(n * n, 0.0), AM(n * n);
  c[n] = 1.0;
  for (int k = 1; k <= n; ++k) {
    // M_k = A M_{k-1} + c_{n-k+1} I ; c_{n-k} = -tr(A M_k) / k
    std::vector<double> Mn(n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double sum = 0.0;
        for (int l = 0; l < n; ++l) sum += T[i * n + l] * Mk[l * n + j];
        Mn[i * n + j] = sum + (i == j ? c[n - k + 1] : 0.0);
      }
    Mk = Mn;
    double tr = 0.0;
    for (int i = 0; i < n; ++i)
      for (int l = 0; l < n; ++l) tr += T[i * n + l] * Mk[l * n + i];
    c[n - k] = -tr / k;
  }
  auto poly = [&](cd x) {
    cd v = 1.0;
    for (int k = n - 1; k >= 0; --k) v = v * x + c[k];
    return v;
  };
  // Durand-Kerner roots, scaled by the Cauchy bound
  double bound = 0.0;
  for (int k = 0; k < n; ++k) bound = std::max(bound, std::fabs(c[k]));
  bound += 1.0;
  std::vector<cd> z(n);
  for (int i = 0; i < n; ++i) z[i] = bound * std::pow(cd(0.4, 0.9), i);
  for (int it = 0; it < 2000; ++it) {
    double change = 0.0;
    for (int i = 0; i < n; ++i) {
      cd den = 1.0;
      for (int j = 0; j < n; ++j)
        if (j != i) den *= (z[i] - z[j]);
      const cd dz = poly(z[i]) / den;
      z[i] -= dz;
      change = std::max(change, std::abs(dz) / std::max(1.0, std::abs(z[i])));
    }
    if (change < 1e-16) break;
  }
  // eigenvectors by inverse iteration; kept set: real ones and Im > 0 of each pair
  std::vector<cd> Q(n * n);
  std::vector<cd> lam_all(n);
  std::vector<int> order;
  for (int i = 0; i < n; ++i)
    if (std::fabs(z[i].imag()) <= 1e-9 * std::abs(z[i])) z[i] = cd(z[i].real(), 0.0);
  std::vector<int> used(n, 0);
  std::vector<cd> lam_sorted;
  for (int i = 0; i < n; ++i)
    if (z[i].imag() == 0.0) lam_sorted.push_back(z[i]);
  for (int i = 0; i < n; ++i)
    if (z[i].imag() > 0.0) {
      lam_sorted.push_back(z[i]);
      lam_sorted.push_back(std::conj(z[i]));
    }
  if (int(lam_sorted.size()) != n) throw std::runtime_error("time eigenvalues: unpaired complex root");
  for (int a = 0; a < n; ++a) {
    const cd lam = lam_sorted[a];
    const cd shift = lam * (1.0 + 1e-10) + cd(1e-12, 0.0);
    std::vector<cd> M(n * n), v(n, cd(1.0, 0.0));
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) M[i * n + j] = cd(T[i * n + j], 0.0) - (i == j ? shift : cd(0.0, 0.0));
    for (int it = 0; it < 3; ++it) {
      v = csolve(M, v, n);
      double nv = 0.0;
      int imax = 0;
      for (int i = 0; i < n; ++i)
        if (std::abs(v[i]) > nv) {
          nv = std::abs(v[i]);
          imax = i;
        }
      const cd s = v[imax];
      for (auto& x : v) x /= s;  // largest entry = 1 (a real eigenvector stays real)
    }
    if (lam.imag() == 0.0)
      for (auto& x : v) x = cd(x.real(), 0.0);
    for (int i = 0; i < n; ++i) Q[i * n + a] = v[i];
    lam_all[a] = lam;
  }
  // Q^{-1} column by column
  std::vector<cd> Qi(n * n);
  for (int j = 0; j < n; ++j) {
    std::vector<cd> e(n, cd(0.0, 0.0));
    e[j] = 1.0;
    std::vector<cd> col = csolve(Q, e, n);
    for (int i = 0; i < n; ++i) Qi[i * n + j] = col[i];
  }
  for (int a = 0; a < n; ++a) {
    if (lam_all[a].imag() < 0.0) continue;  // partner of the previous kept eigenvalue
    B.lam.push_back(lam_all[a]);
    B.is_complex.push_back(lam_all[a].imag() > 0.0 ? 1 : 0);
    for (int b = 0; b < n; ++b) B.tin.push_back(Qi[a * n + b] / Tc.mt[b]);
  }
  B.nblk = int(B.lam.size());
  B.qout.resize(size_t(n) * B.nblk);
  int kb = 0;
  for (int a = 0; a < n; ++a) {
    if (lam_all[a].imag() < 0.0) continue;
    for (int b = 0; b < n; ++b) B.qout[size_t(b) * B.nblk + kb] = Q[b * n + a];
    ++kb;
  }
  return B;
}

// ------------------------------------------------------------- cell matrices
CellMats make_cell_mats(int d, int r, double h, const Material& m, bool disc) {
  CellMats C;
  C.d = d;
  C.r = r;
  C.disc = disc;
  int ns = 1, np = 1;
  for (int a = 0; a < d; ++a) {
    ns *= (r + 1);
    np *= r;
  }
  if (disc) np = int(pdisc_exponents(r - 1, d).size());
  C.nls = ns;
  C.nlv = d * ns;
  C.nlp = np;
  C.gamma_a = 5e4 * r * (r + 1);
  C.gamma_b = 0.5 * r * (r - 1);
  C.hF = std::pow(h, d);
  const int nv = C.nlv;
  C.Mrho.assign(size_t(nv) * nv, 0.0);
  C.Avol.assign(size_t(nv) * nv, 0.0);
  C.Cvol.assign(size_t(np) * nv, 0.0);
  C.Bvol.assign(size_t(np) * np, 0.0);
  C.Mp.assign(size_t(np) * np, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre01(r + 1, gx, gw);
  const int nq1 = r + 1;
  int nq = 1;
  for (int a = 0; a < d; ++a) nq *= nq1;
  Tab s, p;
  const double mu = m.mu, lam = m.lambda;
  for (int q = 0; q < nq; ++q) {
    double xi[3] = {0, 0, 0}, wq = 1.0;
    int rem = q;
    for (int ax = 0; ax < d; ++ax) {
      xi[ax] = gx[rem % nq1];
      wq *= gw[rem % nq1] * h;
      rem /= nq1;
    }
    tabulate(r, d, xi, h, s);
    tabulate_p(disc, r, d, xi, h, p);
    for (int b = 0; b < ns; ++b)
      for (int a = 0; a < ns; ++a) {
        double mass = wq * s.v[a] * s.v[b];
        double gg = 0.0;
        for (int j = 0; j < d; ++j) gg += s.g[a * 3 + j] * s.g[b * 3 + j];
        for (int e = 0; e < d; ++e) {
          C.Mrho[size_t(d * b + e) * nv + d * a + e] += m.rho * mass;
          for (int c = 0; c < d; ++c) {
            // sigma(phi_a e_c) : eps(phi_b e_e) = mu (delta_ce grad a.grad b + d_e a d_c b) + lam d_c a d_e b
            double val = mu * ((c == e ? gg : 0.0) + s.g[a * 3 + e] * s.g[b * 3 + c]) +
                         lam * s.g[a * 3 + c] * s.g[b * 3 + e];
            C.Avol[size_t(d * b + e) * nv + d * a + c] += wq * val;
          }
        }
      }
    for (int t = 0; t < np; ++t) {
      for (int a = 0; a < ns; ++a)
        for (int c = 0; c < d; ++c) C.Cvol[size_t(t) * nv + d * a + c] += -m.alpha * wq * s.g[a * 3 + c] * p.v[t];
      for (int u = 0; u < np; ++u) {
        double gg = 0.0;
        for (int j = 0; j < d; ++j) gg += p.g[u * 3 + j] * p.g[t * 3 + j];
        C.Bvol[size_t(t) * np + u] += wq * gg;
        C.Mp[size_t(t) * np + u] += wq * p.v[u] * p.v[t];
      }
    }
  }
  // boundary faces
  int nqf = 1;
  for (int a = 0; a < d - 1; ++a) nqf *= nq1;
  for (int axis = 0; axis < d; ++axis)
    for (int side = 0; side < 2; ++side) {
      int f = 2 * axis + side;
      auto& Af = C.Aface[f];
      auto& Cf = C.Cface[f];
      auto& BK = C.BfaceK[f];
      auto& Bp = C.Bpen[f];
      Af.assign(size_t(nv) * nv, 0.0);
      Cf.assign(size_t(np) * nv, 0.0);
      BK.assign(size_t(np) * np, 0.0);
      Bp.assign(size_t(np) * np, 0.0);
      double nrm[3] = {0, 0, 0};
      nrm[axis] = side ? 1.0 : -1.0;
      for (int q = 0; q < nqf; ++q) {
        double xi[3] = {0, 0, 0}, wq = 1.0;
        int rem = q;
        for (int ax = 0; ax < d; ++ax) {
          if (ax == axis) {
            xi[ax] = side ? 1.0 : 0.0;
            continue;
          }
          xi[ax] = gx[rem % nq1];
          wq *= gw[rem % nq1] * h;
          rem /= nq1;
        }
        tabulate(r, d, xi, h, s);
        tabulate_p(disc, r, d, xi, h, p);
        for (int b = 0; b < ns; ++b)
          for (int a = 0; a < ns; ++a) {
            double dna = 0.0, dnb = 0.0;
            for (int j = 0; j < d; ++j) {
              dna += s.g[a * 3 + j] * nrm[j];
              dnb += s.g[b * 3 + j] * nrm[j];
            }
            for (int e = 0; e < d; ++e)
              for (int c = 0; c < d; ++c) {
                // traction of w = phi_a e_c: (sigma n)_i = mu(delta_ic d_n a + d_i a n_c) + lam d_c a n_i
                double tw_e = mu * ((e == c ? dna : 0.0) + s.g[a * 3 + e] * nrm[c]) + lam * s.g[a * 3 + c] * nrm[e];
                double tc_c = mu * ((c == e ? dnb : 0.0) + s.g[b * 3 + c] * nrm[e]) + lam * s.g[b * 3 + e] * nrm[c];
                double val = -tw_e * s.v[b] - s.v[a] * tc_c;
                if (c == e) val += C.gamma_a / C.hF * s.v[a] * s.v[b];
                Af[size_t(d * b + e) * nv + d * a + c] += wq * val;
              }
          }
        for (int t = 0; t < np; ++t) {
          for (int a = 0; a < ns; ++a)
            for (int c = 0; c < d; ++c) Cf[size_t(t) * nv + d * a + c] += m.alpha * wq * s.v[a] * nrm[c] * p.v[t];
          double dnt = 0.0;
          for (int j = 0; j < d; ++j) dnt += p.g[t * 3 + j] * nrm[j];
          for (int u = 0; u < np; ++u) {
            double dnu = 0.0;
            for (int j = 0; j < d; ++j) dnu += p.g[u * 3 + j] * nrm[j];
            BK[size_t(t) * np + u] += wq * (-dnu * p.v[t] - p.v[u] * dnt);
            Bp[size_t(t) * np + u] += wq * C.gamma_b / C.hF * p.v[u] * p.v[t];
          }
        }
      }
    }
  if (!disc) return C;
  // interior faces normal to axis: K+ (lower cell) sees the face at xi_axis = 1, K- (upper
  // cell) at xi_axis = 0, the same physical points; n = +e_axis; jump sign +1 on K+, -1 on K-
  for (int axis = 0; axis < d; ++axis) {
    for (int ba = 0; ba < 4; ++ba) {
      C.BiT1[axis][ba].assign(size_t(np) * np, 0.0);
      C.BiT2[axis][ba].assign(size_t(np) * np, 0.0);
      C.BiPen[axis][ba].assign(size_t(np) * np, 0.0);
    }
    for (int q = 0; q < nqf; ++q) {
      double xp[3] = {0, 0, 0}, xm[3] = {0, 0, 0}, wq = 1.0;
      int rem = q;
      for (int ax = 0; ax < d; ++ax) {
        if (ax == axis) {
          xp[ax] = 1.0;
          xm[ax] = 0.0;
          continue;
        }
        xp[ax] = xm[ax] = gx[rem % nq1];
        wq *= gw[rem % nq1] * h;
        rem /= nq1;
      }
      Tab side[2];
      tabulate_pdisc(r - 1, d, xp, h, side[0]);
      tabulate_pdisc(r - 1, d, xm, h, side[1]);
      const double sgn[2] = {1.0, -1.0};
      for (int b = 0; b < 2; ++b)
        for (int a = 0; a < 2; ++a) {
          auto& T1 = C.BiT1[axis][2 * b + a];
          auto& T2 = C.BiT2[axis][2 * b + a];
          auto& Pn = C.BiPen[axis][2 * b + a];
          for (int t = 0; t < np; ++t)      // test function on cell b
            for (int u = 0; u < np; ++u) {  // trial function on cell a
              const double qv = side[a].v[u], qn = side[a].g[u * 3 + axis];
              const double pv = side[b].v[t], pn = side[b].g[t * 3 + axis];
              // -<{K grad q} . n, [psi]>, -<[q], {K grad psi} . n>, gamma/h_F <[q], [psi]>
              T1[size_t(t) * np + u] += wq * (-0.5 * qn * sgn[b] * pv);
              T2[size_t(t) * np + u] += wq * (-0.5 * sgn[a] * qv * pn);
              Pn[size_t(t) * np + u] += wq * C.gamma_b / C.hF * sgn[a] * qv * sgn[b] * pv;
            }
        }
    }
  }
  return C;
}

// ------------------------------------------------------------- level assembly
namespace {

struct Entry {
  int64_t col;
  double val;
};

struct RowBuilder {
  const BuildOptions* o;
  const CellMats* cm;
  const LevelHost* L;
  const Material* m;

  // cells touching lattice point g (per axis) for a degree-p lattice; local index
  int cells_axis(int64_t g, int p, int N, int* cells, int* loc) const {
    int cnt = 0;
    if (g % p == 0) {
      int64_t c = g / p;
      if (c - 1 >= 0) {
        cells[cnt] = int(c - 1);
        loc[cnt++] = p;
      }
      if (c < N) {
        cells[cnt] = int(c);
        loc[cnt++] = 0;
      }
    } else {
      cells[cnt] = int(g / p);
      loc[cnt++] = int(g % p);
    }
    return cnt;
  }

  // global lattice index of local node a of cell (cx,cy,cz) for degree p
  int64_t gnode(const int* cc, int a, int p, int64_t n1) const {
    int d = o->d;
    int64_t g = 0;
    int idx[3];
    int rem = a;
    for (int ax = 0; ax < d; ++ax) {
      idx[ax] = rem % (p + 1);
      rem /= (p + 1);
    }
    for (int ax = d - 1; ax >= 0; --ax) g = g * n1 + (int64_t(p) * cc[ax] + idx[ax]);
    return g;
  }

  static void sort_merge(std::vector<Entry>& v) {
    std::sort(v.begin(), v.end(), [](const Entry& a, const Entry& b) { return a.col < b.col; });
    size_t w = 0;
    for (size_t i = 0; i < v.size(); ++i) {
      if (w > 0 && v[w - 1].col == v[i].col)
        v[w - 1].val += v[i].val;
      else
        v[w++] = v[i];
    }
    v.resize(w);
  }

  // p-equation row of pressure dof j (cell j / nlp, local function j % nlp) for the broken
  // pressure: -C on V, c0 M_p and the SIPG form (volume, boundary faces, interior faces with
  // the neighbour's functions as further columns).
  void disc_prow(int64_t j, std::vector<Entry>& mm, std::vector<Entry>& kk) const {
    const int d = o->d, r = o->r, N = o->N;
    const int64_t nv = L->nv;
    const int nlv = cm->nlv, nls = cm->nls, nlp = cm->nlp;
    const int64_t cell = j / nlp;
    const int st = int(j % nlp);
    int cc[3] = {0, 0, 0};
    int64_t rem = cell;
    for (int ax = 0; ax < d; ++ax) {
      cc[ax] = int(rem % N);
      rem /= N;
    }
    const double K = L->Kcell[cell];
    int faces[6], nf = 0;
    for (int ax = 0; ax < d; ++ax) {
      if (cc[ax] == 0) faces[nf++] = 2 * ax;
      if (cc[ax] == N - 1) faces[nf++] = 2 * ax + 1;
    }
    for (int a = 0; a < nls; ++a) {
      const int64_t gn = gnode(cc, a, r, L->n1);
      for (int c = 0; c < d; ++c) {
        const int at = d * a + c;
        double cv = cm->Cvol[size_t(st) * nlv + at];
        for (int f = 0; f < nf; ++f) cv += cm->Cface[faces[f]][size_t(st) * nlv + at];
        if (o->dtu)
          mm.push_back({nv + d * gn + c, -cv});  // -C(d_t u, psi): on U, time-derivative part
        else
          kk.push_back({d * gn + c, -cv});       // -C(v, psi): on V
      }
    }
    // own cell: volume, boundary faces, and the own-cell blocks of its interior faces
    std::vector<double> own(nlp, 0.0);
    for (int s = 0; s < nlp; ++s) {
      double bv = K * cm->Bvol[size_t(st) * nlp + s];
      for (int f = 0; f < nf; ++f)
        bv += K * cm->BfaceK[faces[f]][size_t(st) * nlp + s] + cm->Bpen[faces[f]][size_t(st) * nlp + s];
      own[s] = bv;
    }
    int64_t stride = 1;
    for (int ax = 0; ax < d; ++ax) {
      for (int side = 0; side < 2; ++side) {
        // side 1: the upper neighbour exists, this cell is K+ (index 0); side 0: lower, this is K-
        if (side == 1 ? cc[ax] == N - 1 : cc[ax] == 0) continue;
        const int64_t nb = side == 1 ? cell + stride : cell - stride;
        const int me = side == 1 ? 0 : 1, ot = 1 - me;
        const double Kn = L->Kcell[nb];
        const size_t bo = size_t(2 * me + ot), bs = size_t(2 * me + me);
        for (int s = 0; s < nlp; ++s) {
          const size_t e = size_t(st) * nlp + s;
          own[s] += K * cm->BiT1[ax][bs][e] + K * cm->BiT2[ax][bs][e] + cm->BiPen[ax][bs][e];
          kk.push_back({2 * nv + nb * nlp + s,
                        Kn * cm->BiT1[ax][bo][e] + K * cm->BiT2[ax][bo][e] + cm->BiPen[ax][bo][e]});
        }
      }
      stride *= N;
    }
    for (int s = 0; s < nlp; ++s) {
      const int64_t gp = 2 * nv + cell * nlp + s;
      mm.push_back({gp, m->c0 * cm->Mp[size_t(st) * nlp + s]});
      kk.push_back({gp, own[s]});
    }
  }

  // Boundary-face part of C in p-equation row j (columns: velocity dofs), sorted and merged.
  void cface_row(int64_t j, std::vector<Entry>& out) const {
    out.clear();
    const int d = o->d, r = o->r, N = o->N;
    const int nlv = cm->nlv, nls = cm->nls;
    int cl[3][2], ll[3][2], cn[3] = {1, 1, 1};
    if (L->disc) {
      int64_t rem = j / cm->nlp;
      for (int ax = 0; ax < d; ++ax) {
        cl[ax][0] = int(rem % N);
        rem /= N;
        ll[ax][0] = 0;
      }
    } else {
      int64_t rem = j;
      for (int ax = 0; ax < d; ++ax) {
        cn[ax] = cells_axis(rem % L->n1p, r - 1, N, cl[ax], ll[ax]);
        rem /= L->n1p;
      }
    }
    int combos = 1;
    for (int ax = 0; ax < d; ++ax) combos *= cn[ax];
    for (int cb = 0; cb < combos; ++cb) {
      int cc[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, t = cb;
      for (int ax = 0; ax < d; ++ax) {
        cc[ax] = cl[ax][t % cn[ax]];
        lo[ax] = ll[ax][t % cn[ax]];
        t /= cn[ax];
      }
      int st = 0;
      if (L->disc) {
        st = int(j % cm->nlp);
      } else {
        for (int ax = d - 1; ax >= 0; --ax) st = st * r + lo[ax];
      }
      int faces[6], nf = 0;
      for (int ax = 0; ax < d; ++ax) {
        if (cc[ax] == 0) faces[nf++] = 2 * ax;
        if (cc[ax] == N - 1) faces[nf++] = 2 * ax + 1;
      }
      if (nf == 0) continue;
      for (int a = 0; a < nls; ++a) {
        const int64_t gn = gnode(cc, a, r, L->n1);
        for (int c = 0; c < d; ++c) {
          double cv = 0.0;
          for (int f = 0; f < nf; ++f) cv += cm->Cface[faces[f]][size_t(st) * nlv + d * a + c];
          out.push_back({d * gn + c, cv});
        }
      }
    }
    sort_merge(out);
  }

  // Spatial row i of MM and KK (sorted, merged).
  void row(int64_t i, std::vector<Entry>& mm, std::vector<Entry>& kk) const {
    mm.clear();
    kk.clear();
    const int d = o->d, r = o->r, N = o->N;
    const int64_t nv = L->nv;
    const int nlv = cm->nlv, nls = cm->nls, nlp = cm->nlp;
    if (i < 2 * nv) {
      const int field = i < nv ? 0 : 1;  // 0: u-equation, 1: v-equation
      const int64_t iv = i - field * nv;
      const int64_t node = iv / d;
      const int comp = int(iv % d);
      int64_t g[3];
      int64_t rem = node;
      for (int ax = 0; ax < d; ++ax) {
        g[ax] = rem % L->n1;
        rem /= L->n1;
      }
      int cl[3][2], ll[3][2], cn[3];
      for (int ax = 0; ax < d; ++ax) cn[ax] = cells_axis(g[ax], r, N, cl[ax], ll[ax]);
      int combos = 1;
      for (int ax = 0; ax < d; ++ax) combos *= cn[ax];
      for (int cb = 0; cb < combos; ++cb) {
        int cc[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, t = cb;
        for (int ax = 0; ax < d; ++ax) {
          cc[ax] = cl[ax][t % cn[ax]];
          lo[ax] = ll[ax][t % cn[ax]];
          t /= cn[ax];
        }
        int a_test = 0;
        for (int ax = d - 1; ax >= 0; --ax) a_test = a_test * (r + 1) + lo[ax];
        const int bt = d * a_test + comp;  // local vector test index
        int64_t cell = 0;
        for (int ax = d - 1; ax >= 0; --ax) cell = cell * N + cc[ax];
        const double K = L->Kcell[cell];
        // boundary faces of this cell
        int faces[6], nf = 0;
        for (int ax = 0; ax < d; ++ax) {
          if (cc[ax] == 0) faces[nf++] = 2 * ax;
          if (cc[ax] == N - 1) faces[nf++] = 2 * ax + 1;
        }
        (void)K;
        for (int a = 0; a < nls; ++a) {
          const int64_t gn = gnode(cc, a, r, L->n1);
          for (int c = 0; c < d; ++c) {
            const int at = d * a + c;
            const int64_t gcol = d * gn + c;
            const double mr = cm->Mrho[size_t(bt) * nlv + at];
            if (field == 0) {
              if (mr != 0.0) {
                mm.push_back({nv + gcol, mr});   // M_rho on U
                kk.push_back({gcol, -mr});       // -M_rho on V
              }
            } else {
              if (mr != 0.0) mm.push_back({gcol, mr});  // M_rho on V
              double av = cm->Avol[size_t(bt) * nlv + at];
              for (int f = 0; f < nf; ++f) av += cm->Aface[faces[f]][size_t(bt) * nlv + at];
              kk.push_back({nv + gcol, av});  // A_gamma on U
            }
          }
        }
        if (field == 1) {
          for (int s = 0; s < nlp; ++s) {
            // (C^T)[i][s] = C(psi_i, xi_s): stored as Cvol[s][i]
            double cv = cm->Cvol[size_t(s) * nlv + bt];
            for (int f = 0; f < nf; ++f) cv += cm->Cface[faces[f]][size_t(s) * nlv + bt];
            const int64_t pc = L->disc ? cell * nlp + s : gnode(cc, s, r - 1, L->n1p);
            kk.push_back({2 * nv + pc, cv});
          }
        }
      }
    } else if (L->disc) {
      disc_prow(i - 2 * nv, mm, kk);
    } else {
      const int64_t node = i - 2 * nv;
      int64_t g[3];
      int64_t rem = node;
      for (int ax = 0; ax < d; ++ax) {
        g[ax] = rem % L->n1p;
        rem /= L->n1p;
      }
      int cl[3][2], ll[3][2], cn[3];
      for (int ax = 0; ax < d; ++ax) cn[ax] = cells_axis(g[ax], r - 1, N, cl[ax], ll[ax]);
      int combos = 1;
      for (int ax = 0; ax < d; ++ax) combos *= cn[ax];
      for (int cb = 0; cb < combos; ++cb) {
        int cc[3] = {0, 0, 0}, lo[3] = {0, 0, 0}, t = cb;
        for (int ax = 0; ax < d; ++ax) {
          cc[ax] = cl[ax][t % cn[ax]];
          lo[ax] = ll[ax][t % cn[ax]];
          t /= cn[ax];
        }
        int st = 0;
        for (int ax = d - 1; ax >= 0; --ax) st = st * r + lo[ax];
        int64_t cell = 0;
        for (int ax = d - 1; ax >= 0; --ax) cell = cell * N + cc[ax];
        const double K = L->Kcell[cell];
        int faces[6], nf = 0;
        for (int ax = 0; ax < d; ++ax) {
          if (cc[ax] == 0) faces[nf++] = 2 * ax;
          if (cc[ax] == N - 1) faces[nf++] = 2 * ax + 1;
        }
        // -C(v, psi_st) on V (Problem 3.1) or -C(d_t u, psi_st) on U (Problem B.1)
        for (int a = 0; a < nls; ++a) {
          const int64_t gn = gnode(cc, a, r, L->n1);
          for (int c = 0; c < d; ++c) {
            const int at = d * a + c;
            double cv = cm->Cvol[size_t(st) * nlv + at];
            for (int f = 0; f < nf; ++f) cv += cm->Cface[faces[f]][size_t(st) * nlv + at];
            if (o->dtu)
              mm.push_back({nv + d * gn + c, -cv});
            else
              kk.push_back({d * gn + c, -cv});
          }
        }
        for (int s = 0; s < nlp; ++s) {
          const int64_t gp = 2 * nv + gnode(cc, s, r - 1, L->n1p);
          mm.push_back({gp, m->c0 * cm->Mp[size_t(st) * nlp + s]});
          double bv = K * cm->Bvol[size_t(st) * nlp + s];
          for (int f = 0; f < nf; ++f)
            bv += K * cm->BfaceK[faces[f]][size_t(st) * nlp + s] + cm->Bpen[faces[f]][size_t(st) * nlp + s];
          kk.push_back({gp, bv});
        }
      }
    }
    sort_merge(mm);
    sort_merge(kk);
  }
};

}  // namespace

void build_level(const BuildOptions& o, const Material& m, const std::vector<double>& Kcell, LevelHost& L,
                 int nthreads) {
  L.d = o.d;
  L.r = o.r;
  L.k = o.k;
  L.N = o.N;
  const int d = o.d, r = o.r, k = o.k, N = o.N;
  L.n1 = int64_t(r) * N + 1;
  L.n1p = int64_t(r - 1) * N + 1;
  L.nQ = 1;
  L.nP = 1;
  for (int a = 0; a < d; ++a) {
    L.nQ *= L.n1;
    L.nP *= L.n1p;
  }
  L.disc = o.disc;
  L.dtu = o.dtu;
  int64_t ncells_l = 1;
  for (int a = 0; a < d; ++a) ncells_l *= N;
  if (o.disc) {
    L.nlp = int(pdisc_exponents(r - 1, d).size());
    L.nP = ncells_l * L.nlp;
  }
  L.nv = d * L.nQ;
  L.ns = 2 * L.nv + L.nP;
  L.n = (k + 1) * L.ns;
  L.Kcell = Kcell;
  const double h = 1.0 / N;
  CellMats cm = make_cell_mats(d, r, h, m, o.disc);
  TimeConsts T = make_time_consts(k, o.tau);
  RowBuilder rb{&o, &cm, &L, &m};
  const int64_t ns = L.ns;
  const int nt = k + 1;

  if (!o.need_A) {
    // no space-time matrix: each spatial row of MM and KK is built once into the buffer of its
    // chunk of rows, and the chunks are copied into place behind the prefix sums
    const int nch = int(std::max<int64_t>(1, std::min<int64_t>(nthreads, (ns + 4095) / 4096)));
    const int64_t chunk = (ns + nch - 1) / nch;
    std::vector<std::vector<Entry>> bm(nch), bk(nch);
    std::vector<int64_t> mmlen(ns), kklen(ns);
    auto run = [&](auto&& body) {
      std::vector<std::thread> th;
      for (int c = 1; c < nch; ++c) th.emplace_back([&body, c] { body(c); });
      body(0);
      for (auto& x : th) x.join();
    };
    run([&](int c) {
      std::vector<Entry> mm, kk;
      for (int64_t i = c * chunk; i < std::min(ns, (c + 1) * chunk); ++i) {
        rb.row(i, mm, kk);
        mmlen[i] = int64_t(mm.size());
        kklen[i] = int64_t(kk.size());
        if (o.need_MM) bm[c].insert(bm[c].end(), mm.begin(), mm.end());
        if (o.need_KK) bk[c].insert(bk[c].end(), kk.begin(), kk.end());
      }
    });
    auto finish = [&](bool need, Csr& M, const std::vector<int64_t>& len, std::vector<std::vector<Entry>>& buf) {
      if (!need) return;
      M.nrows = ns;
      M.ncols = ns;
      M.ptr.assign(ns + 1, 0);
      for (int64_t i = 0; i < ns; ++i) M.ptr[i + 1] = M.ptr[i] + len[i];
      M.col.resize(M.ptr[ns]);
      M.val.resize(M.ptr[ns]);
      run([&](int c) {
        int64_t q = M.ptr[std::min(ns, c * chunk)];
        for (const Entry& e : buf[c]) {
          M.col[q] = int32_t(e.col);
          M.val[q++] = e.val;
        }
        std::vector<Entry>().swap(buf[c]);
      });
    };
    finish(o.need_MM, L.MM, mmlen, bm);
    finish(o.need_KK, L.KK, kklen, bk);
  } else {
  // pass 1: space-time row lengths
  std::vector<int64_t> slen(ns);  // length of one space-time row for spatial row i (same for every b)
  std::vector<int64_t> mmlen(ns), kklen(ns);
  parallel_for(ns, nthreads, [&](int64_t lo, int64_t hi) {
    std::vector<Entry> mm, kk;
    for (int64_t i = lo; i < hi; ++i) {
      rb.row(i, mm, kk);
      // union of MM and KK columns for the diagonal time block
      size_t a = 0, b = 0, u = 0;
      while (a < mm.size() || b < kk.size()) {
        if (b >= kk.size() || (a < mm.size() && mm[a].col < kk[b].col))
          ++a;
        else if (a >= mm.size() || kk[b].col < mm[a].col)
          ++b;
        else {
          ++a;
          ++b;
        }
        ++u;
      }
      slen[i] = int64_t(k) * int64_t(mm.size()) + int64_t(u);
      mmlen[i] = int64_t(mm.size());
      kklen[i] = int64_t(kk.size());
    }
  });
  if (o.need_A) {
    L.A.nrows = L.n;
    L.A.ncols = L.n;
    L.A.ptr.assign(L.n + 1, 0);
    for (int b = 0; b < nt; ++b)
      for (int64_t i = 0; i < ns; ++i) L.A.ptr[b * ns + i + 1] = slen[i];
    for (int64_t i = 0; i < L.n; ++i) L.A.ptr[i + 1] += L.A.ptr[i];
    const int64_t nnz = L.A.ptr[L.n];
    if (nnz > INT64_C(4000000000)) throw std::runtime_error("level operator too large");
    L.A.col.resize(nnz);
    L.A.val.resize(nnz);
  }
  if (o.need_MM) {
    L.MM.nrows = ns;
    L.MM.ncols = ns;
    L.MM.ptr.assign(ns + 1, 0);
    for (int64_t i = 0; i < ns; ++i) L.MM.ptr[i + 1] = L.MM.ptr[i] + mmlen[i];
    L.MM.col.resize(L.MM.ptr[ns]);
    L.MM.val.resize(L.MM.ptr[ns]);
  }
  if (o.need_KK) {
    L.KK.nrows = ns;
    L.KK.ncols = ns;
    L.KK.ptr.assign(ns + 1, 0);
    for (int64_t i = 0; i < ns; ++i) L.KK.ptr[i + 1] = L.KK.ptr[i] + kklen[i];
    L.KK.col.resize(L.KK.ptr[ns]);
    L.KK.val.resize(L.KK.ptr[ns]);
  }
  // pass 2: fill
  parallel_for(ns, nthreads, [&](int64_t lo, int64_t hi) {
    std::vector<Entry> mm, kk;
    for (int64_t i = lo; i < hi; ++i) {
      rb.row(i, mm, kk);
      if (o.need_MM) {
        int64_t p = L.MM.ptr[i];
        for (auto& e : mm) {
          L.MM.col[p] = int32_t(e.col);
          L.MM.val[p++] = e.val;
        }
      }
      if (o.need_KK) {
        int64_t p = L.KK.ptr[i];
        for (auto& e : kk) {
          L.KK.col[p] = int32_t(e.col);
          L.KK.val[p++] = e.val;
        }
      }
      for (int b = 0; b < nt && o.need_A; ++b) {
        int64_t p = L.A.ptr[b * ns + i];
        for (int a = 0; a < nt; ++a) {
          const double D = T.Dt[b * nt + a];
          const int64_t off = int64_t(a) * ns;
          if (a != b) {
            for (auto& e : mm) {
              L.A.col[p] = int32_t(off + e.col);
              L.A.val[p++] = D * e.val;
            }
          } else {
            const double mt = T.mt[b];
            size_t x = 0, y = 0;
            while (x < mm.size() || y < kk.size()) {
              if (y >= kk.size() || (x < mm.size() && mm[x].col < kk[y].col)) {
                L.A.col[p] = int32_t(off + mm[x].col);
                L.A.val[p++] = D * mm[x].val;
                ++x;
              } else if (x >= mm.size() || kk[y].col < mm[x].col) {
                L.A.col[p] = int32_t(off + kk[y].col);
                L.A.val[p++] = mt * kk[y].val;
                ++y;
              } else {
                L.A.col[p] = int32_t(off + mm[x].col);
                L.A.val[p++] = D * mm[x].val + mt * kk[y].val;
                ++x;
                ++y;
              }
            }
          }
        }
      }
    }
  });

  }  // need_A

  if (o.need_Cface) {
    L.Cface = Csr();
    L.Cface.nrows = L.nP;
    L.Cface.ncols = L.nv;
    L.Cface.ptr.assign(L.nP + 1, 0);
    std::vector<Entry> e;
    for (int64_t j = 0; j < L.nP; ++j) {
      rb.cface_row(j, e);
      L.Cface.ptr[j + 1] = L.Cface.ptr[j] + int64_t(e.size());
      for (const Entry& x : e) {
        L.Cface.col.push_back(int32_t(x.col));
        L.Cface.val.push_back(x.val);
      }
    }
  }

  if (!o.need_patches) return;
  // ------------------------------------------------------------ patches
  // vertex patch at grid vertex v: the cells with c in {v-1, v} (per axis) that exist;
  // cell patch: the cell itself.  Closure node boxes per axis.
  const int64_t nverts = o.patch_kind == 1 ? [&] {
    int64_t t = 1;
    for (int a = 0; a < d; ++a) t *= (N + 1);
    return t;
  }()
                                           : 0;
  int64_t ncells = 1;
  for (int a = 0; a < d; ++a) ncells *= N;
  L.npatch = o.patch_kind == 1 ? nverts : ncells;
  auto patch_box = [&](int64_t pidx, int* cmin, int* cmax) {
    int64_t rem = pidx;
    const int base = o.patch_kind == 1 ? N + 1 : N;
    for (int ax = 0; ax < d; ++ax) {
      int v = int(rem % base);
      rem /= base;
      if (o.patch_kind == 1) {
        cmin[ax] = std::max(v - 1, 0);
        cmax[ax] = std::min(v, N - 1);
      } else {
        cmin[ax] = cmax[ax] = v;
      }
    }
  };
  L.poff.assign(L.npatch + 1, 0);
  for (int64_t pi = 0; pi < L.npatch; ++pi) {
    int cmin[3], cmax[3];
    patch_box(pi, cmin, cmax);
    int64_t q = 1, pp = 1, pc = 1;
    for (int ax = 0; ax < d; ++ax) {
      q *= int64_t(r) * (cmax[ax] + 1 - cmin[ax]) + 1;
      pp *= int64_t(r - 1) * (cmax[ax] + 1 - cmin[ax]) + 1;
      pc *= cmax[ax] + 1 - cmin[ax];
    }
    if (o.disc) pp = pc * L.nlp;
    L.poff[pi + 1] = L.poff[pi] + nt * (2 * d * q + pp);
  }
  L.pdof.resize(L.poff[L.npatch]);
  parallel_for(L.npatch, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t pi = lo; pi < hi; ++pi) {
      int cmin[3] = {0, 0, 0}, cmax[3] = {0, 0, 0};
      patch_box(pi, cmin, cmax);
      int64_t w = L.poff[pi];
      int lo3[3] = {0, 0, 0}, hi3[3] = {0, 0, 0}, lop[3] = {0, 0, 0}, hip3[3] = {0, 0, 0};
      for (int ax = 0; ax < 3; ++ax) {
        if (ax < d) {
          lo3[ax] = r * cmin[ax];
          hi3[ax] = r * (cmax[ax] + 1);
          lop[ax] = (r - 1) * cmin[ax];
          hip3[ax] = (r - 1) * (cmax[ax] + 1);
        }
      }
      for (int tn = 0; tn < nt; ++tn) {
        const int64_t off = int64_t(tn) * ns;
        for (int field = 0; field < 2; ++field)
          for (int z = lo3[2]; z <= hi3[2]; ++z)
            for (int y = lo3[1]; y <= hi3[1]; ++y)
              for (int x = lo3[0]; x <= hi3[0]; ++x) {
                int64_t node = x + L.n1 * (y + L.n1 * int64_t(z));
                for (int c = 0; c < d; ++c) L.pdof[w++] = int32_t(off + field * L.nv + d * node + c);
              }
        if (o.disc) {
          // the pressure functions of the patch cells, cells in increasing order
          for (int z = cmin[2]; z <= cmax[2]; ++z)
            for (int y = cmin[1]; y <= cmax[1]; ++y)
              for (int x = cmin[0]; x <= cmax[0]; ++x) {
                const int64_t cell = x + int64_t(N) * (y + int64_t(N) * z);
                for (int s = 0; s < L.nlp; ++s) L.pdof[w++] = int32_t(off + 2 * L.nv + cell * L.nlp + s);
              }
        } else {
          for (int z = lop[2]; z <= hip3[2]; ++z)
            for (int y = lop[1]; y <= hip3[1]; ++y)
              for (int x = lop[0]; x <= hip3[0]; ++x)
                L.pdof[w++] = int32_t(off + 2 * L.nv + x + L.n1p * (y + L.n1p * int64_t(z)));
        }
      }
    }
  });
  // dof-major slots of the patch entries (deterministic: patches in increasing order).  The
  // entries of one (time node, field) of a patch are contiguous and touch only that block of
  // dofs, so the nt * 3 blocks are independent streams.
  L.tptr.assign(L.n + 1, 0);
  for (int64_t t = 0; t < int64_t(L.pdof.size()); ++t) L.tptr[L.pdof[t] + 1]++;
  for (int64_t i = 0; i < L.n; ++i) L.tptr[i + 1] += L.tptr[i];
  L.tpos.resize(L.pdof.size());
  {
    std::vector<int64_t> fill(L.tptr.begin(), L.tptr.end() - 1);
    const int nstream = nt * 3;
    parallel_for(nstream * 4096, std::min(nthreads, nstream), [&](int64_t lo, int64_t hi) {
      for (int64_t sidx = lo / 4096; sidx < (hi + 4095) / 4096 && sidx < nstream; ++sidx) {
        if (sidx * 4096 < lo) continue;  // each stream is handled by the thread holding its first index
        const int tn = int(sidx / 3), field = int(sidx % 3);
        for (int64_t pi = 0; pi < L.npatch; ++pi) {
          const int64_t o = L.poff[pi], nsp = (L.poff[pi + 1] - o) / nt;
          const int32_t* b0 = L.pdof.data() + o + tn * nsp;
          const int64_t nU = std::lower_bound(L.pdof.data() + o, L.pdof.data() + o + nsp, int32_t(L.nv)) -
                             (L.pdof.data() + o);
          const int64_t f0 = field == 0 ? 0 : field == 1 ? nU : 2 * nU, f1 = field == 0 ? nU : field == 1 ? 2 * nU : nsp;
          for (int64_t l = f0; l < f1; ++l) L.tpos[o + tn * nsp + l] = int32_t(fill[b0[l]]++);
        }
      }
    });
  }
  L.winv.resize(L.n);
  for (int64_t i = 0; i < L.n; ++i) {
    int64_t c = L.tptr[i + 1] - L.tptr[i];
    if (c == 0) throw std::runtime_error("dof not covered by any patch");
    L.winv[i] = o.omega / double(c);
  }
}

// ------------------------------------------------------------- node-pair form of the velocity rows
bool build_node_op(const LevelHost& L, NodeOp& out, int nthreads) {
  const int d = L.d;
  const int64_t nQ = L.nQ, nv = L.nv, np = L.nP;
  const Csr &MM = L.MM, &KK = L.KK;
  out = NodeOp();
  if (MM.nrows != L.ns || KK.nrows != L.ns || nv != int64_t(d) * nQ) return false;
  using NodeList = std::vector<std::pair<int32_t, double>>;
  // the sorted node list (j, rhoM_ij) from MM's u-row of component 0 and the union of the
  // pressure columns of KK's v-rows of node i
  auto node_list = [&](int64_t i, NodeList& nodes, std::vector<int32_t>& pcols) -> bool {
    nodes.clear();
    pcols.clear();
    const int64_t r0 = int64_t(d) * i;
    for (int64_t p = MM.ptr[r0]; p < MM.ptr[r0 + 1]; ++p) {
      const int64_t c = MM.col[p];
      if (c >= nv && c < 2 * nv && (c - nv) % d == 0)
        nodes.emplace_back(int32_t((c - nv) / d), MM.val[p]);
      else if (MM.val[p] != 0.0)
        return false;
    }
    std::sort(nodes.begin(), nodes.end());
    for (int c = 0; c < d; ++c) {
      const int64_t rv = nv + int64_t(d) * i + c;
      for (int64_t p = KK.ptr[rv]; p < KK.ptr[rv + 1]; ++p)
        if (KK.col[p] >= 2 * nv) pcols.push_back(int32_t(KK.col[p] - 2 * nv));
    }
    std::sort(pcols.begin(), pcols.end());
    pcols.erase(std::unique(pcols.begin(), pcols.end()), pcols.end());
    return true;
  };
  auto find = [](const NodeList& v, int32_t j) -> int64_t {
    auto it = std::lower_bound(v.begin(), v.end(), j,
                               [](const std::pair<int32_t, double>& e, int32_t k) { return e.first < k; });
    return (it != v.end() && it->first == j) ? int64_t(it - v.begin()) : -1;
  };
  std::vector<int64_t> cnt(nQ + 1, 0), ccnt(nQ + 1, 0);
  std::vector<char> bad(nQ, 0);
  parallel_for(nQ, nthreads, [&](int64_t i0, int64_t i1) {
    NodeList nodes;
    std::vector<int32_t> pcols;
    for (int64_t i = i0; i < i1; ++i) {
      if (!node_list(i, nodes, pcols)) {
        bad[i] = 1;
        continue;
      }
      cnt[i + 1] = int64_t(nodes.size());
      ccnt[i + 1] = int64_t(pcols.size());
    }
  });
  for (int64_t i = 0; i < nQ; ++i)
    if (bad[i]) return false;
  for (int64_t i = 0; i < nQ; ++i) {
    cnt[i + 1] += cnt[i];
    ccnt[i + 1] += ccnt[i];
  }
  NodeOp o;
  o.d = d;
  o.nQ = nQ;
  o.ptr = cnt;
  o.cptr = ccnt;
  o.col.resize(size_t(cnt[nQ]));
  o.m.resize(size_t(cnt[nQ]));
  o.a.assign(size_t(cnt[nQ]) * d * d, 0.0);
  o.ccol.resize(size_t(ccnt[nQ]));
  o.c.assign(size_t(ccnt[nQ]) * d, 0.0);
  // fill, checking every velocity row against the structure; the position of a neighbour node
  // (pressure dof) in the node's list is looked up in a per-thread table, reset after each node
  parallel_for(nQ, nthreads, [&](int64_t i0, int64_t i1) {
    NodeList nodes;
    std::vector<int32_t> pcols;
    std::vector<int32_t> at(size_t(nQ), -1), atp(size_t(np), -1);
    auto find = [&](const NodeList&, int32_t j) -> int64_t { return (j >= 0 && j < nQ) ? at[size_t(j)] : -1; };
    for (int64_t i = i0; i < i1; ++i) {
      node_list(i, nodes, pcols);
      const int64_t e0 = o.ptr[i], c0 = o.cptr[i];
      const int64_t nn = int64_t(nodes.size());
      for (int64_t t = 0; t < nn; ++t) {
        o.col[size_t(e0 + t)] = nodes[size_t(t)].first;
        o.m[size_t(e0 + t)] = nodes[size_t(t)].second;
        at[size_t(nodes[size_t(t)].first)] = int32_t(t);
      }
      for (size_t t = 0; t < pcols.size(); ++t) {
        o.ccol[size_t(c0) + t] = pcols[t];
        atp[size_t(pcols[t])] = int32_t(t);
      }
      // the rows of one kind (which CSR, which row block) must hold sign * rhoM_ij at the
      // column (col_block + d j + c) for every listed node j and nothing else
      auto mass_rows = [&](const Csr& A, int64_t row, int64_t col0, double sign) {
        int64_t seen = 0;
        for (int64_t p = A.ptr[row]; p < A.ptr[row + 1]; ++p) {
          const int64_t cl = A.col[p] - col0;
          const double v = A.val[p];
          if (cl >= 0 && cl < nv && cl % d == (row % d)) {
            const int64_t t = find(nodes, int32_t(cl / d));
            if (t < 0 || nodes[size_t(t)].second != sign * v) return false;
            ++seen;
          } else if (v != 0.0) {
            return false;
          }
        }
        return seen == nn;
      };
      for (int c = 0; c < d && !bad[i]; ++c) {
        const int64_t ru = int64_t(d) * i + c, rv = nv + ru;
        // nv is a multiple of d, so row % d is the component in both row blocks
        if (!mass_rows(MM, ru, nv, 1.0) || !mass_rows(KK, ru, 0, -1.0) || !mass_rows(MM, rv, 0, 1.0)) {
          bad[i] = 1;
          break;
        }
        // KK v-row: A on U (the listed nodes), C^T on P, nothing on V
        for (int64_t p = KK.ptr[rv]; p < KK.ptr[rv + 1] && !bad[i]; ++p) {
          const int64_t cl = KK.col[p];
          const double v = KK.val[p];
          if (cl >= nv && cl < 2 * nv) {
            const int64_t t = find(nodes, int32_t((cl - nv) / d));
            if (t < 0) {
              if (v != 0.0) bad[i] = 1;
              continue;
            }
            o.a[size_t(e0 + t) * d * d + size_t(c) * d + size_t((cl - nv) % d)] = v;
          } else if (cl >= 2 * nv && cl < 2 * nv + np) {
            o.c[size_t(c0 + atp[size_t(cl - 2 * nv)]) * d + c] = v;
          } else if (v != 0.0) {
            bad[i] = 1;
          }
        }
      }
      for (int64_t t = 0; t < nn; ++t) at[size_t(nodes[size_t(t)].first)] = -1;
      for (size_t t = 0; t < pcols.size(); ++t) atp[size_t(pcols[t])] = -1;
    }
  });
  for (int64_t i = 0; i < nQ; ++i)
    if (bad[i]) return false;
  out = std::move(o);
  return true;
}

// ------------------------------------------------------------- transfers
namespace {
// 1D interpolation weights of the coarse Q_p basis at fine lattice point g.
int interp_weights_1d(int p, int Nc, int64_t g, int64_t* cols, double* w) {
  int64_t c = g / (2 * p);
  if (c > Nc - 1) c = Nc - 1;
  double xi = double(g - 2 * p * c) / (2.0 * p);
  double v[8];
  lagrange01(p, xi, v, nullptr);
  int cnt = 0;
  for (int a = 0; a <= p; ++a)
    if (std::fabs(v[a]) > 1e-13) {
      cols[cnt] = int64_t(p) * c + a;
      w[cnt++] = v[a];
    }
  return cnt;
}
}  // namespace

namespace {
// 1D coefficient of the coarse monomial (xi_c - 1/2)^b in the child monomial (xi_f - 1/2)^a
// for the child at offset o (0: lower half, 1: upper half): xi_c - 1/2 = z/2 + (2o - 1)/4 with
// z = xi_f - 1/2, so the coefficient is binom(b, a) 2^-a ((2o - 1)/4)^(b - a) for a <= b.
double disc_child_coef(int o, int a, int b) {
  if (a > b) return 0.0;
  double binom = 1.0;
  for (int i = 0; i < a; ++i) binom = binom * (b - i) / (i + 1);
  return binom * std::ldexp(1.0, -a) * std::pow((2 * o - 1) * 0.25, b - a);
}
}  // namespace

Csr build_prolongation(const LevelHost& C, const LevelHost& F, int nthreads) {
  const int d = F.d, r = F.r;
  Csr P;
  P.nrows = F.n;
  P.ncols = C.n;
  P.ptr.assign(F.n + 1, 0);
  const auto pex = F.disc ? pdisc_exponents(r - 1, d) : std::vector<std::array<int, 3>>();
  // entries of one row (at most 3^d: the 1D weights have at most 3 nonzeros), columns ascending
  auto row_entries = [&](int64_t row, int64_t* cols, double* vals) {
    const int tn = int(row / F.ns);
    const int64_t s = row % F.ns;
    const int64_t coff = int64_t(tn) * C.ns;
    if (F.disc && s >= 2 * F.nv) {
      // broken pressure: the parent's functions restricted to the child, exactly
      const int64_t j = s - 2 * F.nv, cf = j / F.nlp;
      const auto& a = pex[j % F.nlp];
      int64_t rem = cf, cc = 0, mul = 1;
      int o[3] = {0, 0, 0};
      for (int ax = 0; ax < d; ++ax) {
        const int64_t c = rem % F.N;
        rem /= F.N;
        o[ax] = int(c % 2);
        cc += mul * (c / 2);
        mul *= C.N;
      }
      int cnt = 0;
      for (int jb = 0; jb < C.nlp; ++jb) {
        const auto& b = pex[jb];
        bool ok = true;
        double w = 1.0;
        for (int ax = 0; ax < d; ++ax) {
          if (a[ax] > b[ax]) ok = false;
          else w *= disc_child_coef(o[ax], a[ax], b[ax]);
        }
        if (!ok) continue;
        if (cols) {
          cols[cnt] = coff + 2 * C.nv + cc * C.nlp + jb;
          vals[cnt] = w;
        }
        ++cnt;
      }
      return cnt;
    }
    int p, comp, stride;
    int64_t fnode, fn1, cn1, base_col;
    if (s < 2 * F.nv) {
      const int field = s < F.nv ? 0 : 1;
      const int64_t iv = s - field * F.nv;
      p = r, fnode = iv / d, fn1 = F.n1, cn1 = C.n1, base_col = coff + field * C.nv, stride = d, comp = int(iv % d);
    } else {
      p = r - 1, fnode = s - 2 * F.nv, fn1 = F.n1p, cn1 = C.n1p, base_col = coff + 2 * C.nv, stride = 1, comp = 0;
    }
    int64_t g[3], rem = fnode;
    for (int ax = 0; ax < d; ++ax) {
      g[ax] = rem % fn1;
      rem /= fn1;
    }
    int64_t c1[3][8];
    double w1[3][8];
    int n1[3] = {1, 1, 1};
    for (int ax = 0; ax < d; ++ax) n1[ax] = interp_weights_1d(p, C.N, g[ax], c1[ax], w1[ax]);
    int cnt = 0;
    for (int iz = 0; iz < (d > 2 ? n1[2] : 1); ++iz)  // z outer, x inner
      for (int iy = 0; iy < (d > 1 ? n1[1] : 1); ++iy)
        for (int ix = 0; ix < n1[0]; ++ix) {
          int64_t node = c1[0][ix];
          double w = w1[0][ix];
          if (d > 1) {
            node += cn1 * c1[1][iy];
            w *= w1[1][iy];
          }
          if (d > 2) {
            node += cn1 * cn1 * c1[2][iz];
            w *= w1[2][iz];
          }
          if (cols) {
            cols[cnt] = base_col + stride * node + comp;
            vals[cnt] = w;
          }
          ++cnt;
        }
    return cnt;
  };
  parallel_for(F.n, nthreads, [&](int64_t lo, int64_t hi) {
    for (int64_t row = lo; row < hi; ++row) P.ptr[row + 1] = row_entries(row, nullptr, nullptr);
  });
  for (int64_t row = 0; row < F.n; ++row) P.ptr[row + 1] += P.ptr[row];
  P.col.resize(P.ptr[F.n]);
  P.val.resize(P.ptr[F.n]);
  parallel_for(F.n, nthreads, [&](int64_t lo, int64_t hi) {
    int64_t cols[64];
    double vals[64];
    for (int64_t row = lo; row < hi; ++row) {
      const int cnt = row_entries(row, cols, vals);
      for (int q = 0; q < cnt; ++q) {
        P.col[P.ptr[row] + q] = int32_t(cols[q]);
        P.val[P.ptr[row] + q] = vals[q];
      }
    }
  });
  return P;
}

Csr transpose_block_diag(const Csr& a, int64_t ncols_out, const std::vector<int64_t>& rb,
                         const std::vector<int64_t>& cb, int nthreads) {
  const int nb = int(rb.size()) - 1;
  if (int(cb.size()) != nb + 1 || rb[nb] != a.nrows || cb[nb] != a.ncols)
    throw std::runtime_error("transpose_block_diag: block ranges do not cover the matrix");
  Csr t;
  t.nrows = a.ncols;
  t.ncols = ncols_out;
  t.ptr.assign(a.ncols + 1, 0);
  std::atomic<bool> bad{false};
  auto blocks = [&](auto&& body) {
    parallel_for(int64_t(nb) * 4096, std::min(nthreads, nb), [&](int64_t lo, int64_t hi) {
      for (int64_t b = lo / 4096; b < nb && b * 4096 < hi; ++b)
        if (b * 4096 >= lo) body(int(b));
    });
  };
  blocks([&](int b) {  // counts of the columns of block b (disjoint column ranges)
    for (int64_t row = rb[b]; row < rb[b + 1]; ++row)
      for (int64_t p = a.ptr[row]; p < a.ptr[row + 1]; ++p) {
        const int64_t c = a.col[p];
        if (c < cb[b] || c >= cb[b + 1]) {
          bad = true;
          return;
        }
        t.ptr[c + 1]++;
      }
  });
  if (bad) throw std::runtime_error("transpose_block_diag: an entry lies outside its diagonal block");
  for (int64_t i = 0; i < a.ncols; ++i) t.ptr[i + 1] += t.ptr[i];
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  blocks([&](int b) {  // rows in increasing order within every column
    std::vector<int64_t> fill(t.ptr.begin() + cb[b], t.ptr.begin() + cb[b + 1]);
    for (int64_t row = rb[b]; row < rb[b + 1]; ++row)
      for (int64_t p = a.ptr[row]; p < a.ptr[row + 1]; ++p) {
        const int64_t q = fill[a.col[p] - cb[b]]++;
        t.col[q] = int32_t(row);
        t.val[q] = a.val[p];
      }
  });
  return t;
}

Csr transpose(const Csr& a, int64_t ncols_out) {
  Csr t;
  t.nrows = a.ncols;
  t.ncols = ncols_out;
  t.ptr.assign(a.ncols + 1, 0);
  for (auto c : a.col) t.ptr[c + 1]++;
  for (int64_t i = 0; i < a.ncols; ++i) t.ptr[i + 1] += t.ptr[i];
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  std::vector<int64_t> fill(t.ptr.begin(), t.ptr.end() - 1);
  for (int64_t row = 0; row < a.nrows; ++row)
    for (int64_t p = a.ptr[row]; p < a.ptr[row + 1]; ++p) {
      int64_t q = fill[a.col[p]]++;
      t.col[q] = int32_t(row);
      t.val[q] = a.val[p];
    }
  return t;
}

// ------------------------------------------------------------- closed-form sizes
namespace {
int interp_weights_1d(int p, int Nc, int64_t g, int64_t* cols, double* w);
// cells of an N-cell axis touching lattice point g of a degree-p lattice
int adj_cells(int64_t g, int p, int N) {
  if (g % p != 0) return 1;
  const int64_t c = g / p;
  return int(c - 1 >= 0) + int(c < N);
}
}  // namespace

LevelSizes level_sizes(int d, int r, int k, int N, int patch_kind, bool disc, bool dtu) {
  LevelSizes S;
  const int64_t n1 = int64_t(r) * N + 1, n1p = int64_t(r - 1) * N + 1;
  // per-axis sums over a lattice of the closure sizes of the adjacent cells
  auto axis_sum = [&](int lat_p, int64_t lat_n, int clos_p) {
    int64_t s = 0;
    for (int64_t g = 0; g < lat_n; ++g) s += int64_t(adj_cells(g, lat_p, N)) * clos_p + 1;
    return s;
  };
  const int64_t sQQ = axis_sum(r, n1, r), sQP = axis_sum(r, n1, r - 1);
  const int64_t sPP = axis_sum(r - 1, n1p, r - 1), sPQ = axis_sum(r - 1, n1p, r);
  int64_t QQ = 1, QP = 1, PP = 1, PQ = 1, nQ = 1, nP = 1;
  for (int a = 0; a < d; ++a) {
    QQ *= sQQ;
    QP *= sQP;
    PP *= sPP;
    PQ *= sPQ;
    nQ *= n1;
    nP *= n1p;
  }
  const int64_t kt = k + 1;
  int64_t PPm = PP;  // MM (c0 M_p) entries of the p-rows; PP: KK (B) entries
  int nlp = 0;
  if (disc) {
    // broken pressure: nlp functions per cell; a Q_r node's row couples the functions of its
    // adjacent cells, a pressure row the (r+1)^d nodes of its cell and, through B, the
    // functions of its cell and its face neighbours
    nlp = int(pdisc_exponents(r - 1, d).size());
    int64_t sQc = 0, cells = 1, nface = 0, Nd1 = 1, rq = 1;
    for (int64_t g = 0; g < n1; ++g) sQc += adj_cells(g, r, N);
    for (int a = 0; a < d; ++a) cells *= N;
    for (int a = 0; a < d - 1; ++a) Nd1 *= N;
    for (int a = 0; a < d; ++a) rq *= r + 1;
    nface = int64_t(d) * Nd1 * (N - 1);
    nP = cells * nlp;
    QP = nlp;
    for (int a = 0; a < d; ++a) QP *= sQc;
    PQ = cells * nlp * rq;
    PPm = cells * int64_t(nlp) * nlp;
    PP = (cells + 2 * nface) * int64_t(nlp) * nlp;
  }
  S.ns = 2 * d * nQ + nP;
  S.n = kt * S.ns;
  S.nP = nP;
  S.nodeQQ = QQ;
  S.nodeQP = QP;
  if (dtu) {
    // boundary part of C: a pressure row couples the velocity nodes of its adjacent boundary
    // cells; the union of their node boxes is counted by inclusion-exclusion
    auto is_bnd = [&](const int* c) {
      for (int a = 0; a < d; ++a)
        if (c[a] == 0 || c[a] == N - 1) return true;
      return false;
    };
    if (disc) {
      int64_t bcells = 0, cells = 1, rq = 1;
      for (int a = 0; a < d; ++a) cells *= N, rq *= r + 1;
      for (int64_t c = 0; c < cells; ++c) {
        int cc[3] = {0, 0, 0};
        int64_t rem = c;
        for (int a = 0; a < d; ++a) cc[a] = int(rem % N), rem /= N;
        bcells += is_bnd(cc);
      }
      S.nnzCface = bcells * nlp * d * rq;
    } else {
      for (int64_t j = 0; j < nP; ++j) {
        int cl[3][2], cn[3] = {1, 1, 1};
        int64_t rem = j;
        for (int a = 0; a < d; ++a) {
          const int64_t g = rem % n1p;
          rem /= n1p;
          cn[a] = 0;
          if (g % (r - 1) == 0) {
            const int64_t c = g / (r - 1);
            if (c - 1 >= 0) cl[a][cn[a]++] = int(c - 1);
            if (c < N) cl[a][cn[a]++] = int(c);
          } else {
            cl[a][cn[a]++] = int(g / (r - 1));
          }
        }
        int bl[8][3], nb = 0, combos = 1;
        for (int a = 0; a < d; ++a) combos *= cn[a];
        for (int cb = 0; cb < combos; ++cb) {
          int cc[3] = {0, 0, 0}, t = cb;
          for (int a = 0; a < d; ++a) cc[a] = cl[a][t % cn[a]], t /= cn[a];
          if (is_bnd(cc)) {
            for (int a = 0; a < 3; ++a) bl[nb][a] = cc[a];
            ++nb;
          }
        }
        int64_t uni = 0;
        for (int sub = 1; sub < (1 << nb); ++sub) {
          int64_t vol = 1;
          int bits = 0;
          for (int a = 0; a < d; ++a) {
            int lo = -(1 << 30), hi = 1 << 30;
            for (int q = 0; q < nb; ++q)
              if (sub >> q & 1) {
                lo = std::max(lo, r * bl[q][a]);
                hi = std::min(hi, r * (bl[q][a] + 1));
              }
            vol *= std::max(0, hi - lo + 1);
          }
          for (int q = 0; q < nb; ++q) bits += sub >> q & 1;
          uni += (bits % 2 ? 1 : -1) * vol;
        }
        S.nnzCface += uni * d;
      }
    }
  }
  // u-eq rows: MM (M_rho on U) and KK (-M_rho on V), same component, disjoint columns
  // v-eq rows: MM (M_rho on V, same comp); KK (A on U, all comps; C^T on P)
  // p-eq rows: MM (c0 M_p on P); KK (-C on V, all comps; B on P, same columns as MM)
  const int64_t u_rows = kt * d * (kt + 1) * QQ;
  const int64_t v_rows = kt * d * ((kt + d) * QQ + QP);
  // Problem B.1 moves -C from KK (on V) to MM (on U): the same union on the diagonal time
  // block, and d PQ more entries in every off-diagonal one
  const int64_t p_rows = kt * ((kt - 1) * (PPm + (dtu ? d * PQ : 0)) + PP + d * PQ);
  S.nnzA = u_rows + v_rows + p_rows;
  S.nnzMM = 2 * d * QQ + PPm + (dtu ? d * PQ : 0);
  S.nnzKK = d * QQ + d * (d * QQ + QP) + ((dtu ? 0 : d * PQ) + PP);
  // prolongation from N/2 cells: nonzero 1D interpolation weights per fine lattice point
  if (N % 2 == 0) {
    auto pro_sum = [&](int p) {
      int64_t s = 0, cols[8];
      double w[8];
      for (int64_t g = 0; g <= int64_t(p) * N; ++g) s += interp_weights_1d(p, N / 2, g, cols, w);
      return s;
    };
    const int64_t a = pro_sum(r), b = pro_sum(r - 1);
    int64_t A = 1, B = 1;
    for (int x = 0; x < d; ++x) {
      A *= a;
      B *= b;
    }
    if (disc) {
      // per fine cell: the pairs (alpha, beta) with alpha <= beta componentwise
      const auto ex = pdisc_exponents(r - 1, d);
      int64_t pairs = 0, cells = 1;
      for (const auto& x : ex)
        for (const auto& y : ex) pairs += (x[0] <= y[0] && x[1] <= y[1] && x[2] <= y[2]) ? 1 : 0;
      for (int x = 0; x < d; ++x) cells *= N;
      B = cells * pairs;
    }
    S.nnzP = kt * (2 * d * A + B);
  }
  // patches: per axis a patch spans 1 or 2 cells; enumerate the 2^d width classes
  int64_t cnt1 = 0, cnt2 = 0;  // per axis: patches (vertices or cells) of width 1 / 2
  if (patch_kind == 1) {
    cnt2 = N - 1;
    cnt1 = N >= 1 ? 2 : 0;
    if (N == 1) {
      cnt1 = 2;
      cnt2 = 0;
    }
  } else {
    cnt1 = N;
  }
  for (int mask = 0; mask < (1 << d); ++mask) {
    int64_t mult = 1, q = 1, pp = 1, pc = 1;
    for (int a = 0; a < d; ++a) {
      const int w = (mask >> a) & 1 ? 2 : 1;
      mult *= (w == 2 ? cnt2 : cnt1);
      q *= int64_t(r) * w + 1;
      pp *= int64_t(r - 1) * w + 1;
      pc *= w;
    }
    if (mult == 0) continue;
    if (disc) pp = pc * nlp;
    const int64_t np = kt * (2 * d * q + pp);
    const int64_t nsp = 2 * d * q + pp;
    S.sum_ns_ldh += mult * nsp * ((nsp + 3) & ~int64_t(3));
    S.npatch += mult;
    S.sum_np += mult * np;
    S.sum_np_ld += mult * np * ((np + 3) & ~int64_t(3));
    S.max_np = std::max<int>(S.max_np, int(np));
    const int64_t nU = d * q, nr = nU + pp;
    auto ld4 = [](int64_t v) { return (v + 3) & ~int64_t(3); };
    S.sum_red_fixed += mult * (q * ld4(q) + nU * ld4(pp));
    S.sum_nr_ldr += mult * nr * ld4(nr);
    S.alg_red_fixed += mult * (q * q + pp * nU);
    S.sum_nr2 += mult * nr * nr;
    S.sum_tiles += mult * sym_tiles(int(nr));
    S.sum_tiles2 += mult * sym_slots(int(nr), 2);
    S.sum_tiles4 += mult * sym_slots(int(nr), 4);
    S.max_nr = std::max<int>(S.max_nr, int(nr));
    S.max_nn = std::max<int>(S.max_nn, int(q));
  }
  return S;
}

// ------------------------------------------------------------- built-in solution
// u_i = S sin t, v_i = S cos t, p = S cos t, S = prod_j sin(pi x_j).
// f_i = rho u_tt - div sigma(u) + alpha d_i p
//     = [-rho S + mu d pi^2 S - (mu + lambda) sum_c d_i d_c S] sin t + alpha d_i S cos t
// g   = c0 p_t + alpha div v - K lap p = -c0 S sin t + alpha sum_c d_c S cos t + K d pi^2 S cos t
void source_vector(const LevelHost& L, const Material& m, double t, std::vector<double>& out) {
  const int d = L.d, r = L.r, N = L.N;
  const double h = 1.0 / N;
  out.assign(L.ns, 0.0);
  std::vector<double> gx, gw;
  gauss_legendre01(r + 2, gx, gw);
  const int nq1 = r + 2;
  int nq = 1;
  for (int a = 0; a < d; ++a) nq *= nq1;
  // tabulate once (reference coordinates are identical in every cell)
  std::vector<Tab> ts(nq), tp(nq);
  std::vector<double> wq(nq);
  std::vector<std::array<double, 3>> xq(nq);
  for (int q = 0; q < nq; ++q) {
    double xi[3] = {0, 0, 0}, w = 1.0;
    int rem = q;
    for (int ax = 0; ax < d; ++ax) {
      xi[ax] = gx[rem % nq1];
      w *= gw[rem % nq1] * h;
      rem /= nq1;
    }
    tabulate(r, d, xi, h, ts[q]);
    tabulate_p(L.disc, r, d, xi, h, tp[q]);
    wq[q] = w;
    xq[q] = {xi[0], xi[1], xi[2]};
  }
  const double st = std::sin(t), ct = std::cos(t), pi = M_PI;
  int64_t ncells = 1;
  for (int a = 0; a < d; ++a) ncells *= N;
  const int nls = ts[0].nl, nlp = tp[0].nl;
  // cells are split into a fixed number of contiguous chunks, each accumulated
  // into its own vector and summed in chunk order: the result does not depend on
  // the number of threads
  const int nchunk = ncells >= 4096 ? 16 : 1;
  std::vector<std::vector<double>> part(nchunk);
  auto work = [&](int ch) {
    std::vector<double>& acc = part[ch];
    acc.assign(L.ns, 0.0);
    const int64_t c_lo = ncells * ch / nchunk, c_hi = ncells * (ch + 1) / nchunk;
    for (int64_t cell = c_lo; cell < c_hi; ++cell) {
      int cc[3] = {0, 0, 0};
      int64_t rem = cell;
      for (int ax = 0; ax < d; ++ax) {
        cc[ax] = int(rem % N);
        rem /= N;
      }
      const double K = L.Kcell[cell];
      for (int q = 0; q < nq; ++q) {
        double sn[3] = {1, 1, 1}, cs[3] = {0, 0, 0};
        for (int ax = 0; ax < d; ++ax) {
          double x = (cc[ax] + xq[q][ax]) * h;
          sn[ax] = std::sin(pi * x);
          cs[ax] = std::cos(pi * x);
        }
        double S = 1.0, dS[3], ddS[3][3];
        for (int ax = 0; ax < d; ++ax) S *= sn[ax];
        for (int i = 0; i < d; ++i) {
          dS[i] = pi * cs[i];
          for (int j = 0; j < d; ++j)
            if (j != i) dS[i] *= sn[j];
          for (int j = 0; j < d; ++j) {
            if (i == j) {
              ddS[i][j] = -pi * pi * S;
            } else {
              double v = pi * pi * cs[i] * cs[j];
              for (int l = 0; l < d; ++l)
                if (l != i && l != j) v *= sn[l];
              ddS[i][j] = v;
            }
          }
        }
        double f[3];
        for (int i = 0; i < d; ++i) {
          double sum = 0.0;
          for (int c = 0; c < d; ++c) sum += ddS[i][c];
          f[i] = (-m.rho * S + m.mu * d * pi * pi * S - (m.mu + m.lambda) * sum) * st + m.alpha * dS[i] * ct;
        }
        double divS = 0.0;
        for (int c = 0; c < d; ++c) divS += dS[c];
        const double g = -m.c0 * S * st + m.alpha * divS * ct + K * d * pi * pi * S * ct;
        for (int a = 0; a < nls; ++a) {
          int64_t gn = 0;
          int idx[3], rm = a;
          for (int ax = 0; ax < d; ++ax) {
            idx[ax] = rm % (r + 1);
            rm /= (r + 1);
          }
          for (int ax = d - 1; ax >= 0; --ax) gn = gn * L.n1 + (int64_t(r) * cc[ax] + idx[ax]);
          for (int c = 0; c < d; ++c) acc[L.nv + d * gn + c] += wq[q] * ts[q].v[a] * f[c];
        }
        for (int s = 0; s < nlp; ++s) {
          int64_t gn = 0;
          if (L.disc) {
            gn = cell * nlp + s;
          } else {
            int idx[3], rm = s;
            for (int ax = 0; ax < d; ++ax) {
              idx[ax] = rm % r;
              rm /= r;
            }
            for (int ax = d - 1; ax >= 0; --ax) gn = gn * L.n1p + (int64_t(r - 1) * cc[ax] + idx[ax]);
          }
          acc[2 * L.nv + gn] += wq[q] * tp[q].v[s] * g;
        }
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int ch = 1; ch < nchunk; ++ch) th.emplace_back(work, ch);
    work(0);
    for (auto& x : th) x.join();
  }
  out = std::move(part[0]);
  for (int ch = 1; ch < nchunk; ++ch)
    for (int64_t i = 0; i < L.ns; ++i) out[i] += part[ch][i];
}

void source_tables(int d, int r, std::vector<double>& xq, std::vector<double>& wq, std::vector<double>& bq,
                   std::vector<double>& bp, bool disc) {
  std::vector<double> gx, gw;
  gauss_legendre01(r + 2, gx, gw);
  const int nq1 = r + 2;
  int nq = 1;
  for (int a = 0; a < d; ++a) nq *= nq1;
  xq.assign(3 * nq, 0.0);
  wq.assign(nq, 1.0);
  Tab ts, tp;
  int nls = 1, nlp = 1;
  for (int a = 0; a < d; ++a) {
    nls *= r + 1;
    nlp *= r;
  }
  if (disc) nlp = int(pdisc_exponents(r - 1, d).size());
  bq.assign(size_t(nls) * nq, 0.0);
  bp.assign(size_t(nlp) * nq, 0.0);
  for (int q = 0; q < nq; ++q) {
    double xi[3] = {0, 0, 0};
    int rem = q;
    for (int ax = 0; ax < d; ++ax) {
      xi[ax] = gx[rem % nq1];
      wq[q] *= gw[rem % nq1];
      rem /= nq1;
      xq[3 * q + ax] = xi[ax];
    }
    tabulate(r, d, xi, 1.0, ts);
    tabulate_p(disc, r, d, xi, 1.0, tp);
    for (int a = 0; a < nls; ++a) bq[size_t(a) * nq + q] = ts.v[a];
    for (int a = 0; a < nlp; ++a) bp[size_t(a) * nq + q] = tp.v[a];
  }
}

void interpolate_solution(const LevelHost& L, double t, std::vector<double>& out) {
  const int d = L.d;
  out.assign(L.ns, 0.0);
  auto S_at = [&](int64_t node, int64_t n1, int p) {
    double S = 1.0;
    int64_t rem = node;
    for (int ax = 0; ax < d; ++ax) {
      double x = double(rem % n1) / (double(p) * L.N);
      rem /= n1;
      S *= std::sin(M_PI * x);
    }
    return S;
  };
  for (int64_t q = 0; q < L.nQ; ++q) {
    double S = S_at(q, L.n1, L.r);
    for (int c = 0; c < d; ++c) {
      out[d * q + c] = S * std::cos(t);
      out[L.nv + d * q + c] = S * std::sin(t);
    }
  }
  if (!L.disc) {
    for (int64_t q = 0; q < L.nP; ++q) out[2 * L.nv + q] = S_at(q, L.n1p, L.r - 1) * std::cos(t);
    return;
  }
  // broken pressure: the L2 projection onto P_{r-1} of each cell ((r+2)^d Gauss points);
  // the cell mass matrix is the same in every cell (reference coordinates)
  const int nlp = L.nlp, nq1 = L.r + 2;
  std::vector<double> gx, gw;
  gauss_legendre01(nq1, gx, gw);
  int nq = 1;
  for (int a = 0; a < d; ++a) nq *= nq1;
  std::vector<Tab> tp(nq);
  std::vector<double> wq(nq, 1.0), M(size_t(nlp) * nlp, 0.0);
  std::vector<std::array<double, 3>> xq(nq);
  for (int q = 0; q < nq; ++q) {
    double xi[3] = {0, 0, 0};
    int rem = q;
    for (int ax = 0; ax < d; ++ax) {
      xi[ax] = gx[rem % nq1];
      wq[q] *= gw[rem % nq1];
      rem /= nq1;
    }
    xq[q] = {xi[0], xi[1], xi[2]};
    tabulate_pdisc(L.r - 1, d, xi, 1.0, tp[q]);
    for (int i = 0; i < nlp; ++i)
      for (int j = 0; j < nlp; ++j) M[size_t(i) * nlp + j] += wq[q] * tp[q].v[i] * tp[q].v[j];
  }
  // Cholesky of the (symmetric positive definite) reference mass
  std::vector<double> Lc(M);
  for (int j = 0; j < nlp; ++j) {
    for (int kk = 0; kk < j; ++kk)
      for (int i = j; i < nlp; ++i) Lc[size_t(i) * nlp + j] -= Lc[size_t(i) * nlp + kk] * Lc[size_t(j) * nlp + kk];
    const double dj = std::sqrt(Lc[size_t(j) * nlp + j]);
    for (int i = j; i < nlp; ++i) Lc[size_t(i) * nlp + j] /= dj;
  }
  int64_t ncells = 1;
  for (int a = 0; a < d; ++a) ncells *= L.N;
  const double h = 1.0 / L.N;
  std::vector<double> rhs(nlp);
  for (int64_t cell = 0; cell < ncells; ++cell) {
    int cc[3] = {0, 0, 0};
    int64_t rem = cell;
    for (int ax = 0; ax < d; ++ax) {
      cc[ax] = int(rem % L.N);
      rem /= L.N;
    }
    std::fill(rhs.begin(), rhs.end(), 0.0);
    for (int q = 0; q < nq; ++q) {
      double S = 1.0;
      for (int ax = 0; ax < d; ++ax) S *= std::sin(M_PI * (cc[ax] + xq[q][ax]) * h);
      for (int i = 0; i < nlp; ++i) rhs[i] += wq[q] * tp[q].v[i] * S;
    }
    for (int i = 0; i < nlp; ++i) {  // forward
      for (int kk = 0; kk < i; ++kk) rhs[i] -= Lc[size_t(i) * nlp + kk] * rhs[kk];
      rhs[i] /= Lc[size_t(i) * nlp + i];
    }
    for (int i = nlp - 1; i >= 0; --i) {  // backward
      for (int kk = i + 1; kk < nlp; ++kk) rhs[i] -= Lc[size_t(kk) * nlp + i] * rhs[kk];
      rhs[i] /= Lc[size_t(i) * nlp + i];
    }
    for (int i = 0; i < nlp; ++i) out[2 * L.nv + cell * nlp + i] = rhs[i] * std::cos(t);
  }
}

}  // namespace stgmg
