// Host-side construction of grids, tables and the FP64 factorization of the implicit
// operator.  All formulas are restated from the paper (arXiv 2508.16635):
//  * radial Chebyshev expansion in x = (2r - (r_o + r_i))/(r_o - r_i), collocation at the
//    Gauss-Lobatto nodes, 3/2-rule dealiasing in r (Sec. 3.1);
//  * Y_l^m = N_l^m P_l^m(cos th) e^{i m phi}, N_l^m = sqrt((2 - d_m0)(2l+1)(l-m)!/(l+m)!)
//    (Sec. 3.2, normalization after the Legendre recursions);
//  * implicit operator (M - dt K) with the Coriolis coupling of l to l +- 1 (Sec. 3.2,
//    e- and f-equations after applying the recursions), boundary rows replaced (Sec. 3.1).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace sc {

namespace {

const double kPi = 3.14159265358979323846;

int smooth235(int n) {
  if (n < 1) n = 1;
  for (;; ++n) {
    int k = n;
    for (int p : {2, 3, 5})
      while (k % p == 0) k /= p;
    if (k == 1) return n;
  }
}

std::vector<double> matmul(const std::vector<double>& A, const std::vector<double>& B, int n, int k, int m) {
  std::vector<double> C((size_t)n * m, 0.0);
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < k; ++q) {
      double a = A[(size_t)i * k + q];
      if (a == 0.0) continue;
      for (int j = 0; j < m; ++j) C[(size_t)i * m + j] += a * B[(size_t)q * m + j];
    }
  return C;
}

// Barycentric weights of the Chebyshev-Gauss-Lobatto nodes: (-1)^j, halved at the ends.
double bary_w(int j, int n) { return ((j % 2) ? -1.0 : 1.0) * ((j == 0 || j == n - 1) ? 0.5 : 1.0); }

// Differentiation matrix on n Gauss-Lobatto nodes (in x), from the barycentric formula
// D_ij = (w_j/w_i)/(x_i - x_j), diagonal by the negative row sum.
std::vector<double> cheb_diff_x(const std::vector<double>& x) {
  int n = (int)x.size();
  std::vector<double> D((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double v = (bary_w(j, n) / bary_w(i, n)) / (x[i] - x[j]);
      D[(size_t)i * n + j] = v;
      s += v;
    }
    D[(size_t)i * n + i] = -s;
  }
  return D;
}

// Barycentric interpolation matrix from the n-node Gauss-Lobatto set xs to points xt.
std::vector<double> bary_interp(const std::vector<double>& xs, const std::vector<double>& xt) {
  int n = (int)xs.size(), m = (int)xt.size();
  std::vector<double> E((size_t)m * n, 0.0);
  for (int i = 0; i < m; ++i) {
    int hit = -1;
    for (int j = 0; j < n; ++j)
      if (std::fabs(xt[i] - xs[j]) < 1e-15) hit = j;
    if (hit >= 0) {
      E[(size_t)i * n + hit] = 1.0;
      continue;
    }
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += bary_w(j, n) / (xt[i] - xs[j]);
    for (int j = 0; j < n; ++j) E[(size_t)i * n + j] = bary_w(j, n) / (xt[i] - xs[j]) / den;
  }
  return E;
}

// Gauss-Legendre nodes x_j = cos(theta_j) (descending), weights and sin(theta_j), computed in
// the host's extended precision (long double) and rounded once.  Newton's iteration runs on theta
// (northern half; the southern nodes by symmetry).  Next to the poles (x > 1/2) P_n(cos theta)
// comes from the three-term recurrence written for the differences d_k = P_k - P_(k-1), driven
// by y = 1 - x = 2 sin^2(theta/2): d_(k+1) = (k d_k - (2k+1) y P_k)/(k+1), P_(k+1) = P_k + d_(k+1);
// elsewhere from the plain one.  Nothing depends on 1 - x^2 formed from a rounded x, which loses
// digits next to the poles: sin(theta) comes from theta, and at a root of P_n the weight is
// w = 2 (1 - x^2) / (n P_(n-1))^2 = 2 sin^2(theta) / (n P_(n-1))^2.
typedef long double ld_t;

static void legendre_pair(int n, ld_t th, ld_t& pn, ld_t& pn1) {
  const ld_t sh = std::sin(0.5L * th), y = 2.0L * sh * sh, x = std::cos(th);
  ld_t prev = 1.0L, cur = 1.0L - y, d = -y;   // P_0, P_1, P_1 - P_0
  for (int k = 1; k < n; ++k) {
    ld_t dn;
    if (y < 0.5L) dn = (k * d - (2.0L * k + 1.0L) * y * cur) / (k + 1.0L);
    else dn = ((2.0L * k + 1.0L) * x * cur - k * prev) / (k + 1.0L) - cur;
    prev = cur;
    cur += dn;
    d = dn;
  }
  pn = cur;     // P_n
  pn1 = prev;   // P_(n-1)
}

void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w, std::vector<double>& st) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  st.assign(n, 0.0);
  const ld_t pi = 3.14159265358979323846264338327950288L;
  for (int i = 0; i < (n + 1) / 2; ++i) {
    ld_t th = pi * (i + 0.75L) / (n + 0.5L);
    ld_t pn = 0.0L, pn1 = 0.0L;
    for (int it = 0; it < 100; ++it) {
      legendre_pair(n, th, pn, pn1);
      const ld_t dth = n * (std::cos(th) * pn - pn1) / std::sin(th);   // dP_n/dtheta
      const ld_t step = pn / dth;
      th -= step;
      if (std::fabs(step) <= 1e-18L * th) break;
    }
    legendre_pair(n, th, pn, pn1);
    const ld_t s = std::sin(th), q = n * pn1;
    x[i] = (double)std::cos(th);
    st[i] = (double)s;
    w[i] = (double)(2.0L * s * s / (q * q));
    x[n - 1 - i] = -x[i];
    st[n - 1 - i] = st[i];
    w[n - 1 - i] = w[i];
  }
  if (n % 2) x[n / 2] = 0.0;   // the equatorial node of an odd rule
}

}  // namespace

void build_grid(HostGrid& g, int L, int M, int m0, int N, double eta, int Np, int nth, int nphi) {
  if (L < 1 || m0 < 1 || M < 0 || N < 6 || !(eta > 0.0 && eta < 1.0))
    throw std::runtime_error("bad truncation or radius ratio");
  g.L = L;
  g.M = M;
  g.m0 = m0;
  g.N = N;
  g.K = std::min(M, L) / m0;
  g.Np = Np > 0 ? Np : (3 * N + 1) / 2;
  int t = (3 * L + 2) / 2;  // ceil((3L+1)/2)
  t += t % 2;
  g.nth = nth > 0 ? nth : t;
  g.nphi = nphi > 0 ? nphi : smooth235(3 * g.K + 1);
  if (g.Np < N || g.nth < L + 1 || g.nphi < 2 * g.K + 1) throw std::runtime_error("grid too small");
  g.ro = 1.0 / (1.0 - eta);
  g.ri = g.ro - 1.0;
  g.ms.clear();
  g.nl.clear();
  g.lmbase.clear();
  g.lm_k.clear();
  g.lm_l.clear();
  int s = 0;
  for (int k = 0; k <= g.K; ++k) {
    int m = k * m0;
    g.ms.push_back(m);
    g.nl.push_back(L - m + 1);
    g.lmbase.push_back(s);
    for (int l = m; l <= L; ++l) {
      g.lm_k.push_back(k);
      g.lm_l.push_back(l);
    }
    s += L - m + 1;
  }
  g.S = s;

  // radial nodes: r = ((ro - ri) x + ro + ri)/2, d/dr = 2/(ro - ri) d/dx
  auto nodes = [](int n) {
    std::vector<double> x(n);
    for (int j = 0; j < n; ++j) x[j] = std::cos(kPi * j / (n - 1));
    return x;
  };
  g.x = nodes(N);
  g.xp = nodes(g.Np);
  double gap = g.ro - g.ri;
  g.r.resize(N);
  g.rp.resize(g.Np);
  for (int j = 0; j < N; ++j) g.r[j] = (gap * g.x[j] + g.ro + g.ri) / 2.0;
  for (int j = 0; j < g.Np; ++j) g.rp[j] = (gap * g.xp[j] + g.ro + g.ri) / 2.0;
  g.D = cheb_diff_x(g.x);
  for (auto& v : g.D) v *= 2.0 / gap;
  g.Dp = cheb_diff_x(g.xp);
  for (auto& v : g.Dp) v *= 2.0 / gap;
  g.D2 = matmul(g.D, g.D, N, N, N);
  g.D4 = matmul(g.D2, g.D2, N, N, N);
  g.E = bary_interp(g.x, g.xp);
  g.ED = matmul(g.E, g.D, g.Np, N, N);
  g.ED2 = matmul(g.E, g.D2, g.Np, N, N);
  // P: Chebyshev transform on the Np nodes truncated to the first N modes, evaluated at the
  // N nodes.  Coefficients a_k = 2/((Np-1) cb_k) sum_j v_j cos(pi j k/(Np-1)) / cb_j.
  g.P.assign((size_t)N * g.Np, 0.0);
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < g.Np; ++j) {
      double cbj = (j == 0 || j == g.Np - 1) ? 2.0 : 1.0;
      double acc = 0.0;
      for (int k = 0; k < N; ++k) {
        double cbk = (k == 0 || k == g.Np - 1) ? 2.0 : 1.0;
        acc += std::cos(kPi * i * k / (N - 1)) * 2.0 / ((g.Np - 1) * cbk * cbj) * std::cos(kPi * j * k / (g.Np - 1));
      }
      g.P[(size_t)i * g.Np + j] = acc;
    }

  // angular grid and normalized associated Legendre functions (no Condon-Shortley phase)
  gauss_legendre(g.nth, g.ct, g.wt, g.st);
  g.Pb.assign(g.K + 1, {});
  g.dPb.assign(g.K + 1, {});
  g.mPs.assign(g.K + 1, {});
  for (int k = 0; k <= g.K; ++k) {
    int m = g.ms[k];
    int nl = g.nl[k];
    std::vector<double>& Pb = g.Pb[k];
    std::vector<double>& dP = g.dPb[k];
    std::vector<double>& mP = g.mPs[k];
    Pb.assign((size_t)nl * g.nth, 0.0);
    dP.assign((size_t)nl * g.nth, 0.0);
    mP.assign((size_t)nl * g.nth, 0.0);
    double fac = (m == 0) ? 1.0 : std::sqrt(2.0);
    for (int j = 0; j < g.nth; ++j) {
      double xx = g.ct[j], ss = g.st[j];
      // sectoral seed q_m^m = sqrt((2m+1)!!/(2m)!!) sin^m (unit-normalized without the (2-d) factor)
      double q = 1.0;
      for (int i = 1; i <= m; ++i) q *= std::sqrt((2.0 * i + 1.0) / (2.0 * i)) * ss;
      std::vector<double> p(nl + 1, 0.0);  // q_l^m for l = m .. L+1
      p[0] = q;
      if (nl >= 1) p[1] = std::sqrt(2.0 * m + 3.0) * xx * q;
      for (int i = 2; i <= nl; ++i) {
        int l = m + i;
        double a = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
        double b = std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
        p[i] = a * (xx * p[i - 1] - b * p[i - 2]);
      }
      for (int i = 0; i < nl; ++i) {
        int l = m + i;
        double pl = fac * p[i], pl1 = fac * p[i + 1];
        Pb[(size_t)i * g.nth + j] = pl;
        mP[(size_t)i * g.nth + j] = m * pl / ss;
        // sin(th) dP_l/dth = -(l+1) x P_l + (l-m+1) P_{l+1} (unnormalized); normalized factor
        // (l-m+1) N_l/N_{l+1} = sqrt((2l+1)((l+1)^2 - m^2)/(2l+3)).
        double c = std::sqrt((2.0 * l + 1.0) * ((l + 1.0) * (l + 1.0) - (double)m * m) / (2.0 * l + 3.0));
        dP[(size_t)i * g.nth + j] = (-(l + 1.0) * xx * pl + c * pl1) / ss;
      }
    }
  }
}

// ------------------------------------------------------------------------------------------
// Implicit operator blocks and their factorization.
namespace {

double kappa(int l, int m) {
  // Coefficient of the l-1 neighbour in row l of the implicit Coriolis terms:
  // (l-1)(l+1)(l-|m|)/(2l-1) * N_{l-1}^m / N_l^m = (l^2-1) sqrt((l^2-m^2)/(4l^2-1)).
  m = std::abs(m);
  if (l <= 1 || l <= m) return 0.0;
  double ll = l;
  return (ll * ll - 1.0) * std::sqrt((ll * ll - (double)m * m) / (4.0 * ll * ll - 1.0));
}

struct Blocks {
  int N;
  const HostGrid* g;
  OpParams op;
  // A = M - dt K for the self block of field t (0 = e, 1 = f) at (l, m), BC rows applied.
  std::vector<cplx> self(int t, int l, int m) const {
    const HostGrid& G = *g;
    std::vector<cplx> A((size_t)N * N, 0.0);
    double lam = (double)l * (l + 1);
    for (int i = 0; i < N; ++i) {
      double r = G.r[i], r2 = r * r;
      double a = op.Ek * lam / r2;        // Ek lambda / r^2
      cplx cor(0.0, op.cor * 2.0 * m / r2);   // 2 i m / r^2 (0 in the explicit-Coriolis variant)
      for (int j = 0; j < N; ++j) {
        double Lij = G.D2[(size_t)i * N + j] - (i == j ? lam / r2 : 0.0);   // L_l
        cplx v;
        if (t == 0) {
          // M_e - dt K_e:  a e - dt (a L e + cor e)
          v = (i == j ? a : 0.0) - op.dt * (a * Lij + (i == j ? cor : cplx(0.0)));
        } else {
          // M_f - dt K_f: -a L f - dt(-a L^2 f - cor L f)
          double L2ij = 0.0;
          for (int q = 0; q < N; ++q) {
            double Liq = G.D2[(size_t)i * N + q] - (i == q ? lam / r2 : 0.0);
            double rq = G.r[q];
            double Lqj = G.D2[(size_t)q * N + j] - (q == j ? lam / (rq * rq) : 0.0);
            L2ij += Liq * Lqj;
          }
          v = -a * Lij - op.dt * (-a * L2ij - cor * Lij);
        }
        A[(size_t)i * N + j] = v;
      }
    }
    bc_self(A, t);
    return A;
  }
  // -dt K_couple of row l to neighbour l+nb (acting on the other potential), BC rows zeroed.
  std::vector<cplx> couple(int t, int l, int m, int nb) const {
    const HostGrid& G = *g;
    std::vector<cplx> B((size_t)N * N, 0.0);
    double kap = (nb < 0) ? kappa(l, m) : kappa(l + 1, m);
    double c = (nb < 0) ? (double)l : -(l + 1.0);  // (c/r - d_r)
    for (int i = 0; i < N; ++i) {
      double r = G.r[i];
      // K_couple = -(2/r^2) kap (c/r - D);  -dt K_couple = dt (2/r^2) kap (c/r - D)
      double pre = op.cor * op.dt * 2.0 / (r * r) * kap;
      for (int j = 0; j < N; ++j) B[(size_t)i * N + j] = pre * ((i == j ? c / r : 0.0) - G.D[(size_t)i * N + j]);
    }
    for (int row : bc_rows(t)) std::fill(B.begin() + (size_t)row * N, B.begin() + (size_t)(row + 1) * N, cplx(0.0));
    return B;
  }
  std::vector<int> bc_rows(int t) const {
    if (t == 0) return {0, N - 1};
    return {0, 1, N - 2, N - 1};
  }
  void bc_self(std::vector<cplx>& A, int t) const {
    for (int row : bc_rows(t)) std::fill(A.begin() + (size_t)row * N, A.begin() + (size_t)(row + 1) * N, cplx(0.0));
    A[0] = 1.0;
    A[(size_t)(N - 1) * N + N - 1] = 1.0;
    if (t == 1) {
      for (int j = 0; j < N; ++j) {
        A[(size_t)1 * N + j] = g->D[j];                          // d_r f = 0 at r_o
        A[(size_t)(N - 2) * N + j] = g->D[(size_t)(N - 1) * N + j];  // d_r f = 0 at r_i
      }
    }
  }
};

// In-place inverse by Gauss-Jordan elimination with partial pivoting (complex or real).
template <class T>
void invert(std::vector<T>& A, int n) {
  std::vector<T> inv((size_t)n * n, T(0.0));
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = T(1.0);
  for (int c = 0; c < n; ++c) {
    int piv = c;
    double best = std::abs(A[(size_t)c * n + c]);
    for (int r = c + 1; r < n; ++r)
      if (std::abs(A[(size_t)r * n + c]) > best) {
        best = std::abs(A[(size_t)r * n + c]);
        piv = r;
      }
    if (best == 0.0) throw std::runtime_error("singular block");
    if (piv != c)
      for (int j = 0; j < n; ++j) {
        std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
        std::swap(inv[(size_t)c * n + j], inv[(size_t)piv * n + j]);
      }
    T d = T(1.0) / A[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) {
      A[(size_t)c * n + j] *= d;
      inv[(size_t)c * n + j] *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      T f = A[(size_t)r * n + c];
      if (f == T(0.0)) continue;
      for (int j = 0; j < n; ++j) {
        A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
        inv[(size_t)r * n + j] -= f * inv[(size_t)c * n + j];
      }
    }
  }
  A.swap(inv);
}

// Ruiz equilibration of a dense block: returns row/column scalings with max |entries| -> 1.
template <class T>
void ruiz_dense(const std::vector<T>& A, int n, std::vector<double>& R, std::vector<double>& C) {
  R.assign(n, 1.0);
  C.assign(n, 1.0);
  std::vector<double> rm(n), cm(n);
  for (int it = 0; it < 40; ++it) {
    std::fill(rm.begin(), rm.end(), 0.0);
    std::fill(cm.begin(), cm.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double a = std::abs(A[(size_t)i * n + j]) * R[i] * C[j];
        rm[i] = std::max(rm[i], a);
        cm[j] = std::max(cm[j], a);
      }
    double dev = 0.0;
    for (int i = 0; i < n; ++i) {
      dev = std::max(dev, std::fabs(rm[i] - 1.0));
      dev = std::max(dev, std::fabs(cm[i] - 1.0));
      R[i] /= std::sqrt(rm[i]);
      C[i] /= std::sqrt(cm[i]);
    }
    if (dev < 1e-3) break;
  }
}

void factor_chain(const Blocks& B, const HostGrid& g, int k, int cls, ChainFactor& cf) {
  const int N = g.N;
  int m = g.ms[k];
  cf.k = k;
  cf.m = m;
  cf.cls = cls;
  cf.l0 = std::max(m, 1);
  cf.n = g.L - cf.l0 + 1;
  int n = cf.n;
  cf.field.resize(n);
  cf.l.resize(n);
  for (int i = 0; i < n; ++i) {
    cf.l[i] = cf.l0 + i;
    cf.field[i] = ((i % 2 == 0) ? (cls == 0 ? 0 : 1) : (cls == 0 ? 1 : 0));
  }
  if (n <= 0) return;
  std::vector<std::vector<cplx>> Dg(n), Lo(n), Up(n);
  for (int i = 0; i < n; ++i) {
    Dg[i] = B.self(cf.field[i], cf.l[i], m);
    if (i > 0) Lo[i] = B.couple(cf.field[i], cf.l[i], m, -1);
    if (i < n - 1) Up[i] = B.couple(cf.field[i], cf.l[i], m, +1);
  }
  // global Ruiz equilibration of the chain
  std::vector<double> R((size_t)n * N, 1.0), C((size_t)n * N, 1.0), rm((size_t)n * N), cm((size_t)n * N);
  for (int it = 0; it < 40; ++it) {
    std::fill(rm.begin(), rm.end(), 0.0);
    std::fill(cm.begin(), cm.end(), 0.0);
    auto acc = [&](const std::vector<cplx>& blk, int bi, int bj) {
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          double a = std::abs(blk[(size_t)i * N + j]) * R[(size_t)bi * N + i] * C[(size_t)bj * N + j];
          rm[(size_t)bi * N + i] = std::max(rm[(size_t)bi * N + i], a);
          cm[(size_t)bj * N + j] = std::max(cm[(size_t)bj * N + j], a);
        }
    };
    for (int i = 0; i < n; ++i) {
      acc(Dg[i], i, i);
      if (i > 0) acc(Lo[i], i, i - 1);
      if (i < n - 1) acc(Up[i], i, i + 1);
    }
    double dev = 0.0;
    for (size_t q = 0; q < R.size(); ++q) {
      dev = std::max(dev, std::max(std::fabs(rm[q] - 1.0), std::fabs(cm[q] - 1.0)));
      R[q] /= std::sqrt(rm[q]);
      C[q] /= std::sqrt(cm[q]);
    }
    if (dev < 1e-3) break;
  }
  auto scale = [&](std::vector<cplx>& blk, int bi, int bj) {
    for (int i = 0; i < N; ++i)
      for (int j = 0; j < N; ++j) blk[(size_t)i * N + j] *= R[(size_t)bi * N + i] * C[(size_t)bj * N + j];
  };
  for (int i = 0; i < n; ++i) {
    scale(Dg[i], i, i);
    if (i > 0) scale(Lo[i], i, i - 1);
    if (i < n - 1) scale(Up[i], i, i + 1);
  }
  cf.Rg = R;
  cf.Cg = C;
  cf.Sinv.assign((size_t)n * N * N, 0.0);
  cf.Lo.assign((size_t)n * N * N, 0.0);
  cf.H.assign((size_t)n * N * N, 0.0);
  cf.sr.assign((size_t)n * N, 1.0);
  cf.sc.assign((size_t)n * N, 1.0);
  std::vector<cplx> S, Hprev;
  for (int i = 0; i < n; ++i) {
    S = Dg[i];
    if (i > 0) {
      // S_i = A_ii - A_{i,i-1} H_{i-1}
      for (int a = 0; a < N; ++a)
        for (int q = 0; q < N; ++q) {
          cplx lv = Lo[i][(size_t)a * N + q];
          if (lv == cplx(0.0)) continue;
          for (int b = 0; b < N; ++b) S[(size_t)a * N + b] -= lv * Hprev[(size_t)q * N + b];
        }
      std::copy(Lo[i].begin(), Lo[i].end(), cf.Lo.begin() + (size_t)i * N * N);
    }
    std::vector<double> sr, sc;
    ruiz_dense(S, N, sr, sc);
    for (int a = 0; a < N; ++a)
      for (int b = 0; b < N; ++b) S[(size_t)a * N + b] *= sr[a] * sc[b];
    invert(S, N);  // S now holds (diag(sr) S_i diag(sc))^{-1}
    std::copy(S.begin(), S.end(), cf.Sinv.begin() + (size_t)i * N * N);
    std::copy(sr.begin(), sr.end(), cf.sr.begin() + (size_t)i * N);
    std::copy(sc.begin(), sc.end(), cf.sc.begin() + (size_t)i * N);
    if (i < n - 1) {
      // H_i = S_i^{-1} A_{i,i+1} = diag(sc) Shat^{-1} diag(sr) A_{i,i+1}
      Hprev.assign((size_t)N * N, 0.0);
      for (int a = 0; a < N; ++a)
        for (int q = 0; q < N; ++q) {
          cplx sv = S[(size_t)a * N + q] * sr[q];
          for (int b = 0; b < N; ++b) Hprev[(size_t)a * N + b] += sv * Up[i][(size_t)q * N + b];
        }
      for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) Hprev[(size_t)a * N + b] *= sc[a];
      std::copy(Hprev.begin(), Hprev.end(), cf.H.begin() + (size_t)i * N * N);
    }
  }
}

// Propagators of the segmented scan (see ChainFactor).
void build_scan(ChainFactor& cf, int N, int seg) {
  const int n = cf.n;
  const size_t NN = (size_t)N * N;
  cf.Phi.assign((size_t)n * NN, 0.0);
  cf.Psi.assign((size_t)n * NN, 0.0);
  cf.G.assign((size_t)n * NN, 0.0);
  std::vector<cplx> D(NN);
  for (int i = 1; i < n; ++i) {
    // D = S_i^{-1} = diag(sc) Shat^{-1} diag(sr);  G_i = D Lo_i
    const cplx* Si = &cf.Sinv[(size_t)i * NN];
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < N; ++c) D[(size_t)r * N + c] = cf.sc[(size_t)i * N + r] * Si[(size_t)r * N + c] * cf.sr[(size_t)i * N + c];
    const cplx* Li = &cf.Lo[(size_t)i * NN];
    cplx* Gi = &cf.G[(size_t)i * NN];
    for (int r = 0; r < N; ++r)
      for (int q = 0; q < N; ++q) {
        cplx d = D[(size_t)r * N + q];
        for (int c = 0; c < N; ++c) Gi[(size_t)r * N + c] += d * Li[(size_t)q * N + c];
      }
  }
  for (int a = seg; a < n; a += seg) {
    int e = std::min(a + seg, n) - 1;
    for (int i = a; i <= e; ++i) {
      // Phi_a = -G_a, Phi_i = -G_i Phi_{i-1}
      const cplx* Gi = &cf.G[(size_t)i * NN];
      cplx* Pi = &cf.Phi[(size_t)i * NN];
      if (i == a) {
        for (size_t q = 0; q < NN; ++q) Pi[q] = -Gi[q];
      } else {
        const cplx* Pp = &cf.Phi[(size_t)(i - 1) * NN];
        for (int r = 0; r < N; ++r)
          for (int q = 0; q < N; ++q) {
            cplx gv = -Gi[(size_t)r * N + q];
            for (int c = 0; c < N; ++c) Pi[(size_t)r * N + c] += gv * Pp[(size_t)q * N + c];
          }
      }
    }
  }
  for (int a = 0; a < n; a += seg) {
    int e = std::min(a + seg, n) - 1;
    if (e == n - 1) break;
    for (int i = e; i >= a; --i) {
      const cplx* Hi = &cf.H[(size_t)i * NN];
      cplx* Pi = &cf.Psi[(size_t)i * NN];
      if (i == e) {
        for (size_t q = 0; q < NN; ++q) Pi[q] = -Hi[q];
      } else {
        const cplx* Pn = &cf.Psi[(size_t)(i + 1) * NN];
        for (int r = 0; r < N; ++r)
          for (int q = 0; q < N; ++q) {
            cplx hv = -Hi[(size_t)r * N + q];
            for (int c = 0; c < N; ++c) Pi[(size_t)r * N + c] += hv * Pn[(size_t)q * N + c];
          }
      }
    }
  }
}

void factor_T(const HostGrid& g, const OpParams& op, int l, TFactor& tf) {
  const int N = g.N;
  std::vector<double> A((size_t)N * N, 0.0);
  double lam = (double)l * (l + 1);
  for (int i = 0; i < N; ++i) {
    double r = g.r[i];
    for (int j = 0; j < N; ++j) {
      double K = (g.D2[(size_t)i * N + j] + 2.0 / r * g.D[(size_t)i * N + j] - (i == j ? lam / (r * r) : 0.0)) / op.Pr;
      A[(size_t)i * N + j] = (i == j ? 1.0 : 0.0) - op.dt * K;
    }
  }
  for (int row : {0, N - 1}) {
    std::fill(A.begin() + (size_t)row * N, A.begin() + (size_t)(row + 1) * N, 0.0);
    A[(size_t)row * N + row] = 1.0;
  }
  ruiz_dense(A, N, tf.tr, tf.tc);
  for (int a = 0; a < N; ++a)
    for (int b = 0; b < N; ++b) A[(size_t)a * N + b] *= tf.tr[a] * tf.tc[b];
  invert(A, N);
  tf.Tinv = A;
}

}  // namespace

void factor_all(const HostGrid& g, const OpParams& op, std::vector<ChainFactor>& chains,
                std::vector<TFactor>& tf, int nthreads, int seg) {
  Blocks B{g.N, &g, op};
  int nch = 2 * (g.K + 1);
  chains.assign(nch, ChainFactor());
  tf.assign(g.L + 1, TFactor());
  int ntask = nch + g.L + 1;
  std::vector<std::string> err(std::max(1, nthreads));
  auto work = [&](int tid) {
    try {
      for (int t = tid; t < ntask; t += nthreads) {
        if (t < nch) {
          factor_chain(B, g, t / 2, t % 2, chains[t]);
          build_scan(chains[t], g.N, seg);
        }
        else
          factor_T(g, op, t - nch, tf[t - nch]);
      }
    } catch (const std::exception& e) {
      err[tid] = e.what();
    }
  };
  if (nthreads <= 1) {
    nthreads = 1;
    work(0);
  } else {
    std::vector<std::thread> th;
    // heavy chains first: tasks are interleaved so each thread gets a mix
    for (int i = 0; i < nthreads; ++i) th.emplace_back(work, i);
    for (auto& t : th) t.join();
  }
  for (auto& e : err)
    if (!e.empty()) throw std::runtime_error(e);
}

}  // namespace sc
