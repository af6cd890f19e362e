// Host-side dG(r) temporal constants (section "Discretisation in Time").
//
// Lagrange basis on the r+1 right Gauss-Radau points of [0,1] (roots of
// P_{r+1} - P_r mapped from [-1,1]); the points double as the quadrature.
// D_ij = int_0^1 phi_j' phi_i + phi_i(0) phi_j(0), W = diag(weights),
// T = W^-1 D, g = W^-1 phi(0).  The real block form Q^-1 T Q (1x1 blocks for
// real eigenvalues, [[a, b], [-b, a]] for complex pairs; section "Monolithic
// Approach", spectral decomposition) gives the level shifts alpha_j used by
// the blockwise preconditioner.
#include <cmath>
#include <complex>
#include <stdexcept>
#include <vector>

#include "temporal.h"

namespace bt {

namespace {

double legendre(int n, double x, double* dp) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { if (dp) *dp = 0.0; return 1.0; }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    double d2 = d0 + (2.0 * k - 1.0) * p1;   // P'_k = P'_{k-2} + (2k-1) P_{k-1}
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  if (dp) *dp = d1;
  return p1;
}

// solve dense n x n system (partial pivoting), in place
void solve_dense(std::vector<double> A, std::vector<double>& b, int n) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i) if (std::fabs(A[i * n + k]) > std::fabs(A[piv * n + k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k * n + j], A[piv * n + j]);
      std::swap(b[k], b[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[i * n + k] / A[k * n + k];
      for (int j = k; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
      b[i] -= f * b[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double s = b[k];
    for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * b[j];
    b[k] = s / A[k * n + k];
  }
}

// polynomial helpers (coefficients in increasing powers)
using Poly = std::vector<double>;
Poly pmul(const Poly& a, const Poly& b) {
  Poly c(a.size() + b.size() - 1, 0.0);
  for (size_t i = 0; i < a.size(); ++i)
    for (size_t j = 0; j < b.size(); ++j) c[i + j] += a[i] * b[j];
  return c;
}
Poly pder(const Poly& a) {
  if (a.size() <= 1) return Poly{0.0};
  Poly d(a.size() - 1);
  for (size_t i = 1; i < a.size(); ++i) d[i - 1] = i * a[i];
  return d;
}
double pint01(const Poly& a) {
  double s = 0.0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] / (i + 1.0);
  return s;
}
double peval(const Poly& a, double x) {
  double s = 0.0;
  for (size_t i = a.size(); i-- > 0;) s = s * x + a[i];
  return s;
}

using cd = std::complex<double>;

// eigenvalues of a small real matrix: Hessenberg-free, via characteristic
// polynomial (Faddeev-LeVerrier) and Aberth-Ehrlich root refinement.
std::vector<cd> eigenvalues(const std::vector<double>& A, int n) {
  // char poly c: det(lambda I - A) = sum c_k lambda^k, c_n = 1
  std::vector<double> c(n + 1, 0.0);
  c[n] = 1.0;
  std::vector<double> Mk(n * n, 0.0), AM(n * n);
  for (int k = 1; k <= n; ++k) {
    // M_k = A M_{k-1} + c_{n-k+1} I
    std::vector<double> Mn(n * n, 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int l = 0; l < n; ++l) s += A[i * n + l] * Mk[l * n + j];
        Mn[i * n + j] = s + (i == j ? c[n - k + 1] : 0.0);
      }
    Mk = Mn;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        double s = 0.0;
        for (int l = 0; l < n; ++l) s += A[i * n + l] * Mk[l * n + j];
        AM[i * n + j] = s;
      }
    double tr = 0.0;
    for (int i = 0; i < n; ++i) tr += AM[i * n + i];
    c[n - k] = -tr / k;
  }
  std::vector<cd> z(n);
  double rad = 0.0;
  for (int k = 0; k < n; ++k) rad = std::max(rad, std::fabs(c[k]));
  rad = 1.0 + rad;
  for (int k = 0; k < n; ++k) z[k] = std::polar(0.5 * rad, 0.4 + 2.0 * M_PI * k / n);
  for (int it = 0; it < 500; ++it) {
    double maxstep = 0.0;
    for (int k = 0; k < n; ++k) {
      cd p = 0.0, dp = 0.0;
      for (int m = n; m >= 0; --m) { dp = dp * z[k] + p; p = p * z[k] + c[m]; }
      cd ratio = p / dp;
      cd s = 0.0;
      for (int j = 0; j < n; ++j) if (j != k) s += 1.0 / (z[k] - z[j]);
      cd step = ratio / (1.0 - ratio * s);
      z[k] -= step;
      maxstep = std::max(maxstep, std::abs(step));
    }
    if (maxstep < 1e-16 * rad) break;
  }
  return z;
}

// null vector of (A - lambda I) by complex Gaussian elimination with full pivoting
std::vector<cd> null_vector(const std::vector<double>& A, int n, cd lam) {
  std::vector<cd> B(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) B[i * n + j] = A[i * n + j] - (i == j ? lam : 0.0);
  std::vector<int> colp(n);
  for (int j = 0; j < n; ++j) colp[j] = j;
  int rank = 0;
  for (int k = 0; k < n - 1; ++k) {
    int pi = k, pj = k;
    double best = -1.0;
    for (int i = k; i < n; ++i)
      for (int j = k; j < n; ++j)
        if (std::abs(B[i * n + j]) > best) { best = std::abs(B[i * n + j]); pi = i; pj = j; }
    for (int j = 0; j < n; ++j) std::swap(B[k * n + j], B[pi * n + j]);
    for (int i = 0; i < n; ++i) std::swap(B[i * n + k], B[i * n + pj]);
    std::swap(colp[k], colp[pj]);
    for (int i = k + 1; i < n; ++i) {
      cd f = B[i * n + k] / B[k * n + k];
      for (int j = k; j < n; ++j) B[i * n + j] -= f * B[k * n + j];
    }
    rank = k + 1;
  }
  // free variable = last (permuted) unknown
  std::vector<cd> y(n, 0.0);
  y[n - 1] = 1.0;
  for (int k = rank - 1; k >= 0; --k) {
    cd s = 0.0;
    for (int j = k + 1; j < n; ++j) s += B[k * n + j] * y[j];
    y[k] = -s / B[k * n + k];
  }
  std::vector<cd> v(n);
  for (int j = 0; j < n; ++j) v[colp[j]] = y[j];
  double nrm = 0.0;
  for (auto& e : v) nrm += std::norm(e);
  nrm = std::sqrt(nrm);
  for (auto& e : v) e /= nrm;
  return v;
}

}  // namespace

TemporalConstants make_temporal(int r) {
  if (r < 0 || r > 3) throw std::runtime_error("dG order r must be in 0..3");
  const int n = r + 1;
  TemporalConstants tc;
  tc.r = r;
  // Radau nodes: roots of P_{r+1} - P_r on [-1,1]; x = 1 is one of them.
  std::vector<double> x(n);
  x[n - 1] = 1.0;
  for (int k = 0; k < n - 1; ++k) {
    // initial guess: Chebyshev-like spacing
    double xi = -std::cos(M_PI * (2.0 * k + 1.0) / (2.0 * n));
    for (int it = 0; it < 100; ++it) {
      double d1, d0;
      double f = legendre(n, xi, &d1) - legendre(n - 1, xi, &d0);
      double df = d1 - d0;
      // deflate roots already found and the root at 1
      double s = 1.0 / (xi - 1.0);
      for (int j = 0; j < k; ++j) s += 1.0 / (xi - x[j]);
      double step = f / (df - f * s);
      xi -= step;
      if (std::fabs(step) < 1e-16) break;
    }
    x[k] = xi;
  }
  std::vector<double> s(n);
  for (int k = 0; k < n; ++k) s[k] = 0.5 * (x[k] + 1.0);
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b)
      if (s[b] < s[a]) std::swap(s[a], s[b]);
  // weights: exact on 1, s, ..., s^r
  std::vector<double> V(n * n), w(n);
  for (int m = 0; m < n; ++m) {
    for (int k = 0; k < n; ++k) V[m * n + k] = std::pow(s[k], m);
    w[m] = 1.0 / (m + 1.0);
  }
  solve_dense(V, w, n);
  // Lagrange polynomials
  std::vector<Poly> L(n);
  for (int j = 0; j < n; ++j) {
    Poly p{1.0};
    double den = 1.0;
    for (int k = 0; k < n; ++k) {
      if (k == j) continue;
      p = pmul(p, Poly{-s[k], 1.0});
      den *= s[j] - s[k];
    }
    for (auto& cf : p) cf /= den;
    L[j] = p;
  }
  std::vector<double> T(n * n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      double D = pint01(pmul(pder(L[j]), L[i])) + peval(L[i], 0.0) * peval(L[j], 0.0);
      T[i * n + j] = D / w[i];
    }
    tc.g[i] = peval(L[i], 0.0) / w[i];
    tc.s[i] = s[i];
    tc.w[i] = w[i];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) tc.T[i * 4 + j] = T[i * n + j];

  // real block form
  std::vector<cd> ev = eigenvalues(T, n);
  std::vector<bool> used(n, false);
  std::vector<std::vector<double>> cols;
  std::vector<double> alpha, beta;
  // order by decreasing real part
  std::vector<int> order(n);
  for (int k = 0; k < n; ++k) order[k] = k;
  for (int a = 0; a < n; ++a)
    for (int b = a + 1; b < n; ++b)
      if (ev[order[b]].real() > ev[order[a]].real()) std::swap(order[a], order[b]);
  for (int oi = 0; oi < n; ++oi) {
    int k = order[oi];
    if (used[k]) continue;
    if (std::fabs(ev[k].imag()) < 1e-10) {
      auto v = null_vector(T, n, cd(ev[k].real(), 0.0));
      // make it real: rotate by the phase of its largest entry
      int big = 0;
      for (int j = 1; j < n; ++j) if (std::abs(v[j]) > std::abs(v[big])) big = j;
      cd ph = std::abs(v[big]) / v[big];
      std::vector<double> col(n);
      for (int j = 0; j < n; ++j) col[j] = (v[j] * ph).real();
      cols.push_back(col);
      alpha.push_back(ev[k].real());
      beta.push_back(0.0);
      used[k] = true;
    } else {
      cd lam = ev[k].imag() > 0 ? ev[k] : std::conj(ev[k]);
      int partner = -1;
      double best = 1e300;
      for (int j = 0; j < n; ++j) {
        if (j == k || used[j]) continue;
        double dd = std::abs(ev[j] - std::conj(ev[k]));
        if (dd < best) { best = dd; partner = j; }
      }
      auto v = null_vector(T, n, lam);
      std::vector<double> a(n), b(n);
      for (int j = 0; j < n; ++j) { a[j] = v[j].real(); b[j] = v[j].imag(); }
      cols.push_back(a);
      cols.push_back(b);
      alpha.push_back(lam.real()); alpha.push_back(lam.real());
      beta.push_back(lam.imag()); beta.push_back(-lam.imag());
      used[k] = true;
      if (partner >= 0) used[partner] = true;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) tc.Q[i * 4 + j] = cols[j][i];
  // inverse of Q
  for (int j = 0; j < n; ++j) {
    std::vector<double> A(n * n), e(n, 0.0);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) A[a * n + b] = tc.Q[a * 4 + b];
    e[j] = 1.0;
    solve_dense(A, e, n);
    for (int i = 0; i < n; ++i) tc.Qi[i * 4 + j] = e[i];
  }
  for (int k = 0; k < n; ++k) { tc.alpha[k] = alpha[k]; tc.beta[k] = beta[k]; }
  return tc;
}

LevelOrder level_order(const TemporalConstants& tc, bool by_pass) {
  LevelOrder o;
  const int n = tc.r + 1;
  int col[2] = {0, 0};
  for (int j = 0; j + 1 < n; ++j)
    if (tc.beta[j] > 0 && o.npairs < 2) col[o.npairs++] = j;   // columns j, j+1
  if (by_pass && o.npairs > 0) {
    int k = 0;
    for (int i = 0; i < o.npairs; ++i) o.perm[k++] = col[i];
    for (int j = 0; j < n; ++j) {
      bool in_pair = false;
      for (int i = 0; i < o.npairs; ++i) in_pair = in_pair || j == col[i] || j == col[i] + 1;
      if (!in_pair) o.perm[k++] = j;
    }
    for (int i = 0; i < o.npairs; ++i) o.perm[k++] = col[i] + 1;
  }
  for (int i = 0; i < o.npairs; ++i) {
    for (int k = 0; k < n; ++k) {
      if (o.perm[k] == col[i]) o.first[i] = k;
      if (o.perm[k] == col[i] + 1) o.second[i] = k;
    }
    o.beta[i] = tc.beta[col[i]];
  }
  return o;
}

}  // namespace bt
