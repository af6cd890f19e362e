// Host-side element matrices of the uniform box meshes.
//
// Elasticity (section "Poroelasticity", momentum balance): a(u, v) =
// (2 mu eps(u), eps(v)) + (lam div u, div v) by 3-point Gauss per axis (exact
// for Q2).  Coupling E_e[(c, node)][g] = (psi_g, d_c phi_node) by 2-point
// Gauss, exact because psi_g d_c phi is at most cubic per axis.
#include "element.h"

#include <array>
#include <cstddef>

#include "common.h"

namespace bt {

// tau * Q2 elasticity element matrix on a cell of size h (local order [comp][node, x fastest])
std::vector<double> elast_element(int d, const double* hh, double lam, double mu, double tau) {
  const int nn = d == 2 ? 9 : 27, nloc = d * nn;
  std::vector<double> K((size_t)nloc * nloc, 0.0);
  const int nq = d == 2 ? 9 : 27;
  for (int q = 0; q < nq; ++q) {
    const int kq[3] = {q % 3, (q / 3) % 3, d == 3 ? q / 9 : 0};
    double W = 1.0;
    for (int e = 0; e < d; ++e) W *= wq(kq[e]) * hh[e];
    // gradients of the scalar nodal functions at q
    std::vector<std::array<double, 3>> g(nn);
    for (int a = 0; a < nn; ++a) {
      const int aa[3] = {a % 3, (a / 3) % 3, d == 3 ? a / 9 : 0};
      for (int e = 0; e < d; ++e) {
        double v = 1.0;
        for (int f = 0; f < d; ++f) v *= (f == e) ? dphi(aa[f], xq(kq[f])) / hh[f] : phi(aa[f], xq(kq[f]));
        g[a][e] = v;
      }
    }
    for (int c = 0; c < d; ++c)
      for (int a = 0; a < nn; ++a)
        for (int c2 = 0; c2 < d; ++c2)
          for (int b = 0; b < nn; ++b) {
            // a(u,v): v = phi_a e_c (test), u = phi_b e_c2 (trial)
            double val = lam * g[a][c] * g[b][c2];
            val += mu * g[a][c2] * g[b][c];
            if (c == c2)
              for (int e = 0; e < d; ++e) val += mu * g[a][e] * g[b][e];
            K[(size_t)(c * nn + a) * nloc + (c2 * nn + b)] += tau * W * val;
          }
  }
  return K;
}


std::vector<double> coupling_element(int d, const double* hh) {
  const int nn = d == 2 ? 9 : 27, np = d == 2 ? 4 : 8;
  std::vector<double> E((size_t)d * nn * np, 0.0);
  double w = 1.0;
  for (int e = 0; e < d; ++e) w *= 0.5 * hh[e];
  for (int c = 0; c < d; ++c)
    for (int a = 0; a < nn; ++a) {
      const int aa[3] = {a % 3, (a / 3) % 3, d == 3 ? a / 9 : 0};
      for (int g = 0; g < np; ++g) {
        const int gg[3] = {g & 1, (g >> 1) & 1, (g >> 2) & 1};
        double v = w;
        for (int e = 0; e < d; ++e) v *= (e == c) ? dphi(aa[e], gp(gg[e])) / hh[e] : phi(aa[e], gp(gg[e]));
        E[(size_t)(c * nn + a) * np + g] = v;
      }
    }
  return E;
}

// 3D matrix-core layout of the element matrix [tau A_e | E_e] (81 x 81 or
// 81 x 89 with the coupling columns).  Rows are padded per component to 32
// (component c in padded rows 32c .. 32c+26), columns to a multiple of 4.
// Six 16-row tiles, tile w = (component w/2, half w%2); for k-step s and
// lane l the value is the entry at row 16 (w%2) + (l % 16) of that component
// and column 4 s + l / 16 (the A-operand layout of a 16x16x4 MFMA).
std::vector<double> elast_fragments3d(const std::vector<double>& A, const std::vector<double>* E) {
  const int ks = E ? 23 : 21;
  std::vector<double> out((size_t)6 * ks * 64, 0.0);
  for (int w = 0; w < 6; ++w)
    for (int s = 0; s < ks; ++s)
      for (int l = 0; l < 64; ++l) {
        const int pr = 16 * (w % 2) + (l % 16), col = 4 * s + l / 16;
        if (pr >= 27) continue;
        const int row = (w / 2) * 27 + pr;
        double v = 0.0;
        if (col < 81) v = A[(size_t)row * 81 + col];
        else if (E && col < 89) v = (*E)[(size_t)row * 8 + (col - 81)];
        out[((size_t)w * ks + s) * 64 + l] = v;
      }
  return out;
}

}  // namespace bt
