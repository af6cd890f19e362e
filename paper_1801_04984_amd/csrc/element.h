// Host-side element matrices of the uniform box meshes (reference ordering:
// [component][node], nodes x fastest; pressure nodes x fastest).
#pragma once
#include <vector>

namespace bt {
// tau * elasticity element matrix: a(u,v) = (2 mu eps(u), eps(v)) + (lam div u, div v), 3-point Gauss
std::vector<double> elast_element(int d, const double* h, double lam, double mu, double tau);
// E_e[(c, node)][g] = (psi_g, d_c phi_node): the displacement/pressure coupling, 2-point Gauss (exact)
std::vector<double> coupling_element(int d, const double* h);
// 3D matrix-core fragments of [tau A_e | E_e] (E may be null): [tile 6][k-step 23|21][lane 64]
std::vector<double> elast_fragments3d(const std::vector<double>& A, const std::vector<double>* E);
}  // namespace bt
