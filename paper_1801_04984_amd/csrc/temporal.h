// Host-side dG(r) temporal constants.
#pragma once

namespace bt {

struct TemporalConstants {
  int r = 0;
  double s[4] = {0}, w[4] = {0};   // right Gauss-Radau nodes / weights on [0,1]
  double T[16] = {0};              // T = W^-1 D, row-major 4x4 (top-left (r+1)^2 used)
  double g[4] = {0};               // g = W^-1 phi(0)
  double Q[16] = {0}, Qi[16] = {0};// real block eigenbasis and its inverse
  double alpha[4] = {0};           // real part of the block of each column of Q
  double beta[4] = {0};            // +-imaginary part (0 for real eigenvalues)
};

TemporalConstants make_temporal(int r);

// Order of the preconditioner's levels: level k is column perm[k] of Q.  A
// complex pair alpha +- i beta (columns c, c+1 of Q, beta > 0) sits at levels
// first[i] and second[i].  by_pass: pair firsts, then the real levels, then
// the pair seconds (the square-block factorisation solves the first of every
// pair with the real levels and the seconds after them); otherwise Q's order.
struct LevelOrder {
  int perm[4] = {0, 1, 2, 3};
  int npairs = 0;
  int first[2] = {0, 0}, second[2] = {0, 0};
  double beta[2] = {0, 0};
};
LevelOrder level_order(const TemporalConstants& tc, bool by_pass);

}  // namespace bt
