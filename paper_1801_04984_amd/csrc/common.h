// Shared device-side definitions: per-instance descriptors, 1D basis tables,
// DoF addressing and essential-boundary predicates.
//
// Discretisation (Koecher, sections "Discretisation in Space" and
// "Discretisation in Time"): continuous Q2 displacement, RT1 flux with
// nodal tensor basis (closed quadratic along its own axis, open linear on
// the two Gauss points across), DG-Q1 pressure on the Gauss points; dG(r)
// in time on right Gauss-Radau points.  All DoF maps are affine in the cell
// index, so no index arrays exist.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bt {

// threads per block of the element-wise and gather kernels over segments
constexpr int kBlk = 256;

// The 8 XCDs of the chip each have their own L2, and consecutive workgroup ids
// go to consecutive XCDs.  xcd_order(n)[b] = the tile that workgroup b should
// take so that every XCD gets one contiguous run of tiles (neighbouring tiles
// share halo data through that XCD's L2): XCD x = b % 8 takes its k-th
// (k = b / 8) tile from the x-th run.
constexpr int kXcds = 8;
constexpr int kCus = 256;    // compute units of the MI355X (32 per XCD)
inline long long xcd_tile(long long b, long long n) {
  const long long x = b % kXcds, k = b / kXcds;
  const long long base = n / kXcds, rem = n % kXcds;   // run x holds base + (x < rem) tiles
  return x * base + (x < rem ? x : rem) + k;
}

// ---------------------------------------------------------------------------
// 1D bases on [0, 1]
//   closed:  phi_0 = (2s-1)(s-1), phi_1 = 4s(1-s), phi_2 = s(2s-1)
//   open:    psi_0, psi_1 linear Lagrange on g0,1 = 1/2 -+ 1/(2 sqrt 3)
//   3-point Gauss nodes xq_k, weights wq_k
// ---------------------------------------------------------------------------
constexpr double kSqrt3 = 1.7320508075688772935;
constexpr double kSqrt06 = 0.77459666924148337704;
constexpr double kG0 = 0.5 - 0.5 / kSqrt3;
constexpr double kG1 = 0.5 + 0.5 / kSqrt3;

__host__ __device__ constexpr double xq(int k) { return k == 0 ? 0.5 - 0.5 * kSqrt06 : (k == 1 ? 0.5 : 0.5 + 0.5 * kSqrt06); }
__host__ __device__ constexpr double wq(int k) { return k == 1 ? 8.0 / 18.0 : 5.0 / 18.0; }
__host__ __device__ constexpr double gp(int g) { return g == 0 ? kG0 : kG1; }
__host__ __device__ constexpr double phi(int a, double s) {
  return a == 0 ? (2.0 * s - 1.0) * (s - 1.0) : (a == 1 ? 4.0 * s * (1.0 - s) : s * (2.0 * s - 1.0));
}
__host__ __device__ constexpr double dphi(int a, double s) {
  return a == 0 ? 4.0 * s - 3.0 : (a == 1 ? 4.0 - 8.0 * s : 4.0 * s - 1.0);
}
__host__ __device__ constexpr double psi(int g, double s) { return g == 0 ? kSqrt3 * (kG1 - s) : kSqrt3 * (s - kG0); }

// tables (reference cell); indices are compile-time after unrolling
__host__ __device__ constexpr double VQ(int k, int a) { return phi(a, xq(k)); }   // closed value at Gauss-3
__host__ __device__ constexpr double DQ(int k, int a) { return dphi(a, xq(k)); }  // closed derivative at Gauss-3
__host__ __device__ constexpr double PQ(int k, int g) { return psi(g, xq(k)); }   // open value at Gauss-3
__host__ __device__ constexpr double VG(int g, int a) { return phi(a, gp(g)); }   // closed value at Gauss-2
__host__ __device__ constexpr double DG(int g, int a) { return dphi(a, gp(g)); }  // closed derivative at Gauss-2
// int_0^1 phi_a phi_b (closed quadratic mass), exact by 3-point Gauss
__host__ __device__ constexpr double MC(int a, int b) {
  return wq(0) * phi(a, xq(0)) * phi(b, xq(0)) + wq(1) * phi(a, xq(1)) * phi(b, xq(1)) +
         wq(2) * phi(a, xq(2)) * phi(b, xq(2));
}
// int_0^1 phi_a' psi_g, exact by 2-point Gauss (weights 1/2; psi_g(g') = delta)
__host__ __device__ constexpr double GB(int a, int g) { return 0.5 * dphi(a, gp(g)); }

// ---------------------------------------------------------------------------
// Instance descriptor (device copy).  Sizes of the nodal arrays:
//   u_c: su[0] x su[1] (x su[2]), su[e] = 2 n_e + 1
//   q_c: sq[c][e] = su[e] if e == c else 2 n_e
//   p  : sp[e] = 2 n_e
// ---------------------------------------------------------------------------
struct InstDev {
  int n[3];
  int dim;
  int su[3];
  int sp[3];
  int sq[3][3];
  double h[3];
  double tau, lam, mu, b, Minv, eta;
  double s0, t_ramp;
  int load_kind;
  int pad0;
  long long x_off;       // offset of the instance's slab vector
  long long N;           // spatial DoFs per level
  long long off_u[3];    // block offsets within a level
  long long off_q[3];
  long long off_p;
  long long cell_off;    // offset into per-cell arrays
  long long state_off;   // offset into state (one level) vectors
  long long ncells;
  long long emat_off;    // element matrices of the instance (2D: tau*A_e, E_e; 3D: matrix-core fragments)
  double Lfs;            // fixed-stress parameter L
};

// temporal matrices shared by a batch (same r)
struct TimeMat {
  double T[16];   // T[i*4+j]
  double g[4];
  double s[4];    // Radau nodes
  double Q[16];   // real block eigenbasis: Q^-1 T Q = Lambda_R
  double Qi[16];
  double alpha[4];
};

// --- essential-boundary predicates (bottom = last axis lower face) --------
// u_c at node m of a Q2 grid with nodal sizes su: bottom -> all components;
// lateral faces of axes < dim-1 -> the normal component (roller)
__host__ __device__ __forceinline__ bool ugrid_fixed(int dim, const int* su, int c, int mx, int my, int mz) {
  if (dim == 2) {
    if (my == 0) return true;
    return c == 0 && (mx == 0 || mx == su[0] - 1);
  }
  if (mz == 0) return true;
  if (c == 0) return mx == 0 || mx == su[0] - 1;
  if (c == 1) return my == 0 || my == su[1] - 1;
  return false;
}
__device__ __forceinline__ bool u_fixed(const InstDev& I, int c, int mx, int my, int mz) {
  return ugrid_fixed(I.dim, I.su, c, mx, my, mz);
}
// q_c at closed coordinate mc along its own axis
__device__ __forceinline__ bool q_fixed(const InstDev& I, int c, int mc) {
  if (c == I.dim - 1) return mc == 0;
  return mc == 0 || mc == I.su[c] - 1;
}


}  // namespace bt
