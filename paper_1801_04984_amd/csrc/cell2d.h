// 2D per-cell element kernels (registers only).
//
// Elasticity with pressure coupling, sum-factorised through the 3x3 Gauss
// points:  out_c(node) = sum_q  S_ce(q) d_e(phi_node)(q),
//   S = W_q [ ts * (2 mu eps(u) + lam div u I) - cp * p I ],
// i.e. ts*A u - cp*E p for one cell (section "Poroelasticity", momentum
// balance with the effective-stress coupling -b p I).  Node arrays are
// [y][x]; derivative factors 1/h are applied at the quadrature points.
#pragma once
#include "common.h"

namespace bt {

template <typename T>
__device__ __forceinline__ void elast2d(const T ux[3][3], const T uy[3][3], const T pc[2][2],
                                        T hx, T hy, T ts, T cp, T lam, T mu,
                                        T ox[3][3], T oy[3][3]) {
  const T ihx = T(1) / hx, ihy = T(1) / hy;
  // forward x-pass: values / derivatives along x at the 3 Gauss abscissae
  T vxx[3][3], dxx[3][3], vxy[3][3], dxy[3][3];  // [b][kx]
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T v0 = 0, d0 = 0, v1 = 0, d1 = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        v0 += T(VQ(k, a)) * ux[b][a];
        d0 += T(DQ(k, a)) * ux[b][a];
        v1 += T(VQ(k, a)) * uy[b][a];
        d1 += T(DQ(k, a)) * uy[b][a];
      }
      vxx[b][k] = v0; dxx[b][k] = d0; vxy[b][k] = v1; dxy[b][k] = d1;
    }
  // pressure along x at Gauss-3
  T pxk[2][3];
#pragma unroll
  for (int g = 0; g < 2; ++g)
#pragma unroll
    for (int k = 0; k < 3; ++k) pxk[g][k] = T(PQ(k, 0)) * pc[g][0] + T(PQ(k, 1)) * pc[g][1];

  T Axx[3][3], Ayx[3][3], Axy[3][3], Ayy[3][3];  // backward partials [b][kx]
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int k = 0; k < 3; ++k) { Axx[b][k] = 0; Ayx[b][k] = 0; Axy[b][k] = 0; Ayy[b][k] = 0; }

#pragma unroll
  for (int ky = 0; ky < 3; ++ky) {
#pragma unroll
    for (int kx = 0; kx < 3; ++kx) {
      T gxx = 0, gyx = 0, gxy = 0, gyy = 0;   // g<comp><dir>: d u_comp / d dir
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        gxx += T(VQ(ky, b)) * dxx[b][kx];
        gyx += T(DQ(ky, b)) * vxx[b][kx];
        gxy += T(VQ(ky, b)) * dxy[b][kx];
        gyy += T(DQ(ky, b)) * vxy[b][kx];
      }
      gxx *= ihx; gxy *= ihx; gyx *= ihy; gyy *= ihy;
      const T pq = T(PQ(ky, 0)) * pxk[0][kx] + T(PQ(ky, 1)) * pxk[1][kx];
      const T W = T(wq(kx) * wq(ky)) * hx * hy;
      const T div = gxx + gyy;
      const T sxx = ts * (T(2) * mu * gxx + lam * div) - cp * pq;
      const T syy = ts * (T(2) * mu * gyy + lam * div) - cp * pq;
      const T sxy = ts * mu * (gyx + gxy);
      // test weights: comp x: (d/dx: W sxx/hx, d/dy: W sxy/hy); comp y: (W sxy/hx, W syy/hy)
      const T cxx = W * sxx * ihx, cxy = W * sxy * ihy;
      const T cyx = W * sxy * ihx, cyy = W * syy * ihy;
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        Axx[b][kx] += T(VQ(ky, b)) * cxx;
        Ayx[b][kx] += T(DQ(ky, b)) * cxy;
        Axy[b][kx] += T(VQ(ky, b)) * cyx;
        Ayy[b][kx] += T(DQ(ky, b)) * cyy;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T sx = 0, sy = 0;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        sx += T(DQ(k, a)) * Axx[b][k] + T(VQ(k, a)) * Ayx[b][k];
        sy += T(DQ(k, a)) * Axy[b][k] + T(VQ(k, a)) * Ayy[b][k];
      }
      ox[b][a] = sx;
      oy[b][a] = sy;
    }
}

// div u at the 2x2 Gauss points [gy][gx]
template <typename T>
__device__ __forceinline__ void divu2d(const T ux[3][3], const T uy[3][3], T hx, T hy, T out[2][2]) {
#pragma unroll
  for (int gy = 0; gy < 2; ++gy)
#pragma unroll
    for (int gx = 0; gx < 2; ++gx) {
      T sx = 0, sy = 0;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          sx += T(VG(gy, b) * DG(gx, a)) * ux[b][a];
          sy += T(DG(gy, b) * VG(gx, a)) * uy[b][a];
        }
      out[gy][gx] = sx / hx + sy / hy;
    }
}

// div q at the 2x2 Gauss points; qx[gy][a], qy[a][gx]
template <typename T>
__device__ __forceinline__ void divq2d(const T qx[2][3], const T qy[3][2], T hx, T hy, T out[2][2]) {
#pragma unroll
  for (int gy = 0; gy < 2; ++gy)
#pragma unroll
    for (int gx = 0; gx < 2; ++gx) {
      T sx = 0, sy = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        sx += T(DG(gx, a)) * qx[gy][a];
        sy += T(DG(gy, a)) * qy[a][gx];
      }
      out[gy][gx] = sx / hx + sy / hy;
    }
}

}  // namespace bt
