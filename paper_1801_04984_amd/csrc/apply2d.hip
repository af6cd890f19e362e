// 2D space-time slab operator  Y = A X  (or A^T X), all levels of a slab.
//
// Section "Monolithic Approach": the slab matrix is
//   A = T kron M_t + tau I kron K_s,  essential rows = identity,
// so level i of Y is
//   u-rows:  tau (A u_i - b E p_i)                      [A^T: tau A u_i - b E (sum_j T_ji p_j)]
//   q-rows:  tau (Mq q_i + B p_i)                       [same for A^T]
//   p-rows:  -w [tau div q_i + sum_j T_ij (b div u_j + p_j / M)](Gauss-2 point)
//            [A^T: -w (tau div q_i + tau b div u_i + sum_j T_ji p_j / M)]
// The p-rows are exact pointwise collocation on the 2x2 Gauss points (the
// integrands are bi-cubic at most and psi_k is nodal there), Mq and B act
// only along the flux component's own axis because the open basis is
// orthogonal under 2-point Gauss.
//
// The element u-rows use the dense element matrices tau A_e (18x18) and E_e
// (18x4), identical for every cell of an instance: 396 FMA per cell and level,
// fewer than the sum-factorised evaluation in 2D and far lighter on registers.
//
// Work decomposition: one block = one tile of (TS-1)x(TS-1) owned cells plus a
// one-cell halo on the low sides (TS x TS threads, one cell each; TS = 16 or
// 8, chosen per handle by the tile autotuner: both give identical results).  Every
// output DoF is written by exactly one block: u-rows are summed from the
// per-cell element vectors staged in LDS in a fixed order (deterministic,
// no atomics); q-rows are evaluated node by node from X; p-rows are
// cell-local.  Halo cells are recomputed by both neighbours.
#include "cell2d.h"
#include "kernels.h"

namespace bt {

template <typename T, int NL, bool TR, int kT2>
__global__ __launch_bounds__(kT2 * kT2) void apply2d_kernel(const InstDev* __restrict__ insts,
                                                      const int4* __restrict__ work, TimeMat tm,
                                                      const T* __restrict__ kinv_all, const T* __restrict__ emat,
                                                      const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int kO2 = kT2 - 1;
  __shared__ T E[18][kT2 * kT2];
  const int4 w = work[blockIdx.x];
  const InstDev& I = insts[w.x];
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * kT2 + lx;
  const int nx = I.n[0], ny = I.n[1];
  const int i0 = w.y * kO2, j0 = w.z * kO2;
  const int i = i0 - 1 + lx, j = j0 - 1 + ly;
  const bool valid = (i >= 0) && (i < nx) && (j >= 0) && (j < ny);
  const bool owned = valid && lx >= 1 && ly >= 1;
  const int sux = I.su[0], spx = I.sp[0];
  const long long N = I.N;
  const T* Xb = X + I.x_off;
  T* Yb = Y + I.x_off;
  const T hx = T(I.h[0]), hy = T(I.h[1]);
  const T tau = T(I.tau), lam = T(I.lam), mu = T(I.mu), bb = T(I.b), Minv = T(I.Minv);
  const T w2 = hx * hy * T(0.25);
  const T* kinv = kinv_all + I.cell_off;

  // pressure of every level (p is never constrained)
  T pl[NL][2][2];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gx = 0; gx < 2; ++gx)
        pl[l][gy][gx] = valid ? Xb[l * N + I.off_p + (2 * i + gx) + (long long)spx * (2 * j + gy)] : T(0);

  // forward p-rows accumulate over levels: yp_i = tau dq_i + sum_j T_ij zeta_j
  // (register arrays are only indexed with compile-time indices)
  T yp[NL][2][2];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int g = 0; g < 4; ++g) yp[l][g >> 1][g & 1] = T(0);

  // owned node ranges (the last tile along an axis also owns the top face)
  const int mxe = (i0 + kO2 >= nx) ? 2 * nx + 1 : 2 * i0 + 2 * kO2;
  const int mye = (j0 + kO2 >= ny) ? 2 * ny + 1 : 2 * j0 + 2 * kO2;
  const int oxe = min(2 * i0 + 2 * kO2, 2 * nx);
  const int oye = min(2 * j0 + 2 * kO2, 2 * ny);
  const int nmx = mxe - 2 * i0, nmy = mye - 2 * j0, nox = oxe - 2 * i0, noy = oye - 2 * j0;

#pragma unroll 1
  for (int lev = 0; lev < NL; ++lev) {
    const T* Xl = Xb + lev * N;
    T* Yl = Yb + lev * N;
    T ux[3][3], uy[3][3], qx[2][3], qy[3][2];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int mx = 2 * i + a, my = 2 * j + b;
        const long long o = mx + (long long)sux * my;
        ux[b][a] = valid ? ld(Xl + I.off_u[0] + o, u_fixed(I, 0, mx, my, 0)) : T(0);
        uy[b][a] = valid ? ld(Xl + I.off_u[1] + o, u_fixed(I, 1, mx, my, 0)) : T(0);
      }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int mx = 2 * i + a, oy = 2 * j + g;
        qx[g][a] = valid ? ld(Xl + I.off_q[0] + mx + (long long)sux * oy, q_fixed(I, 0, mx)) : T(0);
        const int ox = 2 * i + g, my = 2 * j + a;
        qy[a][g] = valid ? ld(Xl + I.off_q[1] + ox + (long long)spx * my, q_fixed(I, 1, my)) : T(0);
      }
    T pc[2][2];
    T cp;
    if (!TR) {
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < NL; ++l) s += (l == lev) ? pl[l][gy][gx] : T(0);
          pc[gy][gx] = s;
        }
      cp = tau * bb;
    } else {
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < NL; ++l) s += T(tm.T[l * 4 + lev]) * pl[l][gy][gx];
          pc[gy][gx] = s;
        }
      cp = bb;
    }
    // element u-rows: tau A_e u - cp E_e p  (A_e, E_e identical for every cell of the instance)
    {
      const T* AE = emat + I.emat_off;
      const T* EE = AE + 18 * 18;
      T uu[18];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) { uu[b * 3 + a] = ux[b][a]; uu[9 + b * 3 + a] = uy[b][a]; }
#pragma unroll
      for (int rr = 0; rr < 18; ++rr) {
        T acc = 0;
#pragma unroll
        for (int cc = 0; cc < 18; ++cc) acc += AE[rr * 18 + cc] * uu[cc];
        T ep = EE[rr * 4 + 0] * pc[0][0] + EE[rr * 4 + 1] * pc[0][1] + EE[rr * 4 + 2] * pc[1][0] +
               EE[rr * 4 + 3] * pc[1][1];
        E[rr][tid] = acc - cp * ep;
      }
    }
    T du[2][2], dq[2][2];
    divu2d<T>(ux, uy, hx, hy, du);
    divq2d<T>(qx, qy, hx, hy, dq);
    if (!TR) {
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          const T z = bb * du[gy][gx] + Minv * pc[gy][gx];
#pragma unroll
          for (int l = 0; l < NL; ++l)
            yp[l][gy][gx] += T(tm.T[l * 4 + lev]) * z + ((l == lev) ? tau * dq[gy][gx] : T(0));
        }
    } else if (owned) {
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < NL; ++l) s += T(tm.T[l * 4 + lev]) * pl[l][gy][gx];
          Yl[I.off_p + (2 * i + gx) + (long long)spx * (2 * j + gy)] =
              -w2 * (tau * dq[gy][gx] + tau * bb * du[gy][gx] + Minv * s);
        }
    }
    __syncthreads();

    // ---- u-rows: sum element contributions of the (up to 4) cells of each node
    const int nu = nmx * nmy;
    for (int idx = tid; idx < 2 * nu; idx += kT2 * kT2) {
      const int c = idx >= nu;
      const int r = idx - c * nu;
      const int mx = 2 * i0 + r % nmx, my = 2 * j0 + r / nmx;
      const long long go = (c ? I.off_u[1] : I.off_u[0]) + mx + (long long)sux * my;
      T v;
      if (u_fixed(I, c, mx, my, 0)) {
        v = Xl[go];
      } else {
        // the (up to) two cells along each axis that share the node, low first
        const bool xo = mx & 1, yo = my & 1;
        const int cx0 = xo ? (mx - 1) / 2 : mx / 2 - 1, ax0 = xo ? 1 : 2;
        const int cy0 = yo ? (my - 1) / 2 : my / 2 - 1, ay0 = yo ? 1 : 2;
        const bool vx0 = cx0 >= 0, vx1 = !xo && (mx / 2 < nx);
        const bool vy0 = cy0 >= 0, vy1 = !yo && (my / 2 < ny);
        const int tx0 = cx0 - i0 + 1, ty0 = cy0 - j0 + 1;
        v = 0;
        if (vy0 && vx0) v += E[c * 9 + ay0 * 3 + ax0][ty0 * kT2 + tx0];
        if (vy0 && vx1) v += E[c * 9 + ay0 * 3 + 0][ty0 * kT2 + tx0 + 1];
        if (vy1 && vx0) v += E[c * 9 + 0 * 3 + ax0][(ty0 + 1) * kT2 + tx0];
        if (vy1 && vx1) v += E[c * 9 + 0][(ty0 + 1) * kT2 + tx0 + 1];
      }
      Yl[go] = v;
    }
    // ---- q-rows: tau (Mq q + B p), node by node along the flux axis
    const T cqx = tau * hx * hy * T(0.5), cbx = tau * hy * T(0.5);
    const int nqx = nmx * noy;
    for (int idx = tid; idx < nqx; idx += kT2 * kT2) {
      const int mx = 2 * i0 + idx % nmx, oy = 2 * j0 + idx / nmx;
      const long long go = I.off_q[0] + mx + (long long)sux * oy;
      T v;
      if (q_fixed(I, 0, mx)) {
        v = Xl[go];
      } else {
        v = 0;
        const int jj = oy >> 1;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          int ii, a;
          if (mx & 1) { if (s) break; ii = (mx - 1) / 2; a = 1; }
          else { ii = mx / 2 - 1 + s; a = s ? 0 : 2; if (ii < 0 || ii >= nx) continue; }
          T m = 0;
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2) {
            const int m2 = 2 * ii + a2;
            m += T(MC(a, a2)) * ld(Xl + I.off_q[0] + m2 + (long long)sux * oy, q_fixed(I, 0, m2));
          }
          const T* pp = Xl + I.off_p + 2 * ii + (long long)spx * oy;
          const T bp = T(GB(a, 0)) * pp[0] + T(GB(a, 1)) * pp[1];
          v += cqx * kinv[ii + (long long)nx * jj] * m - cbx * bp;
        }
      }
      Yl[go] = v;
    }
    const T cqy = tau * hx * hy * T(0.5), cby = tau * hx * T(0.5);
    const int nqy = nox * nmy;
    for (int idx = tid; idx < nqy; idx += kT2 * kT2) {
      const int ox = 2 * i0 + idx % nox, my = 2 * j0 + idx / nox;
      const long long go = I.off_q[1] + ox + (long long)spx * my;
      T v;
      if (q_fixed(I, 1, my)) {
        v = Xl[go];
      } else {
        v = 0;
        const int ii = ox >> 1;
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          int jj, a;
          if (my & 1) { if (s) break; jj = (my - 1) / 2; a = 1; }
          else { jj = my / 2 - 1 + s; a = s ? 0 : 2; if (jj < 0 || jj >= ny) continue; }
          T m = 0;
#pragma unroll
          for (int a2 = 0; a2 < 3; ++a2) {
            const int m2 = 2 * jj + a2;
            m += T(MC(a, a2)) * ld(Xl + I.off_q[1] + ox + (long long)spx * m2, q_fixed(I, 1, m2));
          }
          const T* pp = Xl + I.off_p + ox + (long long)spx * (2 * jj);
          const T bp = T(GB(a, 0)) * pp[0] + T(GB(a, 1)) * pp[spx];
          v += cqy * kinv[ii + (long long)nx * jj] * m - cby * bp;
        }
      }
      Yl[go] = v;
    }
    __syncthreads();
  }

  if (!TR && owned) {
#pragma unroll
    for (int lev = 0; lev < NL; ++lev)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx)
          Yb[lev * N + I.off_p + (2 * i + gx) + (long long)spx * (2 * j + gy)] = -w2 * yp[lev][gy][gx];
  }
}

template <typename T, int NL, int TS>
static void launch_ts(const ApplyArgs& a, const void* x, void* y, int transpose) {
  dim3 blk(TS, TS);
  if (transpose)
    hipLaunchKernelGGL((apply2d_kernel<T, NL, true, TS>), dim3(a.nwork), blk, 0, a.stream, a.inst, a.work, *a.tm,
                       (const T*)a.kinv, (const T*)a.emat, (const T*)x, (T*)y);
  else
    hipLaunchKernelGGL((apply2d_kernel<T, NL, false, TS>), dim3(a.nwork), blk, 0, a.stream, a.inst, a.work, *a.tm,
                       (const T*)a.kinv, (const T*)a.emat, (const T*)x, (T*)y);
}

template <typename T, int NL>
static void launch_nl(const ApplyArgs& a, const void* x, void* y, int transpose) {
  if (a.variant == 1) launch_ts<T, NL, 8>(a, x, y, transpose);
  else launch_ts<T, NL, 16>(a, x, y, transpose);
}

template <typename T>
void launch_apply2d(const ApplyArgs& a, const void* x, void* y, int transpose) {
  switch (a.nl) {
    case 1: launch_nl<T, 1>(a, x, y, transpose); break;
    case 2: launch_nl<T, 2>(a, x, y, transpose); break;
    case 3: launch_nl<T, 3>(a, x, y, transpose); break;
    default: launch_nl<T, 4>(a, x, y, transpose); break;
  }
}

template void launch_apply2d<double>(const ApplyArgs&, const void*, void*, int);
template void launch_apply2d<float>(const ApplyArgs&, const void*, void*, int);

// tile variants: 0 = 16x16 threads (15x15 owned cells), 1 = 8x8 (7x7)
int apply2d_variants() { return 2; }
int apply2d_tile_cells(int variant) { return variant == 1 ? 7 : 15; }

}  // namespace bt
