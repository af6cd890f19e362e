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
// 8, with the time levels in a loop or, for 8, in parallel thread layers;
// chosen per handle by the tile autotuner: all give identical results).
// Every cell computes its element rows (u, then flux), stages them in LDS,
// and each owned cell sums its own nodes - the lower-left 2x2 node block of
// the cell, plus the top/right boundary nodes of the last cells - from the
// rows of the (up to four) cells sharing them, in a fixed order: every output
// is written by exactly one thread, deterministically, without atomics or
// index divisions.  p-rows are cell-local.  Halo cells are recomputed by both
// neighbouring tiles.
#include "common.h"
#include "kernels.h"

namespace bt {

// LP (level-parallel): the block holds one kT2 x kT2 thread layer per time
// level (threadIdx.z = level), each layer doing that level's rows; the forward
// p-rows, which sum over levels, exchange the per-level values through LDS
// and add them in the same order as the level loop, so both forms give
// bitwise the same result.
template <typename T, int NL, bool TR, int kT2, bool LP>
__global__ __launch_bounds__(kT2 * kT2 * (LP ? NL : 1)) void apply2d_kernel(
    const InstDev* __restrict__ insts, const int4* __restrict__ work, TimeMat tm, const T* __restrict__ kinv_all,
    const T* __restrict__ emat, const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int kO2 = kT2 - 1;
  constexpr int kLay = LP ? NL : 1;
  __shared__ T Es[kLay][18][kT2 * kT2];
  __shared__ T Zs[LP && !TR ? NL : 1][4][LP && !TR ? kT2 * kT2 : 1];
  const int lev0 = LP ? (int)threadIdx.z : 0, lev1 = LP ? lev0 + 1 : NL;
  T(*E)[kT2 * kT2] = Es[LP ? lev0 : 0];
  const int4 w = work[blockIdx.x];
  const InstDev& I = insts[w.x];
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * kT2 + lx;
  const int nx = I.n[0], ny = I.n[1];
  const int i = w.y * kO2 - 1 + lx, j = w.z * kO2 - 1 + ly;
  const bool valid = (i >= 0) && (i < nx) && (j >= 0) && (j < ny);
  const bool owned = valid && lx >= 1 && ly >= 1;
  const bool lastx = i == nx - 1, lasty = j == ny - 1;
  const int sux = I.su[0], spx = I.sp[0];
  const int N = (int)I.N;
  const T* Xb = X + I.x_off;
  T* Yb = Y + I.x_off;
  const T hx = T(I.h[0]), hy = T(I.h[1]);
  const T ihx = T(1.0 / I.h[0]), ihy = T(1.0 / I.h[1]);
  const T tau = T(I.tau), bb = T(I.b), Minv = T(I.Minv);
  const T w2 = hx * hy * T(0.25);
  const T kraw = kinv_all[I.cell_off + (valid ? i + nx * j : 0)];
  const T kc = valid ? kraw : T(0);
  // offsets of the cell's lowest node in each nodal array (x fastest)
  const int ub = 2 * i + sux * (2 * j);      // u_c (su0 x su1) and q_x (su0 x sp1) arrays
  const int qyb = 2 * i + spx * (2 * j);     // q_y (sp0 x su1) and p (sp0 x sp1) arrays
  const int ou0 = (int)I.off_u[0], ou1 = (int)I.off_u[1];
  const int oq0 = (int)I.off_q[0], oq1 = (int)I.off_q[1], op = (int)I.off_p;
  // flux-row scales: tau h_e (h_f / 2) eta/K for the mass part, tau (h_f / 2) for B p
  const T cqx = tau * hx * hy * T(0.5) * kc, cbx = tau * hy * T(0.5);
  const T cqy = tau * hx * hy * T(0.5) * kc, cby = tau * hx * T(0.5);

  // Loads use clamped in-range offsets and are masked afterwards, so that no
  // load waits behind a branch; the raw values of the cell's own nodes also
  // serve the identity rows of essential nodes.
  const int ubc = valid ? ub : 0, qybc = valid ? qyb : 0;
  // pressure of every level (p is never constrained)
  T pl[NL][2][2];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gx = 0; gx < 2; ++gx) {
        const T v = Xb[l * N + op + qybc + gx + spx * gy];
        pl[l][gy][gx] = valid ? v : T(0);
      }

  // forward p-rows accumulate over levels: yp_i = tau dq_i + sum_j T_ij zeta_j
  // (register arrays are only indexed with compile-time indices)
  T yp[NL][2][2];
#pragma unroll
  for (int l = 0; l < NL; ++l)
#pragma unroll
    for (int g = 0; g < 4; ++g) yp[l][g >> 1][g & 1] = T(0);

  T tdq[2][2];   // level-parallel forward: tau div q of this thread's level
#pragma unroll 1
  for (int lev = lev0; lev < lev1; ++lev) {
    const T* Xl = Xb + lev * N;
    T* Yl = Yb + lev * N;
    // ---- cell data of this level (raw), then with essential values masked
    T uxr[3][3], uyr[3][3], qxr[2][3], qyr[3][2];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int o = ubc + a + sux * b;
        uxr[b][a] = Xl[ou0 + o];
        uyr[b][a] = Xl[ou1 + o];
      }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        qxr[g][a] = Xl[oq0 + ubc + a + sux * g];
        qyr[a][g] = Xl[oq1 + qybc + g + spx * a];
      }
    T ux[3][3], uy[3][3], qx[2][3], qy[3][2];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const bool bot = b == 0 && j == 0;
        const bool fx = bot || (a == 0 && i == 0) || (a == 2 && lastx);
        ux[b][a] = (valid && !fx) ? uxr[b][a] : T(0);
        uy[b][a] = (valid && !bot) ? uyr[b][a] : T(0);
      }
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const bool fqx = (a == 0 && i == 0) || (a == 2 && lastx);   // no-flow on the x faces
        const bool fqy = a == 0 && j == 0;                           // no-flow at the bottom
        qx[g][a] = (valid && !fqx) ? qxr[g][a] : T(0);
        qy[a][g] = (valid && !fqy) ? qyr[a][g] : T(0);
      }
    T pcur[2][2], pc[2][2];
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gx = 0; gx < 2; ++gx) {
        T s = 0, st = 0;
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          s += (l == lev) ? pl[l][gy][gx] : T(0);
          st += T(tm.T[l * 4 + lev]) * pl[l][gy][gx];
        }
        pcur[gy][gx] = s;
        pc[gy][gx] = TR ? st : s;
      }
    const T cp = TR ? bb : tau * bb;
    // ---- element u-rows: tau A_e u - cp E_e p  (A_e, E_e identical for every cell of the instance)
    {
      const T* AE = emat + I.emat_off;
      const T* EE = AE + 18 * 18;
      T uu[18];
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int a = 0; a < 3; ++a) { uu[b * 3 + a] = ux[b][a]; uu[9 + b * 3 + a] = uy[b][a]; }
      // one row of the uniform element matrices per iteration (scalar loads;
      // unrolling all 18 rows would spill the scalar registers)
#pragma unroll 1
      for (int rr = 0; rr < 18; ++rr) {
        T acc = 0;
#pragma unroll
        for (int cc = 0; cc < 18; ++cc) acc += AE[rr * 18 + cc] * uu[cc];
        T ep = EE[rr * 4 + 0] * pc[0][0] + EE[rr * 4 + 1] * pc[0][1] + EE[rr * 4 + 2] * pc[1][0] +
               EE[rr * 4 + 3] * pc[1][1];
        E[rr][tid] = acc - cp * ep;
      }
    }
    // ---- element flux rows (kept in registers until the u-rows are gathered):
    //   q_x node (a, g): cqx sum_a2 MC(a, a2) qx[g][a2] - cbx (GB(a,0) p(g,0) + GB(a,1) p(g,1))
    //   q_y node (a, g): cqy sum_a2 MC(a, a2) qy[a2][g] - cby (GB(a,0) p(0,g) + GB(a,1) p(1,g))
    T fqx[2][3], fqy[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        T mx_ = 0, my_ = 0;
#pragma unroll
        for (int a2 = 0; a2 < 3; ++a2) {
          mx_ += T(MC(a, a2)) * qx[g][a2];
          my_ += T(MC(a, a2)) * qy[a2][g];
        }
        fqx[g][a] = cqx * mx_ - cbx * (T(GB(a, 0)) * pcur[g][0] + T(GB(a, 1)) * pcur[g][1]);
        fqy[a][g] = cqy * my_ - cby * (T(GB(a, 0)) * pcur[0][g] + T(GB(a, 1)) * pcur[1][g]);
      }
    // ---- p-rows (cell-local)
    T du[2][2], dq[2][2];
#pragma unroll
    for (int gy = 0; gy < 2; ++gy)
#pragma unroll
      for (int gx = 0; gx < 2; ++gx) {
        T sx = 0, sy = 0, tx = 0, ty = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
          for (int b = 0; b < 3; ++b) {
            sx += T(VG(gy, b) * DG(gx, a)) * ux[b][a];
            sy += T(DG(gy, b) * VG(gx, a)) * uy[b][a];
          }
          tx += T(DG(gx, a)) * qx[gy][a];
          ty += T(DG(gy, a)) * qy[a][gx];
        }
        du[gy][gx] = sx * ihx + sy * ihy;
        dq[gy][gx] = tx * ihx + ty * ihy;
      }
    if (!TR) {
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          const T z = bb * du[gy][gx] + Minv * pcur[gy][gx];
          if constexpr (LP) {
            Zs[LP && !TR ? lev : 0][gy * 2 + gx][LP && !TR ? tid : 0] = z;
            tdq[gy][gx] = tau * dq[gy][gx];
          } else {
#pragma unroll
            for (int l = 0; l < NL; ++l)
              yp[l][gy][gx] += T(tm.T[l * 4 + lev]) * z + ((l == lev) ? tau * dq[gy][gx] : T(0));
          }
        }
    } else if (owned) {
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
#pragma unroll
          for (int l = 0; l < NL; ++l) s += T(tm.T[l * 4 + lev]) * pl[l][gy][gx];
          Yl[op + qyb + gx + spx * gy] = -w2 * (tau * dq[gy][gx] + tau * bb * du[gy][gx] + Minv * s);
        }
    }
    __syncthreads();

    // ---- u-rows: each owned cell sums its lower-left 2x2 nodes (and the top/right
    // boundary nodes of the last cells) from the element rows of the cells sharing them
    if (owned) {
#pragma unroll 1
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            if ((a == 2 && !lastx) || (b == 2 && !lasty)) continue;
            const int mx = 2 * i + a, my = 2 * j + b;
            const int go = (c ? ou1 : ou0) + ub + a + sux * b;
            const bool fixed = my == 0 || (c == 0 && (mx == 0 || mx == 2 * nx));
            T v;
            if (fixed) {
              v = c ? uyr[b][a] : uxr[b][a];
            } else {
              v = 0;
#pragma unroll
              for (int sy = 0; sy < 2; ++sy) {
                // cells along y sharing row b: b == 0 -> (j-1: local 2), (j: local 0); else (j: local b)
                if (b != 0 && sy == 0) continue;
                const int lb = b != 0 ? b : (sy == 0 ? 2 : 0);
                const int dy = (b == 0 && sy == 0) ? -kT2 : 0;
#pragma unroll
                for (int sx = 0; sx < 2; ++sx) {
                  if (a != 0 && sx == 0) continue;
                  const int la = a != 0 ? a : (sx == 0 ? 2 : 0);
                  const int dx = (a == 0 && sx == 0) ? -1 : 0;
                  v += E[c * 9 + lb * 3 + la][tid + dy + dx];
                }
              }
            }
            Yl[go] = v;
          }
    }
    __syncthreads();
    // ---- flux rows: stage the element rows, then each owned cell sums its nodes
#pragma unroll
    for (int g = 0; g < 2; ++g)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        E[g * 3 + a][tid] = fqx[g][a];
        E[6 + a * 2 + g][tid] = fqy[a][g];
      }
    __syncthreads();
    if (owned) {
#pragma unroll 1
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          // q_x node (2i + a, 2j + g)
          if (!(a == 2 && !lastx)) {
            const int go = oq0 + ub + a + sux * g;
            const bool fixed = (a == 0 && i == 0) || (a == 2 && lastx);
            T v;
            if (fixed) v = g ? qxr[1][a] : qxr[0][a];
            else if (a == 0) v = E[g * 3 + 2][tid - 1] + E[g * 3 + 0][tid];
            else v = E[g * 3 + a][tid];
            Yl[go] = v;
          }
          // q_y node (2i + g, 2j + a)
          if (!(a == 2 && !lasty)) {
            const int go = oq1 + qyb + g + spx * a;
            const bool fixed = a == 0 && j == 0;
            T v;
            if (fixed) v = g ? qyr[a][1] : qyr[a][0];
            else if (a == 0) v = E[6 + 2 * 2 + g][tid - kT2] + E[6 + 0 * 2 + g][tid];
            else v = E[6 + a * 2 + g][tid];
            Yl[go] = v;
          }
        }
    }
    __syncthreads();
  }

  if (!TR && owned) {
    if constexpr (LP) {
      // the level loop's sum for this thread's level, same terms in the same order
      // (the loop's last barrier made every level's values visible)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T y = T(0);
#pragma unroll
          for (int l = 0; l < NL; ++l)
            y += T(tm.T[lev0 * 4 + l]) * Zs[LP && !TR ? l : 0][gy * 2 + gx][LP && !TR ? tid : 0] +
                 ((l == lev0) ? tdq[gy][gx] : T(0));
          Yb[lev0 * N + op + qyb + gx + spx * gy] = -w2 * y;
        }
    } else {
#pragma unroll
      for (int lev = 0; lev < NL; ++lev)
#pragma unroll
        for (int gy = 0; gy < 2; ++gy)
#pragma unroll
          for (int gx = 0; gx < 2; ++gx) Yb[lev * N + op + qyb + gx + spx * gy] = -w2 * yp[lev][gy][gx];
    }
  }
}

template <typename T, int NL, int TS, bool LP>
static void launch_ts(const ApplyArgs& a, const void* x, void* y, int transpose) {
  dim3 blk(TS, TS, LP ? NL : 1);
  if (transpose)
    hipLaunchKernelGGL((apply2d_kernel<T, NL, true, TS, LP>), dim3(a.nwork), blk, 0, a.stream, a.inst, a.work, *a.tm,
                       (const T*)a.kinv, (const T*)a.emat, (const T*)x, (T*)y);
  else
    hipLaunchKernelGGL((apply2d_kernel<T, NL, false, TS, LP>), dim3(a.nwork), blk, 0, a.stream, a.inst, a.work,
                       *a.tm, (const T*)a.kinv, (const T*)a.emat, (const T*)x, (T*)y);
}

template <typename T, int NL>
static void launch_nl(const ApplyArgs& a, const void* x, void* y, int transpose) {
  if (a.variant == 2) launch_ts<T, NL, 8, true>(a, x, y, transpose);
  else if (a.variant == 1) launch_ts<T, NL, 8, false>(a, x, y, transpose);
  else launch_ts<T, NL, 16, false>(a, x, y, transpose);
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

// tile variants: 0 = 16x16 threads (15x15 owned cells), 1 = 8x8 (7x7),
// 2 = 8x8 per time level, the levels in parallel (7x7)
int apply2d_variants() { return 3; }
int apply2d_tile_cells(int variant) { return variant >= 1 ? 7 : 15; }

}  // namespace bt
