// Node- and cell-local pieces of the slab operator shared by several kernels
// (any dimension): DoF decoding, the flux-row gathers tau Mq q and B p, the
// E p gather at a displacement node and the Gauss-2 point divergences used by
// the pressure rows.  Indices within one instance's level are 32-bit (the
// host rejects instances whose slab holds 2^31 unknowns or more).
#pragma once
#include "common.h"

namespace bt {

// coordinates of flat index t in a nodal array of sizes s (x fastest)
__device__ __forceinline__ void unrank(unsigned t, const int* s, int co[3]) {
  const unsigned s0 = (unsigned)s[0], s1 = (unsigned)s[1];
  const unsigned q = t / s0;
  const unsigned z = q / s1;
  co[0] = (int)(t - q * s0);
  co[1] = (int)(q - z * s1);
  co[2] = (int)z;
}

// blk: 0 = u, 1 = q, 2 = p; comp; coordinates in the block's nodal array
__device__ __forceinline__ void decode_dof(const InstDev& I, int t, int& blk, int& comp, int co[3]) {
  if (t >= (int)I.off_p) {
    blk = 2; comp = 0;
    unrank((unsigned)(t - (int)I.off_p), I.sp, co);
    return;
  }
  if (t >= (int)I.off_q[0]) {
    blk = 1;
    comp = (t >= (int)I.off_q[1] ? 1 : 0) + ((I.dim == 3 && t >= (int)I.off_q[2]) ? 1 : 0);
    unrank((unsigned)(t - (int)I.off_q[comp]), I.sq[comp], co);
    return;
  }
  blk = 0;
  comp = (t >= (int)I.off_u[1] ? 1 : 0) + ((I.dim == 3 && t >= (int)I.off_u[2]) ? 1 : 0);
  unrank((unsigned)(t - (int)I.off_u[comp]), I.su, co);
}

__device__ __forceinline__ int sel3(int e, const int v[3]) { return e == 0 ? v[0] : (e == 1 ? v[1] : v[2]); }

// cells of the 1D node m (closed coordinate) on an axis with n cells:
// side 0 = low cell (local node a = 2, or a = 1 for a midpoint), side 1 = high cell (a = 0)
__device__ __forceinline__ bool node_cell(int m, int n, int side, int& c, int& a) {
  if (m & 1) { c = m >> 1; a = 1; return side == 0; }
  if (side == 0) { c = (m >> 1) - 1; a = 2; return c >= 0; }
  c = m >> 1; a = 0;
  return c < n;
}

// 1D tables at a runtime local node a (second index compile-time after unrolling)
__device__ __forceinline__ double gb_sel(int a, int g) { return a == 0 ? GB(0, g) : (a == 1 ? GB(1, g) : GB(2, g)); }
__device__ __forceinline__ double vg_sel(int g, int a) { return a == 0 ? VG(g, 0) : (a == 1 ? VG(g, 1) : VG(g, 2)); }
__device__ __forceinline__ double mc_sel(int a, int b) { return a == 0 ? MC(0, b) : (a == 1 ? MC(1, b) : MC(2, b)); }
__device__ __forceinline__ double mc_diag(int a) { return a == 0 ? MC(0, 0) : (a == 1 ? MC(1, 1) : MC(2, 2)); }

// Flux row pieces at node co of q_e (local index `loc` within the q_e array)
// of one level Xl:  mq = tau (Mq q)(node) with essential q masked, dg = its
// diagonal entry (both only if MASS), bp = (B p)(node) =
// -hp_e sum_{cells of the node} sum_g GB(a, g) p(g).
template <typename T, bool MASS = true>
__device__ __forceinline__ void flux_row(const InstDev& I, const T* __restrict__ kc, const T* __restrict__ Xl, int e,
                                         const int co[3], int loc, T& mq, T& dg, T& bp) {
  const int d = I.dim;
  const int m = sel3(e, co);
  const int ne = sel3(e, I.n);
  const double he = e == 0 ? I.h[0] : (e == 1 ? I.h[1] : I.h[2]);
  double hp = 1.0;
  for (int f = 0; f < d; ++f)
    if (f != e) hp *= 0.5 * I.h[f];
  const int qstr = e == 0 ? 1 : (e == 1 ? I.sq[1][0] : I.sq[2][0] * I.sq[2][1]);
  const int cstr = e == 0 ? 1 : (e == 1 ? I.n[0] : I.n[0] * I.n[1]);
  const int pstr = e == 0 ? 1 : (e == 1 ? I.sp[0] : I.sp[0] * I.sp[1]);
  const T* Q = Xl + I.off_q[e] + (loc - m * qstr);           // line of q_e through the node
  const int cell0 = (co[0] >> 1) + I.n[0] * ((co[1] >> 1) + I.n[1] * (co[2] >> 1)) - (m >> 1) * cstr;
  const T* P = Xl + I.off_p + ((co[0] + I.sp[0] * (co[1] + I.sp[1] * co[2])) - m * pstr);
  const T fq = T(I.tau * he * hp);
  T acc = 0, dacc = 0;
  double sb = 0.0;
  // Both cells of the node are read at a clamped in-range cell (the missing one
  // contributes nothing), so that no load waits behind a per-lane branch.
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    int ce, a;
    const bool ok = node_cell(m, ne, side, ce, a);
    const int cc = ok ? ce : 0;
    const T kcv = MASS ? kc[cell0 + cc * cstr] : T(0);
    T qv[3];
#pragma unroll
    for (int a2 = 0; a2 < 3; ++a2) qv[a2] = MASS ? Q[(2 * cc + a2) * qstr] : T(0);
    const T p0 = P[(2 * cc) * pstr], p1 = P[(2 * cc + 1) * pstr];
    // the loaded values are used on every lane (weight 0 for a missing cell), so
    // the compiler cannot sink the loads back behind a branch
    const T wk = ok ? T(1) : T(0);
    if (MASS) {
      const T f = wk * kcv * fq;
      T s = 0;
#pragma unroll
      for (int a2 = 0; a2 < 3; ++a2) {
        const int m2 = 2 * cc + a2;
        s += (q_fixed(I, e, m2) ? T(0) : T(mc_sel(a, a2))) * qv[a2];
      }
      acc += f * s;
      dacc += f * T(mc_diag(a));
    }
    sb += (double)wk * (gb_sel(a, 0) * (double)p0 + gb_sel(a, 1) * (double)p1);
  }
  mq = acc;
  dg = dacc;
  bp = T(-hp * sb);
}

// (E p) at the u_c node co of one level's pressure block P:
//   sum_{cells of the node} sum_g GB(a_c, g_c) prod_{f != c} (h_f / 2) VG(g_f, a_f) p(g)
template <typename T, int DIM>
__device__ __forceinline__ T ep_node(const InstDev& I, const T* __restrict__ P, int c, const int co[3]) {
  double s = 0.0;
  const double hh[3] = {0.5 * I.h[0], 0.5 * I.h[1], DIM == 3 ? 0.5 * I.h[2] : 1.0};
  if constexpr (DIM == 3) {
    // 3D: cell by cell (reading all 64 values at once costs more registers than
    // it saves in waiting, measured on 48^3)
#pragma unroll
    for (int sz = 0; sz < 2; ++sz) {
      int cz, az;
      if (!node_cell(co[2], I.n[2], sz, cz, az)) continue;
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
        int cy, ay;
        if (!node_cell(co[1], I.n[1], sy, cy, ay)) continue;
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
          int cx, ax;
          if (!node_cell(co[0], I.n[0], sx, cx, ax)) continue;
          const T* pc = P + (2 * cx) + I.sp[0] * ((2 * cy) + I.sp[1] * (2 * cz));
#pragma unroll
          for (int g = 0; g < 8; ++g) {
            const int gx = g & 1, gy = (g >> 1) & 1, gz = (g >> 2) & 1;
            const double wx = c == 0 ? gb_sel(ax, gx) : hh[0] * vg_sel(gx, ax);
            const double wy = c == 1 ? gb_sel(ay, gy) : hh[1] * vg_sel(gy, ay);
            const double wz = c == 2 ? gb_sel(az, gz) : hh[2] * vg_sel(gz, az);
            s += wx * wy * wz * (double)pc[gx + I.sp[0] * (gy + I.sp[1] * gz)];
          }
        }
      }
    }
    return (T)s;
  }
  // 2D: cells of the node per axis (a missing cell is read at a clamped
  // in-range cell and contributes nothing), so that no load waits behind a branch
  int cx[2], ax[2], cy[2], ay[2], cz[2], az[2];
  bool okx[2], oky[2], okz[2];
#pragma unroll
  for (int sd = 0; sd < 2; ++sd) {
    okx[sd] = node_cell(co[0], I.n[0], sd, cx[sd], ax[sd]);
    oky[sd] = node_cell(co[1], I.n[1], sd, cy[sd], ay[sd]);
    if (DIM == 3) okz[sd] = node_cell(co[2], I.n[2], sd, cz[sd], az[sd]);
    else { okz[sd] = sd == 0; cz[sd] = 0; az[sd] = 0; }
    if (!okx[sd]) cx[sd] = 0;
    if (!oky[sd]) cy[sd] = 0;
    if (!okz[sd]) cz[sd] = 0;
  }
  constexpr int NG = 1 << DIM;
#pragma unroll
  for (int sz = 0; sz < (DIM == 3 ? 2 : 1); ++sz)
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const T* pc = P + (2 * cx[sx]) + I.sp[0] * ((2 * cy[sy]) + I.sp[1] * (2 * cz[sz]));
        T pv[NG];
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const int gx = g & 1, gy = (g >> 1) & 1, gz = (g >> 2) & 1;
          pv[g] = pc[gx + I.sp[0] * (gy + I.sp[1] * gz)];
        }
        // weight 0 for a missing cell: the loaded values are used on every lane
        const double wm = (okx[sx] && oky[sy] && okz[sz]) ? 1.0 : 0.0;
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          const int gx = g & 1, gy = (g >> 1) & 1, gz = (g >> 2) & 1;
          const double wx = wm * (c == 0 ? gb_sel(ax[sx], gx) : hh[0] * vg_sel(gx, ax[sx]));
          const double wy = c == 1 ? gb_sel(ay[sy], gy) : hh[1] * vg_sel(gy, ay[sy]);
          double w = wx * wy;
          if (DIM == 3) w *= c == 2 ? gb_sel(az[sz], gz) : hh[2] * vg_sel(gz, az[sz]);
          s += w * (double)pv[g];
        }
      }
  return (T)s;
}

// div u of one level at the 2^DIM Gauss points of cell ce (x fastest),
// essential values masked.  Sum factorisation: per component c the nodal
// values are contracted axis by axis with the 2x3 tables DG (derivative, axis
// c) and VG (value, other axes), which keeps the constants to those two tables.
template <typename T, int DIM>
__device__ __forceinline__ void cell_divu(const InstDev& I, const T* __restrict__ Xl, const int ce[3],
                                          T du[1 << DIM]) {
  constexpr int NG = 1 << DIM;
  constexpr int NZ = DIM == 3 ? 3 : 1, GZ = DIM == 3 ? 2 : 1;
#pragma unroll
  for (int g = 0; g < NG; ++g) du[g] = 0;
  const int su0 = I.su[0], su1 = I.su[1];
  const bool bx0 = ce[0] == 0, bx1 = ce[0] == I.n[0] - 1;
  const bool by0 = ce[1] == 0, by1 = ce[1] == I.n[1] - 1;
  const bool bz0 = DIM == 3 ? ce[2] == 0 : false;
  const int nb = 2 * ce[0] + su0 * (2 * ce[1] + su1 * (DIM == 3 ? 2 * ce[2] : 0));
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const T ih = T(1.0 / I.h[c]);
    const T* U = Xl + I.off_u[c] + nb;
    T v[NZ][3][3];
#pragma unroll
    for (int az = 0; az < NZ; ++az)
#pragma unroll
      for (int ay = 0; ay < 3; ++ay)
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          // essential u_c: bottom face (all components), lateral faces (normal component)
          bool fx = DIM == 3 ? (az == 0 && bz0) : (ay == 0 && by0);
          if (c == 0) fx = fx || (ax == 0 && bx0) || (ax == 2 && bx1);
          if (DIM == 3 && c == 1) fx = fx || (ay == 0 && by0) || (ay == 2 && by1);
          const T raw = U[ax + su0 * (ay + su1 * az)];
          v[az][ay][ax] = fx ? T(0) : raw;
        }
    // contract x, then y, then z
    T tx[NZ][3][2];
#pragma unroll
    for (int az = 0; az < NZ; ++az)
#pragma unroll
      for (int ay = 0; ay < 3; ++ay)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) s += T(c == 0 ? DG(gx, ax) : VG(gx, ax)) * v[az][ay][ax];
          tx[az][ay][gx] = s;
        }
    T ty[NZ][2][2];
#pragma unroll
    for (int az = 0; az < NZ; ++az)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
#pragma unroll
          for (int ay = 0; ay < 3; ++ay) s += T(c == 1 ? DG(gy, ay) : VG(gy, ay)) * tx[az][ay][gx];
          ty[az][gy][gx] = s;
        }
#pragma unroll
    for (int gz = 0; gz < GZ; ++gz)
#pragma unroll
      for (int gy = 0; gy < 2; ++gy)
#pragma unroll
        for (int gx = 0; gx < 2; ++gx) {
          T s = 0;
          if (DIM == 3) {
#pragma unroll
            for (int az = 0; az < NZ; ++az) s += T(c == 2 ? DG(gz, az) : VG(gz, az)) * ty[az][gy][gx];
          } else {
            s = ty[0][gy][gx];
          }
          du[gx + 2 * gy + 4 * gz] += ih * s;
        }
  }
}

// div q of one level at the 2^DIM Gauss points of cell ce; q_c is closed
// along c (3 nodes) and nodal (open) across, essential values masked.
template <typename T, int DIM>
__device__ __forceinline__ void cell_divq(const InstDev& I, const T* __restrict__ Xl, const int ce[3],
                                          T dq[1 << DIM]) {
  constexpr int NG = 1 << DIM;
#pragma unroll
  for (int g = 0; g < NG; ++g) dq[g] = 0;
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const T ih = T(1.0 / I.h[c]);
    const int qs0 = I.sq[c][0], qs1 = I.sq[c][1];
    const int mc0 = 2 * ce[c];
    const bool lo_fixed = q_fixed(I, c, mc0), hi_fixed = q_fixed(I, c, mc0 + 2);
    const int cstr = c == 0 ? 1 : (c == 1 ? qs0 : qs0 * qs1);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      int o[3] = {2 * ce[0] + (g & 1), 2 * ce[1] + ((g >> 1) & 1), DIM == 3 ? 2 * ce[2] + ((g >> 2) & 1) : 0};
      const int gc = (g >> c) & 1;
      if (c == 0) o[0] = mc0;
      if (c == 1) o[1] = mc0;
      if (c == 2) o[2] = mc0;
      const T* Q = Xl + I.off_q[c] + (o[0] + qs0 * (o[1] + qs1 * o[2]));
      // essential end nodes masked by their weight, not by a branch around the load
      const T q0 = Q[0], q1 = Q[cstr], q2 = Q[2 * cstr];
      T acc = T(DG(gc, 1)) * q1;
      acc += (lo_fixed ? T(0) : T(DG(gc, 0))) * q0;
      acc += (hi_fixed ? T(0) : T(DG(gc, 2))) * q2;
      dq[g] += ih * acc;
    }
  }
}

}  // namespace bt
