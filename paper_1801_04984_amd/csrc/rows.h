// Node- and cell-local pieces of the slab operator shared by several kernels
// (any dimension): flux-row gathers tau Mq q and B p, DoF decoding, and the
// Gauss-2 point divergences used by the pressure rows.
#pragma once
#include "common.h"

namespace bt {

// blk: 0 = u, 1 = q, 2 = p; comp; coordinates in the block's nodal array
__device__ __forceinline__ void decode_dof(const InstDev& I, long long t, int& blk, int& comp, int co[3]) {
  const int d = I.dim;
  if (t >= I.off_p) {
    blk = 2; comp = 0;
    long long rem = t - I.off_p;
    for (int f = 0; f < 3; ++f) { co[f] = rem % I.sp[f]; rem /= I.sp[f]; }
    return;
  }
  if (t >= I.off_q[0]) {
    blk = 1; comp = 0;
    for (int c = 1; c < d; ++c)
      if (t >= I.off_q[c]) comp = c;
    long long rem = t - I.off_q[comp];
    for (int f = 0; f < 3; ++f) { co[f] = rem % I.sq[comp][f]; rem /= I.sq[comp][f]; }
    return;
  }
  blk = 0;
  comp = 0;
  for (int c = 1; c < d; ++c)
    if (t >= I.off_u[c]) comp = c;
  long long rem = t - I.off_u[comp];
  for (int f = 0; f < 3; ++f) { co[f] = rem % I.su[f]; rem /= I.su[f]; }
}

__device__ __forceinline__ long long p_index(const InstDev& I, int ox, int oy, int oz) {
  return I.off_p + ox + (long long)I.sp[0] * (oy + (long long)I.sp[1] * oz);
}

// (B p) at the flux node of component e with coordinates co (closed along e):
//   -hp_e sum_{cells of the node along e} sum_g GB(a, g) p(2c + g)
template <typename T>
__device__ T bp_node(const InstDev& I, const T* P, int e, const int co[3]) {
  const int d = I.dim;
  double hp = 1.0;
  for (int f = 0; f < d; ++f)
    if (f != e) hp *= 0.5 * I.h[f];
  const int m = co[e];
  double s = 0.0;
  for (int side = 0; side < 2; ++side) {
    int ce, a;
    if (m & 1) { if (side) break; ce = (m - 1) / 2; a = 1; }
    else { ce = m / 2 - 1 + side; a = side ? 0 : 2; if (ce < 0 || ce >= I.n[e]) continue; }
    int o[3] = {co[0], co[1], co[2]};
    o[e] = 2 * ce;
    const double p0 = (double)P[p_index(I, o[0], o[1], o[2])];
    o[e] = 2 * ce + 1;
    const double p1 = (double)P[p_index(I, o[0], o[1], o[2])];
    s += GB(a, 0) * p0 + GB(a, 1) * p1;
  }
  return (T)(-hp * s);
}

// tau Mq q at the flux node (e, co); dg receives the diagonal entry
template <typename T>
__device__ __forceinline__ T mq_node(const InstDev& I, const T* kc, const T* X, int e, const int co[3], T& dg) {
  const int d = I.dim;
  T hp = 1;
  for (int f = 0; f < d; ++f)
    if (f != e) hp *= T(0.5 * I.h[f]);
  const int m = co[e];
  const long long qstr_e = e == 0 ? 1 : (e == 1 ? (long long)I.sq[e][0] : (long long)I.sq[e][0] * I.sq[e][1]);
  long long base = I.off_q[e];
  {
    long long s = 1;
    for (int f = 0; f < d; ++f) {
      if (f != e) base += (long long)co[f] * s;
      s *= I.sq[e][f];
    }
  }
  T acc = 0;
  dg = 0;
  for (int side = 0; side < 2; ++side) {
    int ce, a;
    if (m & 1) { if (side) break; ce = (m - 1) / 2; a = 1; }
    else { ce = m / 2 - 1 + side; a = side ? 0 : 2; if (ce < 0 || ce >= I.n[e]) continue; }
    int cc[3] = {co[0] >> 1, co[1] >> 1, co[2] >> 1};
    cc[e] = ce;
    const long long cell = cc[0] + (long long)I.n[0] * (cc[1] + (long long)I.n[1] * (d == 3 ? cc[2] : 0));
    const T f = kc[cell] * T(I.tau * I.h[e]) * hp;
    T s = 0;
    for (int a2 = 0; a2 < 3; ++a2) {
      const int m2 = 2 * ce + a2;
      if (q_fixed(I, e, m2)) continue;
      s += T(MC(a, a2)) * X[base + m2 * qstr_e];
    }
    acc += f * s;
    dg += f * T(MC(a, a));
  }
  return acc;
}

// div u and div q of one level at the 2^d Gauss points of cell ce (x fastest), masked inputs
template <typename T, int DIM>
__device__ void cell_div(const InstDev& I, const T* Xl, const int ce[3], T du[1 << DIM], T dq[1 << DIM]) {
  constexpr int NG = 1 << DIM;
#pragma unroll
  for (int g = 0; g < NG; ++g) { du[g] = 0; dq[g] = 0; }
  const long long us[3] = {1, (long long)I.su[0], (long long)I.su[0] * I.su[1]};
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    const T ih = T(1.0 / I.h[c]);
    // u_c: closed in every axis
    for (int nidx = 0; nidx < (DIM == 3 ? 27 : 9); ++nidx) {
      const int a[3] = {nidx % 3, (nidx / 3) % 3, DIM == 3 ? nidx / 9 : 0};
      const int m[3] = {2 * ce[0] + a[0], 2 * ce[1] + a[1], DIM == 3 ? 2 * ce[2] + a[2] : 0};
      if (u_fixed(I, c, m[0], m[1], m[2])) continue;
      const T v = Xl[I.off_u[c] + m[0] + us[1] * m[1] + us[2] * m[2]];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        T f = ih;
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
          const int ge = (g >> e) & 1;
          f *= T(e == c ? DG(ge, a[e]) : VG(ge, a[e]));
        }
        du[g] += f * v;
      }
    }
    // q_c: closed along c, nodal (open) across
    long long qs[3], s = 1;
    for (int f = 0; f < 3; ++f) { qs[f] = s; s *= I.sq[c][f]; }
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      long long base = I.off_q[c];
#pragma unroll
      for (int f = 0; f < DIM; ++f)
        if (f != c) base += (long long)(2 * ce[f] + ((g >> f) & 1)) * qs[f];
      const int gc = (g >> c) & 1;
      T acc = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int mc = 2 * ce[c] + a;
        if (q_fixed(I, c, mc)) continue;
        acc += T(DG(gc, a)) * Xl[base + mc * qs[c]];
      }
      dq[g] += ih * acc;
    }
  }
}

}  // namespace bt
