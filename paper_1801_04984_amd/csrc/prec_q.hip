// Fixed-stress flow/mechanics coupling terms and the flux-mass block.
//
// After the pressure correction p of a level block is known, the flux and
// displacement right-hand sides of the block-triangular fixed-stress step are
//   f_q = r_q - tau B p,     f_u = r_u + b tau E p
// (essential rows zero).  With the nodal bases both products are gathers
// from the DG-Q1 pressure of the cells around a node:
//   (B p)(q_e node m)  = -hp_e sum_{cells of m} sum_g GB(a, g) p(g)
//   (E p)(u_c node)    = sum_{cells} sum_g GB(a_c, g_c) prod_{f != c} (h_f/2) VG(g_f, a_f) p(g).
// The flux block tau Mq is solved by Chebyshev-Jacobi; Mq acts only along the
// flux component's own axis (the open basis is orthogonal under 2-point
// Gauss) with the cellwise eta/K.
#include "prec.h"

namespace bt {

static dim3 grid3(long long maxlen, int nseg, int nj) {
  long long b = (maxlen + 255) / 256;
  return dim3((unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b)), nseg, nj);
}

__device__ __forceinline__ void decode(const InstDev& I, long long t, int& blk, int& comp, int co[3]) {
  // blk: 0 = u, 1 = q, 2 = p
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

__device__ __forceinline__ long long pidx(const InstDev& I, int ox, int oy, int oz) {
  return I.off_p + ox + (long long)I.sp[0] * (oy + (long long)I.sp[1] * oz);
}

template <typename T>
__device__ T bp_at(const InstDev& I, const T* P, int e, const int co[3]) {
  // (B p) at flux node of component e with coordinates co (closed along e)
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
    const double p0 = (double)P[pidx(I, o[0], o[1], o[2])];
    o[e] = 2 * ce + 1;
    const double p1 = (double)P[pidx(I, o[0], o[1], o[2])];
    s += GB(a, 0) * p0 + GB(a, 1) * p1;
  }
  return (T)(-hp * s);
}

template <typename T>
__device__ T ep_at(const InstDev& I, const T* P, int c, const int co[3]) {
  // (E p) at the u_c node co: sum over cells sharing the node, Gauss-2 collocation
  const int d = I.dim;
  int cl[3][2], al[3][2], nl[3];
  for (int f = 0; f < 3; ++f) {
    nl[f] = 0;
    if (f >= d) { cl[f][0] = 0; al[f][0] = 0; nl[f] = 1; continue; }
    const int m = co[f];
    if (m & 1) { cl[f][0] = (m - 1) / 2; al[f][0] = 1; nl[f] = 1; }
    else {
      if (m / 2 - 1 >= 0) { cl[f][nl[f]] = m / 2 - 1; al[f][nl[f]] = 2; ++nl[f]; }
      if (m / 2 < I.n[f]) { cl[f][nl[f]] = m / 2; al[f][nl[f]] = 0; ++nl[f]; }
    }
  }
  double s = 0.0;
  for (int iz = 0; iz < nl[2]; ++iz)
    for (int iy = 0; iy < nl[1]; ++iy)
      for (int ix = 0; ix < nl[0]; ++ix) {
        const int cc[3] = {cl[0][ix], cl[1][iy], cl[2][iz]};
        const int aa[3] = {al[0][ix], al[1][iy], al[2][iz]};
        for (int g = 0; g < (d == 3 ? 8 : 4); ++g) {
          const int gg[3] = {g & 1, (g >> 1) & 1, (g >> 2) & 1};
          double w = 1.0;
          for (int f = 0; f < d; ++f) w *= (f == c) ? GB(aa[f], gg[f]) : 0.5 * I.h[f] * VG(gg[f], aa[f]);
          s += w * (double)P[pidx(I, 2 * cc[0] + gg[0], 2 * cc[1] + gg[1], d == 3 ? 2 * cc[2] + gg[2] : 0)];
        }
      }
  return (T)s;
}

template <typename T>
__global__ __launch_bounds__(256) void coupling_kernel(const InstDev* __restrict__ insts, const T* __restrict__ rt, const T* __restrict__ zp,
                                T* __restrict__ fu, T* __restrict__ fq) {
  const InstDev& I = insts[blockIdx.y];
  const int j = blockIdx.z;
  const long long lo = I.x_off + j * I.N;
  const T* P = zp + lo;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.off_p;
       t += (long long)gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode(I, t, blk, comp, co);
    if (blk == 0) {
      T v = 0;
      if (!u_fixed(I, comp, co[0], co[1], co[2])) v = rt[lo + t] + T(I.b * I.tau) * ep_at<T>(I, P, comp, co);
      fu[lo + t] = v;
    } else {
      T v = 0;
      if (!q_fixed(I, comp, co[comp])) v = rt[lo + t] - T(I.tau) * bp_at<T>(I, P, comp, co);
      fq[lo + t] = v;
    }
  }
}
template <typename T>
void launch_coupling(int dim, const InstDev* insts, int count, int nj, long long maxN, const T* rt, const T* zp, T* fu,
                     T* fq, hipStream_t s) {
  (void)dim;
  hipLaunchKernelGGL((coupling_kernel<T>), grid3(maxN, count, nj), dim3(256), 0, s, insts, rt, zp, fu, fq);
}
template void launch_coupling<double>(int, const InstDev*, int, int, long long, const double*, const double*,
                                      double*, double*, hipStream_t);
template void launch_coupling<float>(int, const InstDev*, int, int, long long, const float*, const float*, float*,
                                     float*, hipStream_t);

// ---- tau Mq and its Chebyshev solve ---------------------------------------------------------
template <typename T>
__device__ __forceinline__ T mq_at(const InstDev& I, const T* kc, const T* X, int e, const int co[3], T& dg) {
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

template <typename T>
__global__ __launch_bounds__(256) void mq_kernel(const InstDev* __restrict__ insts, int mode, ChebCoef cc, const T* __restrict__ kinv,
                          const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ din,
                          T* __restrict__ dout) {
  const InstDev& I = insts[blockIdx.y];
  const int j = blockIdx.z;
  const long long lo = I.x_off + j * I.N;
  const T* kc = kinv + I.cell_off;
  for (long long t = I.off_q[0] + (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.off_p;
       t += (long long)gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode(I, t, blk, comp, co);
    if (q_fixed(I, comp, co[comp])) {
      if (mode == kResInitZero) { x[lo + t] = 0; r[lo + t] = 0; }
      dout[lo + t] = 0;
      continue;
    }
    if (mode == kResInitZero) {
      T dg;
      mq_at<T>(I, kc, b + lo, comp, co, dg);   // diagonal only
      const T rr = b[lo + t];
      x[lo + t] = 0;
      r[lo + t] = rr;
      dout[lo + t] = T(cc.s0) * rr / dg;
    } else if (mode == kStep) {
      T dg;
      const T Sd = mq_at<T>(I, kc, din + lo, comp, co, dg);
      const T dd = din[lo + t];
      x[lo + t] += dd;
      const T rr = r[lo + t] - Sd;
      r[lo + t] = rr;
      dout[lo + t] = T(cc.rho) * dd + T(cc.sig) * rr / dg;
    } else {
      T dg;
      const T Sx = mq_at<T>(I, kc, din + lo, comp, co, dg);
      dout[lo + t] = Sx / dg;
    }
  }
}
template <typename T>
void launch_mq(int dim, const InstDev* insts, int count, int nj, long long maxN, int mode, ChebCoef cc, const T* kinv,
               const T* dinvq, const T* b, T* x, T* r, const T* din, T* dout, hipStream_t s) {
  (void)dim;
  (void)dinvq;
  hipLaunchKernelGGL((mq_kernel<T>), grid3(maxN, count, nj), dim3(256), 0, s, insts, mode, cc, kinv, b, x, r, din,
                     dout);
}
template void launch_mq<double>(int, const InstDev*, int, int, long long, int, ChebCoef, const double*, const double*,
                                const double*, double*, double*, const double*, double*, hipStream_t);
template void launch_mq<float>(int, const InstDev*, int, int, long long, int, ChebCoef, const float*, const float*,
                               const float*, float*, float*, const float*, float*, hipStream_t);

// ---- finalize -----------------------------------------------------------------------------------
template <typename T, int NL>
__global__ __launch_bounds__(256) void finalize_kernel(const InstDev* __restrict__ insts, Mat4 Q, const T* __restrict__ zt,
                                const T* __restrict__ r, T* __restrict__ z) {
  const InstDev& I = insts[blockIdx.y];
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode(I, t, blk, comp, co);
    bool fixed = false;
    if (blk == 0) fixed = u_fixed(I, comp, co[0], co[1], co[2]);
    else if (blk == 1) fixed = q_fixed(I, comp, co[comp]);
    T v[NL];
#pragma unroll
    for (int l = 0; l < NL; ++l) v[l] = zt[I.x_off + l * I.N + t];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      T s = 0;
#pragma unroll
      for (int l = 0; l < NL; ++l) s += T(Q.m[i * 4 + l]) * v[l];
      z[I.x_off + i * I.N + t] = fixed ? r[I.x_off + i * I.N + t] : s;
    }
  }
}
template <typename T>
void launch_prec_finalize(const InstDev* insts, int count, long long maxN, int nl, const Mat4& Q, const T* zt,
                          const T* r, T* z, hipStream_t s) {
  dim3 g = grid3(maxN, count, 1);
  switch (nl) {
    case 1: hipLaunchKernelGGL((finalize_kernel<T, 1>), g, dim3(256), 0, s, insts, Q, zt, r, z); break;
    case 2: hipLaunchKernelGGL((finalize_kernel<T, 2>), g, dim3(256), 0, s, insts, Q, zt, r, z); break;
    case 3: hipLaunchKernelGGL((finalize_kernel<T, 3>), g, dim3(256), 0, s, insts, Q, zt, r, z); break;
    default: hipLaunchKernelGGL((finalize_kernel<T, 4>), g, dim3(256), 0, s, insts, Q, zt, r, z); break;
  }
}
template void launch_prec_finalize<double>(const InstDev*, int, long long, int, const Mat4&, const double*,
                                           const double*, double*, hipStream_t);
template void launch_prec_finalize<float>(const InstDev*, int, long long, int, const Mat4&, const float*,
                                          const float*, float*, hipStream_t);

}  // namespace bt
