// Fixed-stress flow/mechanics coupling terms and the flux-mass block.
//
// After the pressure correction p of a level block is known, the flux and
// displacement right-hand sides of the block-triangular fixed-stress step are
//   f_q = r_q - tau B p,     f_u = r_u + b tau E p
// (essential rows zero).  With the nodal bases both products are gathers
// from the DG-Q1 pressure of the cells around a node:
//   (B p)(q_e node m)  = -hp_e sum_{cells of m} sum_g GB(a, g) p(g)
//   (E p)(u_c node)    = sum_{cells} sum_g GB(a_c, g_c) prod_{f != c} (h_f/2) VG(g_f, a_f) p(g).
// In 3D one thread computes the three components of a displacement node, from one
// read of its cells' pressures.
// The flux block tau Mq is solved by Chebyshev-Jacobi; Mq acts only along the
// flux component's own axis (the open basis is orthogonal under 2-point
// Gauss) with the cellwise eta/K.
#include "prec.h"
#include "rows.h"

namespace bt {

static dim3 grid3(long long maxlen, int nseg, int nj) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b)), nseg, nj);
}

// (E p) of the three displacement components of one 3D node: the pressures of the
// node's cells are read once for all three (same terms, same order as ep_node)
template <typename T>
__device__ __forceinline__ void ep_node3(const InstDev& I, const T* __restrict__ P, const int co[3], double s[3]) {
  const double hx = 0.5 * I.h[0], hy = 0.5 * I.h[1], hz = 0.5 * I.h[2];
  s[0] = s[1] = s[2] = 0.0;
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
          const double p = (double)pc[gx + I.sp[0] * (gy + I.sp[1] * gz)];
          const double bx = gb_sel(ax, gx), vx = hx * vg_sel(gx, ax);
          const double by = gb_sel(ay, gy), vy = hy * vg_sel(gy, ay);
          const double bz = gb_sel(az, gz), vz = hz * vg_sel(gz, az);
          s[0] += bx * vy * vz * p;
          s[1] += vx * by * vz * p;
          s[2] += vx * vy * bz * p;
        }
      }
    }
  }
}

template <typename T, int DIM>
__global__ __launch_bounds__(256) void coupling_kernel(const InstDev* __restrict__ insts, LevelCoef cu,
                                                       const T* __restrict__ rt, const T* __restrict__ zp,
                                                       T* __restrict__ fu, T* __restrict__ fq) {
  const InstDev& I = insts[blockIdx.y];
  const int j = blockIdx.z;
  const T cuj = T(cu.c[j] * I.b);
  const long long lo = I.x_off + j * I.N;
  const T* P = zp + lo + I.off_p;
  const int nuq = (int)I.off_p;
  if constexpr (DIM == 3) {
    // one thread per displacement node (its three rows), then one per flux row
    const int nu1 = I.su[0] * I.su[1] * I.su[2];
    const int q0 = (int)I.off_q[0];
    const int nt = nu1 + (nuq - q0);
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += gridDim.x * blockDim.x) {
      if (t < nu1) {
        int co[3];
        unrank((unsigned)t, I.su, co);
        T r[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) r[c] = rt[lo + I.off_u[c] + t];
        double ep[3];
        ep_node3<T>(I, P, co, ep);
#pragma unroll
        for (int c = 0; c < 3; ++c)
          fu[lo + I.off_u[c] + t] = u_fixed(I, c, co[0], co[1], co[2]) ? T(0) : r[c] + cuj * (T)ep[c];
      } else {
        const int tq = q0 + (t - nu1);
        int blk, comp, co[3];
        decode_dof(I, tq, blk, comp, co);
        const T r = rt[lo + tq];
        T mq, dg, bp;
        flux_row<T, false>(I, nullptr, zp + lo, comp, co, tq - (int)I.off_q[comp], mq, dg, bp);
        fq[lo + tq] = q_fixed(I, comp, co[comp]) ? T(0) : r - T(I.tau) * bp;
      }
    }
    return;
  }
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nuq; t += gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode_dof(I, t, blk, comp, co);
    const T r = rt[lo + t];
    // the gathers run for essential rows too (their result is discarded), so
    // that no load waits behind a per-lane branch
    if (blk == 0) {
      const T ep = ep_node<T, DIM>(I, P, comp, co);
      fu[lo + t] = u_fixed(I, comp, co[0], co[1], co[2]) ? T(0) : r + cuj * ep;
    } else {
      T mq, dg, bp;
      flux_row<T, false>(I, nullptr, zp + lo, comp, co, t - (int)I.off_q[comp], mq, dg, bp);
      fq[lo + t] = q_fixed(I, comp, co[comp]) ? T(0) : r - T(I.tau) * bp;
    }
  }
}
template <typename T>
void launch_coupling(int dim, const InstDev* insts, int count, int nj, long long maxN, const LevelCoef& cu,
                     const T* rt, const T* zp, T* fu, T* fq, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL((coupling_kernel<T, 2>), grid3(maxN, count, nj), dim3(kBlk), 0, s, insts, cu, rt, zp, fu, fq);
  else
    hipLaunchKernelGGL((coupling_kernel<T, 3>), grid3(maxN, count, nj), dim3(kBlk), 0, s, insts, cu, rt, zp, fu, fq);
}
template void launch_coupling<double>(int, const InstDev*, int, int, long long, const LevelCoef&, const double*,
                                      const double*, double*, double*, hipStream_t);
template void launch_coupling<float>(int, const InstDev*, int, int, long long, const LevelCoef&, const float*,
                                     const float*, float*, float*, hipStream_t);

// ---- tau Mq and its Chebyshev solve ---------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void mq_kernel(const InstDev* __restrict__ insts, int mode, ChebCoef cc,
                                                 const T* __restrict__ kinv, const T* __restrict__ b,
                                                 T* __restrict__ x, T* __restrict__ r, const T* __restrict__ din,
                                                 T* __restrict__ dout) {
  const InstDev& I = insts[blockIdx.y];
  const int j = blockIdx.z;
  const long long lo = I.x_off + j * I.N;
  const T* kc = kinv + I.cell_off;
  const int q0 = (int)I.off_q[0], q1 = (int)I.off_p;
  for (int t = q0 + blockIdx.x * blockDim.x + threadIdx.x; t < q1; t += gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode_dof(I, t, blk, comp, co);
    if (q_fixed(I, comp, co[comp])) {
      if (mode == kResInitZero) { x[lo + t] = 0; r[lo + t] = 0; }
      dout[lo + t] = 0;
      continue;
    }
    const int loc = t - (int)I.off_q[comp];
    T Sd, dg, bp;
    if (mode == kResInitZero) {
      flux_row<T>(I, kc, b + lo, comp, co, loc, Sd, dg, bp);   // diagonal only
      const T rr = b[lo + t];
      x[lo + t] = 0;
      r[lo + t] = rr;
      dout[lo + t] = T(cc.s0) * rr / dg;
    } else if (mode == kStep) {
      flux_row<T>(I, kc, din + lo, comp, co, loc, Sd, dg, bp);
      const T dd = din[lo + t];
      x[lo + t] += dd;
      const T rr = r[lo + t] - Sd;
      r[lo + t] = rr;
      dout[lo + t] = T(cc.rho) * dd + T(cc.sig) * rr / dg;
    } else {
      flux_row<T>(I, kc, din + lo, comp, co, loc, Sd, dg, bp);
      dout[lo + t] = Sd / dg;
    }
  }
}
template <typename T>
void launch_mq(int dim, const InstDev* insts, int count, int nj, long long maxN, int mode, ChebCoef cc, const T* kinv,
               const T* dinvq, const T* b, T* x, T* r, const T* din, T* dout, hipStream_t s) {
  (void)dim;
  (void)dinvq;
  hipLaunchKernelGGL((mq_kernel<T>), grid3(maxN, count, nj), dim3(kBlk), 0, s, insts, mode, cc, kinv, b, x, r, din,
                     dout);
}
template void launch_mq<double>(int, const InstDev*, int, int, long long, int, ChebCoef, const double*, const double*,
                                const double*, double*, double*, const double*, double*, hipStream_t);
template void launch_mq<float>(int, const InstDev*, int, int, long long, int, ChebCoef, const float*, const float*,
                               const float*, float*, float*, const float*, float*, hipStream_t);

// ---- exact flux-mass solve: tau Mq x = b, line by line -------------------------------------
// Mq couples the nodes of q_e only along axis e (the open basis is orthogonal
// under 2-point Gauss across), so tau Mq is block diagonal with one banded
// SPD block per line of q_e nodes.  Within a cell the three nodes couple
// through f_c MC (f_c = eta/K_c tau h_e hp_e).  Condensing the cell-interior
// node leaves a tridiagonal system on the cell-end nodes:
//   diag_i = S00 (f_{i-1} + f_i),  off-diagonal (i, i+1) = S02 f_i,
//   rhs_i  = b_2i - (MC01 / MC11) (b_{2i-1} + b_{2i+1}),
// with S00 = MC00 - MC01^2 / MC11 and S02 = MC02 - MC01 MC12 / MC11; it is
// solved by a Thomas sweep and the interior node recovered from its row.
// Essential nodes stay zero (identity rows with zero right-hand side).
template <typename T, int DIM>
__global__ __launch_bounds__(256) void mq_line_kernel(const InstDev* __restrict__ insts, const T* __restrict__ kinv,
                                                      const T* __restrict__ b, T* __restrict__ x,
                                                      T* __restrict__ w) {
  constexpr double kS00 = MC(0, 0) - MC(0, 1) * MC(1, 0) / MC(1, 1);
  constexpr double kS02 = MC(0, 2) - MC(0, 1) * MC(1, 2) / MC(1, 1);
  constexpr double kR = MC(0, 1) / MC(1, 1);
  const InstDev& I = insts[blockIdx.y];
  const long long lo = I.x_off + blockIdx.z * I.N;
  const T* kc = kinv + I.cell_off;
  int nlines[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    int c = 1;
#pragma unroll
    for (int f = 0; f < DIM; ++f)
      if (f != e) c *= I.sp[f];
    nlines[e] = c;
  }
  const int total = nlines[0] + nlines[1] + nlines[2];
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < total; t += gridDim.x * blockDim.x) {
    const int e = t < nlines[0] ? 0 : (t < nlines[0] + nlines[1] ? 1 : 2);
    const int ln = t - (e == 0 ? 0 : (e == 1 ? nlines[0] : nlines[0] + nlines[1]));
    // open coordinates across the line (the two axes other than e, lower first)
    const int fa = e == 0 ? 1 : 0, fb = e == 2 ? 1 : 2;
    const int sa = I.sp[fa];
    const int oa = ln % sa, ob = DIM == 3 ? ln / sa : 0;
    // strides of q_e along e and across
    const int qs0 = I.sq[e][0], qs1 = I.sq[e][1];
    const int qstr[3] = {1, qs0, qs0 * qs1};
    const int cstr[3] = {1, I.n[0], I.n[0] * I.n[1]};
    const int base = oa * qstr[fa] + (DIM == 3 ? ob * qstr[fb] : 0);
    const int cbase = (oa >> 1) * cstr[fa] + (DIM == 3 ? (ob >> 1) * cstr[fb] : 0);
    const int qs = qstr[e], cs = cstr[e];
    const int n = I.n[e];
    double hp = 1.0;
#pragma unroll
    for (int f = 0; f < DIM; ++f)
      if (f != e) hp *= 0.5 * I.h[f];
    const T fsc = T(I.tau * I.h[e] * hp);
    const T* B = b + lo + I.off_q[e] + base;
    T* X = x + lo + I.off_q[e] + base;
    T* W = w + lo + I.off_q[e] + base;
    const bool top_free = e == DIM - 1;      // the top face carries no flux condition
    // forward sweep over the cell-end nodes i = 0..n (node 2i)
    T cprev = 0, dprev = 0, fprev = 0;
    for (int i = 0; i <= n; ++i) {
      const T fi = i < n ? kc[cbase + i * cs] * fsc : T(0);
      const bool fixed = i == 0 || (i == n && !top_free);
      T cp, dp;
      if (fixed) {
        cp = 0; dp = 0;
      } else {
        const T diag = T(kS00) * (fprev + fi);
        const T low = T(kS02) * fprev, up = T(kS02) * fi;
        T rhs = B[(2 * i) * qs];
        if (i > 0) rhs -= T(kR) * B[(2 * i - 1) * qs];
        if (i < n) rhs -= T(kR) * B[(2 * i + 1) * qs];
        const T den = diag - low * cprev;
        cp = up / den;
        dp = (rhs - low * dprev) / den;
      }
      W[(2 * i) * qs] = cp;
      X[(2 * i) * qs] = dp;
      cprev = cp; dprev = dp; fprev = fi;
    }
    // back substitution, interior nodes from their rows
    T xn = X[(2 * n) * qs];
    for (int i = n - 1; i >= 0; --i) {
      const T xi = X[(2 * i) * qs] - W[(2 * i) * qs] * xn;
      X[(2 * i) * qs] = xi;
      const T fi = kc[cbase + i * cs] * fsc;
      X[(2 * i + 1) * qs] = (B[(2 * i + 1) * qs] / fi - T(MC(1, 0)) * xi - T(MC(1, 2)) * xn) / T(MC(1, 1));
      xn = xi;
    }
  }
}
// The same condensed tridiagonal system, one wavefront per line: lane l holds
// the cell-end equations i = l, l + 64, ... (K per lane), and parallel cyclic
// reduction eliminates the couplings at distance 1, 2, 4, ... until every
// equation stands alone.  With a_i, b_i, c_i the couplings to i-s, i, i+s:
//   al = -a_i / b_{i-s},  ga = -c_i / b_{i+s},
//   a_i <- al a_{i-s},  c_i <- ga c_{i+s},
//   b_i <- b_i + al c_{i-s} + ga a_{i+s},  d_i <- d_i + al d_{i-s} + ga d_{i+s}
// (out-of-range neighbours are identity rows).  The condensed matrix is
// strictly diagonally dominant (|S00| = 3 |S02| per cell), so no pivoting is
// needed.  Equations beyond the line's end and essential nodes are identity rows.
template <typename T, int DIM, int K>
__global__ __launch_bounds__(64) void mq_pcr_kernel(const InstDev* __restrict__ insts, const T* __restrict__ kinv,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  constexpr int M = 64 * K;
  constexpr double kS00 = MC(0, 0) - MC(0, 1) * MC(1, 0) / MC(1, 1);
  constexpr double kS02 = MC(0, 2) - MC(0, 1) * MC(1, 2) / MC(1, 1);
  constexpr double kR = MC(0, 1) / MC(1, 1);
  __shared__ T sa[M], sb[M], sc[M], sd[M];
  const InstDev& I = insts[blockIdx.y];
  int nlines[3] = {0, 0, 0};
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    int c = 1;
#pragma unroll
    for (int f = 0; f < DIM; ++f)
      if (f != e) c *= I.sp[f];
    nlines[e] = c;
  }
  const int t = blockIdx.x;
  if (t >= nlines[0] + nlines[1] + nlines[2]) return;   // whole block
  const long long lo = I.x_off + blockIdx.z * I.N;
  const T* kc = kinv + I.cell_off;
  const int e = t < nlines[0] ? 0 : (t < nlines[0] + nlines[1] ? 1 : 2);
  const int ln = t - (e == 0 ? 0 : (e == 1 ? nlines[0] : nlines[0] + nlines[1]));
  const int fa = e == 0 ? 1 : 0, fb = e == 2 ? 1 : 2;
  const int sa_ = I.sp[fa];
  const int oa = ln % sa_, ob = DIM == 3 ? ln / sa_ : 0;
  const int qs0 = I.sq[e][0], qs1 = I.sq[e][1];
  const int qstr[3] = {1, qs0, qs0 * qs1};
  const int cstr[3] = {1, I.n[0], I.n[0] * I.n[1]};
  const int base = oa * qstr[fa] + (DIM == 3 ? ob * qstr[fb] : 0);
  const int cbase = (oa >> 1) * cstr[fa] + (DIM == 3 ? (ob >> 1) * cstr[fb] : 0);
  const int qs = qstr[e], cs = cstr[e];
  const int n = I.n[e];
  double hp = 1.0;
#pragma unroll
  for (int f = 0; f < DIM; ++f)
    if (f != e) hp *= 0.5 * I.h[f];
  const T fsc = T(I.tau * I.h[e] * hp);
  const T* B = b + lo + I.off_q[e] + base;
  T* X = x + lo + I.off_q[e] + base;
  const bool top_free = e == DIM - 1;
  const int lane = threadIdx.x;
  T f_own[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = lane + 64 * k;
    T a = 0, bd = 1, c = 0, d = 0, fi = 0;
    if (i <= n) {
      fi = i < n ? kc[cbase + i * cs] * fsc : T(0);
      const bool fixed = i == 0 || (i == n && !top_free);
      if (!fixed) {
        const T fp = kc[cbase + (i - 1) * cs] * fsc;   // i >= 1 here
        bd = T(kS00) * (fp + fi);
        a = T(kS02) * fp;
        c = T(kS02) * fi;
        d = B[(2 * i) * qs] - T(kR) * B[(2 * i - 1) * qs];
        if (i < n) d -= T(kR) * B[(2 * i + 1) * qs];
      }
    }
    f_own[k] = fi;
    sa[i] = a; sb[i] = bd; sc[i] = c; sd[i] = d;
  }
  __syncthreads();
  for (int st = 1; st <= n; st <<= 1) {
    T na[K], nb[K], nc[K], nd[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = lane + 64 * k;
      const T ai = sa[i], ci = sc[i];
      T al = 0, ga = 0, aL = 0, cL = 0, dL = 0, aR = 0, cR = 0, dR = 0;
      if (i - st >= 0) { al = -ai / sb[i - st]; aL = sa[i - st]; cL = sc[i - st]; dL = sd[i - st]; }
      if (i + st < M) { ga = -ci / sb[i + st]; aR = sa[i + st]; cR = sc[i + st]; dR = sd[i + st]; }
      na[k] = al * aL;
      nc[k] = ga * cR;
      nb[k] = sb[i] + al * cL + ga * aR;
      nd[k] = sd[i] + al * dL + ga * dR;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int i = lane + 64 * k;
      sa[i] = na[k]; sb[i] = nb[k]; sc[i] = nc[k]; sd[i] = nd[k];
    }
    __syncthreads();
  }
  // every equation now stands alone: x_i = d_i / b_i; then the interior nodes
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = lane + 64 * k;
    const T xi = sd[i] / sb[i];
    sa[i] = xi;
    if (i <= n) X[(2 * i) * qs] = xi;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int i = lane + 64 * k;
    if (i < n)
      X[(2 * i + 1) * qs] =
          (B[(2 * i + 1) * qs] / f_own[k] - T(MC(1, 0)) * sa[i] - T(MC(1, 2)) * sa[i + 1]) / T(MC(1, 1));
  }
}

template <typename T, int DIM>
static void launch_pcr(int K, dim3 g, const InstDev* insts, const T* kinv, const T* b, T* x, hipStream_t s) {
  switch (K) {
    case 1: hipLaunchKernelGGL((mq_pcr_kernel<T, DIM, 1>), g, dim3(64), 0, s, insts, kinv, b, x); break;
    case 2: hipLaunchKernelGGL((mq_pcr_kernel<T, DIM, 2>), g, dim3(64), 0, s, insts, kinv, b, x); break;
    case 4: hipLaunchKernelGGL((mq_pcr_kernel<T, DIM, 4>), g, dim3(64), 0, s, insts, kinv, b, x); break;
    default: hipLaunchKernelGGL((mq_pcr_kernel<T, DIM, 8>), g, dim3(64), 0, s, insts, kinv, b, x); break;
  }
}

template <typename T>
void launch_mq_lines(int dim, const InstDev* insts, int count, int nj, long long maxlines, int maxcells_line,
                     const T* kinv, const T* b, T* x, T* w, hipStream_t s) {
  if (maxcells_line <= kPcrMaxCells) {
    // equations per line = cells + 1, K per lane (a power of two)
    int K = 1;
    while (64 * K < maxcells_line + 1) K *= 2;
    const dim3 g((unsigned)maxlines, (unsigned)count, (unsigned)nj);
    if (dim == 2) launch_pcr<T, 2>(K, g, insts, kinv, b, x, s);
    else launch_pcr<T, 3>(K, g, insts, kinv, b, x, s);
    return;
  }
  if (dim == 2)
    hipLaunchKernelGGL((mq_line_kernel<T, 2>), grid3(maxlines, count, nj), dim3(kBlk), 0, s, insts, kinv, b, x, w);
  else
    hipLaunchKernelGGL((mq_line_kernel<T, 3>), grid3(maxlines, count, nj), dim3(kBlk), 0, s, insts, kinv, b, x, w);
}
template void launch_mq_lines<double>(int, const InstDev*, int, int, long long, int, const double*, const double*,
                                      double*, double*, hipStream_t);
template void launch_mq_lines<float>(int, const InstDev*, int, int, long long, int, const float*, const float*,
                                     float*, float*, hipStream_t);

// ---- finalize -----------------------------------------------------------------------------------
template <typename T, int NL>
__global__ __launch_bounds__(256) void finalize_kernel(const InstDev* __restrict__ insts, Mat4 Q, const T* __restrict__ zt,
                                const T* __restrict__ r, T* __restrict__ z) {
  const InstDev& I = insts[blockIdx.y];
  const int n = (int)I.N;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode_dof(I, t, blk, comp, co);
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
    case 1: hipLaunchKernelGGL((finalize_kernel<T, 1>), g, dim3(kBlk), 0, s, insts, Q, zt, r, z); break;
    case 2: hipLaunchKernelGGL((finalize_kernel<T, 2>), g, dim3(kBlk), 0, s, insts, Q, zt, r, z); break;
    case 3: hipLaunchKernelGGL((finalize_kernel<T, 3>), g, dim3(kBlk), 0, s, insts, Q, zt, r, z); break;
    default: hipLaunchKernelGGL((finalize_kernel<T, 4>), g, dim3(kBlk), 0, s, insts, Q, zt, r, z); break;
  }
}
template void launch_prec_finalize<double>(const InstDev*, int, long long, int, const Mat4&, const double*,
                                           const double*, double*, hipStream_t);
template void launch_prec_finalize<float>(const InstDev*, int, long long, int, const Mat4&, const float*,
                                          const float*, float*, hipStream_t);

}  // namespace bt
