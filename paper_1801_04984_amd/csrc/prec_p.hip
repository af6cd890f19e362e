// Pressure Schur-complement multigrid (fixed-stress flow block).
//
// S_j = c_j Mp + tau B^T Dq^-1 B  on the DG-Q1 pressure, c_j = alpha_j (1/M + L),
// Dq = diag(Mq).  Fine level: matrix free.  Along axis e the product
// B^T Dq^-1 B couples the pressure DoFs of a line through the three closed
// flux nodes of each cell:
//   (B^T Dq^-1 B x)_o = hp_e^2 sum_{a} GB(a, g_o) Dq^-1(m_a) sum_{cells c' of m_a} sum_g' GB(a', g') x_{c', g'}
// (hp_e = prod_{f != e} h_f / 2; Mp = diag(prod h_f / 2)).
// Coarse levels: Galerkin products with the cell-constant restriction; they
// are exactly two-point-flux cell stencils with face transmissibilities
// t = tau hp^2 sum_{face flux nodes} Dq^-1 (the interior flux node carries
// no constant mode), a Dirichlet-type term on the drained top face, and the
// cell mass.  Further levels aggregate 2^d cells (sums of coefficients).
#include "prec.h"
#include "rows.h"

namespace bt {

static dim3 grid3(long long maxlen, int nseg, int nj) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b)), nseg, nj);
}

// ---- fine DG level -------------------------------------------------------------
template <typename T, int DIM>
__device__ __forceinline__ void pdg_eval(const InstDev& I, const T* __restrict__ x, const T* __restrict__ dqi,
                                         long long o, T cm, T& Sx, T& diag) {
  int oc[3] = {0, 0, 0};
  long long rem = o;
  oc[0] = rem % I.sp[0]; rem /= I.sp[0];
  oc[1] = rem % I.sp[1]; rem /= I.sp[1];
  if (DIM == 3) oc[2] = (int)rem;
  T wp = 1;
#pragma unroll
  for (int e = 0; e < DIM; ++e) wp *= T(0.5 * I.h[e]);
  const T xo = x[o];
  Sx = cm * wp * xo;
  diag = cm * wp;
  const long long pstr[3] = {1, (long long)I.sp[0], (long long)I.sp[0] * I.sp[1]};
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    const int ce = oc[e] >> 1, ge = oc[e] & 1;
    T hp = 1;
#pragma unroll
    for (int f = 0; f < DIM; ++f)
      if (f != e) hp *= T(0.5 * I.h[f]);
    // flux node index of q_e: closed coord m along e, open coords elsewhere
    long long qbase = I.off_q[e];
    long long qstr_e = 1, s = 1;
    long long qoth = 0;
#pragma unroll
    for (int f = 0; f < DIM; ++f) {
      if (f == e) qstr_e = s;
      else qoth += (long long)oc[f] * s;
      s *= I.sq[e][f];
    }
    const long long lineo = o - (long long)oc[e] * pstr[e];   // p index with coord e = 0
    T acc = 0, dacc = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int m = 2 * ce + a;
      const T di = dqi[qbase + qoth + m * qstr_e];
      if (di == T(0)) continue;
      T bx = 0;
      // cells sharing node m along e
      if (a == 1) {
        bx = T(GB(1, 0)) * x[lineo + (2 * ce) * pstr[e]] + T(GB(1, 1)) * x[lineo + (2 * ce + 1) * pstr[e]];
      } else {
        const int cl = (a == 0) ? ce - 1 : ce;      // cell on the low side of node m
        const int ch = cl + 1;
        if (cl >= 0)
          bx += T(GB(2, 0)) * x[lineo + (2 * cl) * pstr[e]] + T(GB(2, 1)) * x[lineo + (2 * cl + 1) * pstr[e]];
        if (ch < I.n[e])
          bx += T(GB(0, 0)) * x[lineo + (2 * ch) * pstr[e]] + T(GB(0, 1)) * x[lineo + (2 * ch + 1) * pstr[e]];
      }
      acc += T(GB(a, ge)) * di * bx;
      dacc += T(GB(a, ge)) * T(GB(a, ge)) * di;
    }
    Sx += T(I.tau) * hp * hp * acc;
    diag += T(I.tau) * hp * hp * dacc;
  }
}

// S x on the 2^DIM pressure DoFs of cell ce (x: p-block of one level).  Per
// axis e and per line through the cell along e, the three flux nodes of the
// cell are shared by the two DoFs of the line.
template <typename T, int DIM>
__device__ __forceinline__ void pdg_cell(const InstDev& I, const T* __restrict__ x, const T* __restrict__ dqi,
                                         const int ce[3], T cm, T Sx[1 << DIM]) {
  constexpr int NG = 1 << DIM;
  const long long pstr[3] = {1, (long long)I.sp[0], (long long)I.sp[0] * I.sp[1]};
  long long base = 0;
#pragma unroll
  for (int e = 0; e < DIM; ++e) base += (long long)(2 * ce[e]) * pstr[e];
  T wp = 1;
#pragma unroll
  for (int e = 0; e < DIM; ++e) wp *= T(0.5 * I.h[e]);
#pragma unroll
  for (int g = 0; g < NG; ++g) {
    long long o = base;
#pragma unroll
    for (int e = 0; e < DIM; ++e) o += ((g >> e) & 1) * pstr[e];
    Sx[g] = cm * wp * x[o];
  }
#pragma unroll
  for (int e = 0; e < DIM; ++e) {
    T hp = 1;
#pragma unroll
    for (int f = 0; f < DIM; ++f)
      if (f != e) hp *= T(0.5 * I.h[f]);
    const T c2 = T(I.tau) * hp * hp;
    // flux node strides of q_e: closed along e, open elsewhere
    long long qs[3], sacc = 1;
#pragma unroll
    for (int f = 0; f < DIM; ++f) { qs[f] = sacc; sacc *= I.sq[e][f]; }
    const bool has_lo = ce[e] > 0, has_hi = ce[e] + 1 < I.n[e];
#pragma unroll
    for (int line = 0; line < (NG >> 1); ++line) {
      // DoF index of the line's low DoF: insert a 0 bit for axis e into `line`
      const int g0 = ((line >> e) << (e + 1)) | (line & ((1 << e) - 1));
      long long lb = base, qb = I.off_q[e];
#pragma unroll
      for (int f = 0; f < DIM; ++f)
        if (f != e) {
          const int gf = (g0 >> f) & 1;
          lb += gf * pstr[f];
          qb += (long long)(2 * ce[f] + gf) * qs[f];
        }
      // neighbour loads at clamped (in-range) indices, masked afterwards: no
      // load sits behind a branch, so all of them are in flight together
      const long long lo_b = has_lo ? lb - 2 * pstr[e] : lb, hi_b = has_hi ? lb + 2 * pstr[e] : lb;
      const T x0 = x[lb], x1 = x[lb + pstr[e]];
      const T vl0 = x[lo_b], vl1 = x[lo_b + pstr[e]], vh0 = x[hi_b], vh1 = x[hi_b + pstr[e]];
      const T xl0 = has_lo ? vl0 : T(0), xl1 = has_lo ? vl1 : T(0);
      const T xh0 = has_hi ? vh0 : T(0), xh1 = has_hi ? vh1 : T(0);
      const long long qn = qb + (long long)(2 * ce[e]) * qs[e];
      const T d0 = dqi[qn], d1 = dqi[qn + qs[e]], d2 = dqi[qn + 2 * qs[e]];
      const T own2 = T(GB(2, 0)) * x0 + T(GB(2, 1)) * x1, own0 = T(GB(0, 0)) * x0 + T(GB(0, 1)) * x1;
      const T b0 = (T(GB(2, 0)) * xl0 + T(GB(2, 1)) * xl1) + own0;     // node 2ce   (cells ce-1, ce)
      const T b1 = T(GB(1, 0)) * x0 + T(GB(1, 1)) * x1;                // node 2ce+1 (cell ce)
      const T b2 = own2 + (T(GB(0, 0)) * xh0 + T(GB(0, 1)) * xh1);     // node 2ce+2 (cells ce, ce+1)
      const T f0 = d0 * b0, f1 = d1 * b1, f2 = d2 * b2;
      Sx[g0] += c2 * (T(GB(0, 0)) * f0 + T(GB(1, 0)) * f1 + T(GB(2, 0)) * f2);
      Sx[g0 | (1 << e)] += c2 * (T(GB(0, 1)) * f0 + T(GB(1, 1)) * f1 + T(GB(2, 1)) * f2);
    }
  }
}

template <typename T, int DIM, int MODE>
__global__ __launch_bounds__(256) void pdg_kernel(const PDgSeg* __restrict__ segs, ChebCoef cc,
                           const T* __restrict__ dqinv, const T* __restrict__ dinv,
                           const T* __restrict__ b, T* __restrict__ x, T* __restrict__ r,
                           const T* __restrict__ din, T* __restrict__ dout) {
  constexpr int NG = 1 << DIM;
  const PDgSeg& sg = segs[blockIdx.y];
  const InstDev& I = sg.I;
  const int j = blockIdx.z;
  const long long vo = sg.voff + j * sg.vjstride;
  const long long dof = sg.doff + j * sg.djstride;
  const T* dqi = dqinv + sg.dqoff;
  const T cm = T(sg.cm[j]);
  const long long pstr[3] = {1, (long long)I.sp[0], (long long)I.sp[0] * I.sp[1]};
  const int ncl = (int)I.ncells;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncl; c += gridDim.x * blockDim.x) {
    int ce[3];
    unrank((unsigned)c, I.n, ce);
    long long base = 0;
#pragma unroll
    for (int e = 0; e < DIM; ++e) base += (long long)(2 * ce[e]) * pstr[e];
    long long oo[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      long long o = base;
#pragma unroll
      for (int e = 0; e < DIM; ++e) o += ((g >> e) & 1) * pstr[e];
      oo[g] = o;
    }
    if constexpr (MODE == kResInitZero) {            // x = 0: r = bsign b, d = s0 Dinv r
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const T rr = T(cc.bsign) * b[vo + oo[g]];
        x[vo + oo[g]] = 0;
        r[vo + oo[g]] = rr;
        dout[vo + oo[g]] = T(cc.s0) * dinv[dof + oo[g]] * rr;
      }
    } else if constexpr (MODE == kResInit) {         // r = bsign b - S x, d = s0 Dinv r
      // every load precedes every store, so the loads are all in flight together
      T bv[NG], dv[NG], Sx[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) { bv[g] = b[vo + oo[g]]; dv[g] = dinv[dof + oo[g]]; }
      pdg_cell<T, DIM>(I, x + vo, dqi, ce, cm, Sx);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const T rr = T(cc.bsign) * bv[g] - Sx[g];
        r[vo + oo[g]] = rr;
        dout[vo + oo[g]] = T(cc.s0) * dv[g] * rr;
      }
    } else if constexpr (MODE == kStep) {            // x += d; r -= S d; d' = rho d + sig Dinv r
      T dd[NG], xv[NG], rv[NG], dv[NG], Sd[NG];
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        dd[g] = din[vo + oo[g]];
        xv[g] = x[vo + oo[g]];
        rv[g] = r[vo + oo[g]];
        dv[g] = dinv[dof + oo[g]];
      }
      pdg_cell<T, DIM>(I, din + vo, dqi, ce, cm, Sd);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        x[vo + oo[g]] = xv[g] + dd[g];
        const T rr = rv[g] - Sd[g];
        r[vo + oo[g]] = rr;
        dout[vo + oo[g]] = T(cc.rho) * dd[g] + T(cc.sig) * dv[g] * rr;
      }
    } else {                               // y = Dinv S x  (power iteration)
      T Sx[NG];
      pdg_cell<T, DIM>(I, din + vo, dqi, ce, cm, Sx);
#pragma unroll
      for (int g = 0; g < NG; ++g) dout[vo + oo[g]] = dinv[dof + oo[g]] * Sx[g];
    }
  }
}

template <int DIM>
__global__ __launch_bounds__(256) void pdg_diag_kernel(const InstDev* __restrict__ insts, const PDgSeg* __restrict__ segs,
                                const double* __restrict__ dqinv, double* __restrict__ dinv) {
  const PDgSeg sg = segs[blockIdx.y];
  const InstDev& I = insts[sg.inst];
  const int j = blockIdx.z;
  const long long np = (long long)I.sp[0] * I.sp[1] * I.sp[2];
  for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < np; o += (long long)gridDim.x * blockDim.x) {
    double Sx, dg;
    // only the diagonal is used; the value operand is any readable array of the instance
    pdg_eval<double, DIM>(I, dqinv + sg.dqoff, dqinv + sg.dqoff, o, sg.cm[j], Sx, dg);
    dinv[sg.doff + j * sg.djstride + o] = 1.0 / dg;
  }
}

template <typename T, int D>
static void launch_pdg_dim(dim3 g, int mode, hipStream_t s, const PDgSeg* segs, ChebCoef cc, const T* dqinv,
                           const T* dinv, const T* b, T* x, T* r, const T* din, T* dout) {
  switch (mode) {
    case kResInitZero:
      hipLaunchKernelGGL((pdg_kernel<T, D, kResInitZero>), g, dim3(kBlk), 0, s, segs, cc, dqinv, dinv, b, x, r, din,
                         dout);
      break;
    case kResInit:
      hipLaunchKernelGGL((pdg_kernel<T, D, kResInit>), g, dim3(kBlk), 0, s, segs, cc, dqinv, dinv, b, x, r, din, dout);
      break;
    case kStep:
      hipLaunchKernelGGL((pdg_kernel<T, D, kStep>), g, dim3(kBlk), 0, s, segs, cc, dqinv, dinv, b, x, r, din, dout);
      break;
    default:
      hipLaunchKernelGGL((pdg_kernel<T, D, kApplyDinv>), g, dim3(kBlk), 0, s, segs, cc, dqinv, dinv, b, x, r, din,
                         dout);
      break;
  }
}

template <typename T>
void launch_pdg(int dim, const InstDev* insts, const PDgSeg* segs, int nseg, int nj, long long maxnp, int mode,
                ChebCoef cc, const T* dqinv, const T* dinv, const T* b, T* x, T* r, const T* din, T* dout,
                hipStream_t s) {
  (void)insts;   // the segments carry a copy of their instance descriptor
  const long long maxc = maxnp >> dim;      // one thread per cell
  const dim3 g = grid3(maxc, nseg, nj);
  if (dim == 2) launch_pdg_dim<T, 2>(g, mode, s, segs, cc, dqinv, dinv, b, x, r, din, dout);
  else launch_pdg_dim<T, 3>(g, mode, s, segs, cc, dqinv, dinv, b, x, r, din, dout);
}
template void launch_pdg<double>(int, const InstDev*, const PDgSeg*, int, int, long long, int, ChebCoef,
                                 const double*, const double*, const double*, double*, double*, const double*,
                                 double*, hipStream_t);
template void launch_pdg<float>(int, const InstDev*, const PDgSeg*, int, int, long long, int, ChebCoef, const float*,
                                const float*, const float*, float*, float*, const float*, float*, hipStream_t);
void launch_pdg_diag(int dim, const InstDev* insts, const PDgSeg* segs, int nseg, int nj, long long maxnp,
                     const double* dqinv, double* dinv, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL(pdg_diag_kernel<2>, grid3(maxnp, nseg, nj), dim3(kBlk), 0, s, insts, segs, dqinv, dinv);
  else
    hipLaunchKernelGGL(pdg_diag_kernel<3>, grid3(maxnp, nseg, nj), dim3(kBlk), 0, s, insts, segs, dqinv, dinv);
}

// ---- cell levels ------------------------------------------------------------------------
// Loads at clamped in-range indices, masked afterwards (a missing neighbour
// contributes a zero transmissibility), so no load sits behind a branch.
template <typename T>
__device__ __forceinline__ void pcell_eval(const PCellSeg& sg, const T* __restrict__ coef, const T* __restrict__ x,
                                           int c, T cm, T& Sx, T& diag) {
  const long long nc = sg.ncells;
  int ce[3];
  unrank((unsigned)c, sg.n, ce);
  const T* C = coef + sg.coff;
  const long long str[3] = {1, (long long)sg.n[0], (long long)sg.n[0] * sg.n[1]};
  T tl[3], th[3], xl[3], xh[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    const bool lo = e < sg.dim && ce[e] > 0, hi = e < sg.dim && ce[e] + 1 < sg.n[e];
    const long long cl = lo ? c - str[e] : c, ch = hi ? c + str[e] : c;
    const T* t = C + e * nc;
    const T a = t[c], bq = t[ch], xa = x[cl], xb = x[ch];
    tl[e] = lo ? a : T(0);
    th[e] = hi ? bq : T(0);
    xl[e] = xa;
    xh[e] = xb;
  }
  const T xc = x[c];
  T dg = cm * C[4 * nc + c] + C[3 * nc + c];
  T s = dg * xc;
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    dg += tl[e];
    s += tl[e] * (xc - xl[e]);
    dg += th[e];
    s += th[e] * (xc - xh[e]);
  }
  Sx = s;
  diag = dg;
}

template <typename T, int MODE>
__global__ __launch_bounds__(256) void pcell_kernel(const PCellSeg* __restrict__ segs, ChebCoef cc, const T* __restrict__ coef,
                             const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x,
                             T* __restrict__ r, const T* __restrict__ din, T* __restrict__ dout) {
  const PCellSeg sg = segs[blockIdx.y];
  const int j = blockIdx.z;
  const long long vo = sg.voff + j * sg.vjstride;
  const long long dof = sg.doff + j * sg.djstride;
  const T cm = T(sg.cm[j]);
  const int ncl = (int)sg.ncells;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncl; c += gridDim.x * blockDim.x) {
    const T di = dinv[dof + c];
    // every load of a mode precedes its stores
    if constexpr (MODE == kResInitZero) {
      const T rr = T(cc.bsign) * b[vo + c];
      x[vo + c] = 0;
      r[vo + c] = rr;
      dout[vo + c] = T(cc.s0) * di * rr;
    } else if constexpr (MODE == kResInit) {
      const T bb = b[vo + c];
      T Sx, dg;
      pcell_eval<T>(sg, coef, x + vo, c, cm, Sx, dg);
      const T rr = T(cc.bsign) * bb - Sx;
      r[vo + c] = rr;
      dout[vo + c] = T(cc.s0) * di * rr;
    } else if constexpr (MODE == kStep) {
      const T dd = din[vo + c], xv = x[vo + c], rv = r[vo + c];
      T Sd, dg;
      pcell_eval<T>(sg, coef, din + vo, c, cm, Sd, dg);
      x[vo + c] = xv + dd;
      const T rr = rv - Sd;
      r[vo + c] = rr;
      dout[vo + c] = T(cc.rho) * dd + T(cc.sig) * di * rr;
    } else {
      T Sx, dg;
      pcell_eval<T>(sg, coef, din + vo, c, cm, Sx, dg);
      dout[vo + c] = di * Sx;
    }
  }
}
__global__ __launch_bounds__(256) void pcell_diag_kernel(const PCellSeg* __restrict__ segs, const double* __restrict__ coef,
                                  double* __restrict__ dinv) {
  const PCellSeg sg = segs[blockIdx.y];
  const int j = blockIdx.z;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < sg.ncells;
       c += (long long)gridDim.x * blockDim.x) {
    double Sx, dg;
    pcell_eval<double>(sg, coef, coef + sg.coff, c, sg.cm[j], Sx, dg);
    dinv[sg.doff + j * sg.djstride + c] = 1.0 / dg;
  }
}
template <typename T>
void launch_pcell(const PCellSeg* segs, int nseg, int nj, long long maxc, int mode, ChebCoef cc, const T* coef,
                  const T* dinv, const T* b, T* x, T* r, const T* din, T* dout, hipStream_t s) {
  const dim3 g = grid3(maxc, nseg, nj);
  switch (mode) {
    case kResInitZero:
      hipLaunchKernelGGL((pcell_kernel<T, kResInitZero>), g, dim3(kBlk), 0, s, segs, cc, coef, dinv, b, x, r, din,
                         dout);
      break;
    case kResInit:
      hipLaunchKernelGGL((pcell_kernel<T, kResInit>), g, dim3(kBlk), 0, s, segs, cc, coef, dinv, b, x, r, din, dout);
      break;
    case kStep:
      hipLaunchKernelGGL((pcell_kernel<T, kStep>), g, dim3(kBlk), 0, s, segs, cc, coef, dinv, b, x, r, din, dout);
      break;
    default:
      hipLaunchKernelGGL((pcell_kernel<T, kApplyDinv>), g, dim3(kBlk), 0, s, segs, cc, coef, dinv, b, x, r, din, dout);
      break;
  }
}
template void launch_pcell<double>(const PCellSeg*, int, int, long long, int, ChebCoef, const double*, const double*,
                                   const double*, double*, double*, const double*, double*, hipStream_t);
template void launch_pcell<float>(const PCellSeg*, int, int, long long, int, ChebCoef, const float*, const float*,
                                  const float*, float*, float*, const float*, float*, hipStream_t);
void launch_pcell_diag(const PCellSeg* segs, int nseg, int nj, long long maxc, const double* coef, double* dinv,
                       hipStream_t s) {
  hipLaunchKernelGGL(pcell_diag_kernel, grid3(maxc, nseg, nj), dim3(kBlk), 0, s, segs, coef, dinv);
}

// ---- Galerkin coefficients ----------------------------------------------------------------
__global__ __launch_bounds__(256) void pcoef_first_kernel(const InstDev* __restrict__ insts, const PDgSeg* __restrict__ fine,
                                   const PCellSeg* __restrict__ lev1, const double* __restrict__ dqinv,
                                   double* __restrict__ coef) {
  const PDgSeg fs = fine[blockIdx.y];
  const PCellSeg cs = lev1[blockIdx.y];
  const InstDev& I = insts[fs.inst];
  const double* dqi = dqinv + fs.dqoff;
  const int d = I.dim;
  const long long nc = cs.ncells;
  double* C = coef + cs.coff;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += (long long)gridDim.x * blockDim.x) {
    const int ce[3] = {(int)(c % I.n[0]), (int)((c / I.n[0]) % I.n[1]),
                       d == 3 ? (int)(c / ((long long)I.n[0] * I.n[1])) : 0};
    double vol = 1.0;
    for (int e = 0; e < d; ++e) vol *= I.h[e];
    C[4 * nc + c] = vol;
    double ttop = 0.0;
    for (int e = 0; e < 3; ++e) {
      if (e >= d) { C[e * nc + c] = 0.0; continue; }
      double hp = 1.0;
      for (int f = 0; f < d; ++f)
        if (f != e) hp *= 0.5 * I.h[f];
      // flux nodes of the low face (m = 2 ce) and, for the top axis, the top face
      for (int side = 0; side < 2; ++side) {
        if (side == 0 && ce[e] == 0) { C[e * nc + c] = 0.0; continue; }
        if (side == 1 && !(e == d - 1 && ce[e] == I.n[e] - 1)) continue;
        const int m = side == 0 ? 2 * ce[e] : 2 * I.n[e];
        double sum = 0.0;
        const int nf = d == 3 ? 4 : 2;
        for (int fi = 0; fi < nf; ++fi) {
          long long idx = 0, s = 1;
          int bit = 0;
          for (int f = 0; f < d; ++f) {
            int coord;
            if (f == e) coord = m;
            else { coord = 2 * ce[f] + ((fi >> bit) & 1); ++bit; }
            idx += (long long)coord * s;
            s *= I.sq[e][f];
          }
          sum += dqi[I.off_q[e] + idx];
        }
        const double t = I.tau * hp * hp * sum;
        if (side == 0) C[e * nc + c] = t;
        else ttop += t;
      }
    }
    C[3 * nc + c] = ttop;
  }
}
void launch_pcoef_first(const InstDev* insts, const PDgSeg* fine, const PCellSeg* lev1, int nseg, long long maxc,
                        const double* dqinv, double* coef, hipStream_t s) {
  hipLaunchKernelGGL(pcoef_first_kernel, grid3(maxc, nseg, 1), dim3(kBlk), 0, s, insts, fine, lev1, dqinv, coef);
}

__global__ __launch_bounds__(256) void pcoef_coarsen_kernel(const PCellSeg* __restrict__ fine, const PCellSeg* __restrict__ coarse,
                                     const double* __restrict__ coef_f, double* __restrict__ coef_c) {
  const PCellSeg fs = fine[blockIdx.y];
  const PCellSeg cs = coarse[blockIdx.y];
  const long long ncf = fs.ncells, ncc = cs.ncells;
  const double* F = coef_f + fs.coff;
  double* Cc = coef_c + cs.coff;
  const int d = cs.dim;
  for (long long C = (long long)blockIdx.x * blockDim.x + threadIdx.x; C < ncc; C += (long long)gridDim.x * blockDim.x) {
    const int Ce[3] = {(int)(C % cs.n[0]), (int)((C / cs.n[0]) % cs.n[1]),
                       d == 3 ? (int)(C / ((long long)cs.n[0] * cs.n[1])) : 0};
    double t[3] = {0, 0, 0}, ttop = 0, m = 0;
    const int nz = d == 3 ? 2 : 1;
    for (int dz = 0; dz < nz; ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int cc3[3] = {2 * Ce[0] + dx, 2 * Ce[1] + dy, 2 * Ce[2] + dz};
          if (cc3[0] >= fs.n[0] || cc3[1] >= fs.n[1] || (d == 3 && cc3[2] >= fs.n[2])) continue;
          const long long c = cc3[0] + (long long)fs.n[0] * (cc3[1] + (long long)fs.n[1] * (d == 3 ? cc3[2] : 0));
          const int off[3] = {dx, dy, dz};
          for (int e = 0; e < d; ++e)
            if (off[e] == 0) t[e] += F[e * ncf + c];
          ttop += F[3 * ncf + c];
          m += F[4 * ncf + c];
        }
    for (int e = 0; e < 3; ++e) Cc[e * ncc + C] = (e < d && Ce[e] > 0) ? t[e] : 0.0;
    Cc[3 * ncc + C] = ttop;
    Cc[4 * ncc + C] = m;
  }
}
void launch_pcoef_coarsen(const PCellSeg* fine, const PCellSeg* coarse, int nseg, long long maxc, const double* coef_f,
                          double* coef_c, hipStream_t s) {
  hipLaunchKernelGGL(pcoef_coarsen_kernel, grid3(maxc, nseg, 1), dim3(kBlk), 0, s, fine, coarse, coef_f, coef_c);
}

// ---- transfers ------------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void p_restrict_dg_kernel(const InstDev* __restrict__ insts, const PDgSeg* __restrict__ fine,
                                     const PCellSeg* __restrict__ coarse, const T* __restrict__ r,
                                     T* __restrict__ b) {
  const PDgSeg& fs = fine[blockIdx.y];
  const PCellSeg cs = coarse[blockIdx.y];
  const InstDev& I = fs.I;
  const int j = blockIdx.z;
  const T* R = r + fs.voff + j * fs.vjstride;
  T* Bc = b + cs.voff + j * cs.vjstride;
  const int d = I.dim;
  const int ncl = (int)cs.ncells;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncl; c += gridDim.x * blockDim.x) {
    int ce3[3];
    unrank((unsigned)c, I.n, ce3);
    const int i = ce3[0], jy = ce3[1], k = ce3[2];
    T s = 0;
    for (int g = 0; g < (d == 3 ? 8 : 4); ++g) {
      const long long o = (2 * i + (g & 1)) + (long long)I.sp[0] * ((2 * jy + ((g >> 1) & 1)) +
                                                                    (long long)I.sp[1] * (d == 3 ? 2 * k + (g >> 2) : 0));
      s += R[o];
    }
    Bc[c] = s;
  }
}
template <typename T>
__global__ __launch_bounds__(256) void p_prolong_dg_kernel(const InstDev* __restrict__ insts, const PDgSeg* __restrict__ fine,
                                    const PCellSeg* __restrict__ coarse, double w, const T* __restrict__ e,
                                    T* __restrict__ x) {
  const PDgSeg& fs = fine[blockIdx.y];
  const PCellSeg cs = coarse[blockIdx.y];
  const InstDev& I = fs.I;
  const int j = blockIdx.z;
  const long long np = (long long)I.sp[0] * I.sp[1] * I.sp[2];
  T* X = x + fs.voff + j * fs.vjstride;
  const T* Ec = e + cs.voff + j * cs.vjstride;
  const int npi = (int)np;
  for (int o = blockIdx.x * blockDim.x + threadIdx.x; o < npi; o += gridDim.x * blockDim.x) {
    int oc[3];
    unrank((unsigned)o, I.sp, oc);
    const int ox = oc[0], oy = oc[1], oz = oc[2];
    const long long c = (ox >> 1) + (long long)I.n[0] * ((oy >> 1) + (long long)I.n[1] * (oz >> 1));
    X[o] += T(w) * Ec[c];
  }
}
template <typename T>
__global__ __launch_bounds__(256) void p_restrict_cell_kernel(const PCellSeg* __restrict__ fine, const PCellSeg* __restrict__ coarse,
                                       const T* __restrict__ r, T* __restrict__ b) {
  const PCellSeg fs = fine[blockIdx.y];
  const PCellSeg cs = coarse[blockIdx.y];
  const int j = blockIdx.z;
  const T* R = r + fs.voff + j * fs.vjstride;
  T* Bc = b + cs.voff + j * cs.vjstride;
  const int d = cs.dim;
  const int ncc = (int)cs.ncells;
  for (int C = blockIdx.x * blockDim.x + threadIdx.x; C < ncc; C += gridDim.x * blockDim.x) {
    int Ce[3];
    unrank((unsigned)C, cs.n, Ce);
    T s = 0;
    for (int dz = 0; dz < (d == 3 ? 2 : 1); ++dz)
      for (int dy = 0; dy < 2; ++dy)
        for (int dx = 0; dx < 2; ++dx) {
          const int a = 2 * Ce[0] + dx, bb = 2 * Ce[1] + dy, cz = 2 * Ce[2] + dz;
          if (a >= fs.n[0] || bb >= fs.n[1] || (d == 3 && cz >= fs.n[2])) continue;
          s += R[a + (long long)fs.n[0] * (bb + (long long)fs.n[1] * (d == 3 ? cz : 0))];
        }
    Bc[C] = s;
  }
}
template <typename T>
__global__ __launch_bounds__(256) void p_prolong_cell_kernel(const PCellSeg* __restrict__ fine, const PCellSeg* __restrict__ coarse, double w,
                                      const T* __restrict__ e, T* __restrict__ x) {
  const PCellSeg fs = fine[blockIdx.y];
  const PCellSeg cs = coarse[blockIdx.y];
  const int j = blockIdx.z;
  T* X = x + fs.voff + j * fs.vjstride;
  const T* Ec = e + cs.voff + j * cs.vjstride;
  const int ncf = (int)fs.ncells;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncf; c += gridDim.x * blockDim.x) {
    int ce3[3];
    unrank((unsigned)c, fs.n, ce3);
    const int i = ce3[0], jy = ce3[1], k = ce3[2];
    X[c] += T(w) * Ec[(i >> 1) + (long long)cs.n[0] * ((jy >> 1) + (long long)cs.n[1] * (k >> 1))];
  }
}
template <typename T>
void launch_p_restrict_dg(const InstDev* insts, const PDgSeg* fine, const PCellSeg* coarse, int nseg, int nj,
                          long long maxc, const T* r, T* b, hipStream_t s) {
  hipLaunchKernelGGL((p_restrict_dg_kernel<T>), grid3(maxc, nseg, nj), dim3(kBlk), 0, s, insts, fine, coarse, r, b);
}
template <typename T>
void launch_p_prolong_dg(const InstDev* insts, const PDgSeg* fine, const PCellSeg* coarse, int nseg, int nj,
                         long long maxnp, double w, const T* e, T* x, hipStream_t s) {
  hipLaunchKernelGGL((p_prolong_dg_kernel<T>), grid3(maxnp, nseg, nj), dim3(kBlk), 0, s, insts, fine, coarse, w, e, x);
}
template <typename T>
void launch_p_restrict_cell(const PCellSeg* fine, const PCellSeg* coarse, int nseg, int nj, long long maxc,
                            const T* r, T* b, hipStream_t s) {
  hipLaunchKernelGGL((p_restrict_cell_kernel<T>), grid3(maxc, nseg, nj), dim3(kBlk), 0, s, fine, coarse, r, b);
}
template <typename T>
void launch_p_prolong_cell(const PCellSeg* fine, const PCellSeg* coarse, int nseg, int nj, long long maxc, double w,
                           const T* e, T* x, hipStream_t s) {
  hipLaunchKernelGGL((p_prolong_cell_kernel<T>), grid3(maxc, nseg, nj), dim3(kBlk), 0, s, fine, coarse, w, e, x);
}
#define BT_INST_P(T)                                                                                                 \
  template void launch_p_restrict_dg<T>(const InstDev*, const PDgSeg*, const PCellSeg*, int, int, long long, const T*, \
                                        T*, hipStream_t);                                                            \
  template void launch_p_prolong_dg<T>(const InstDev*, const PDgSeg*, const PCellSeg*, int, int, long long, double,    \
                                       const T*, T*, hipStream_t);                                                   \
  template void launch_p_restrict_cell<T>(const PCellSeg*, const PCellSeg*, int, int, long long, const T*, T*,          \
                                          hipStream_t);                                                              \
  template void launch_p_prolong_cell<T>(const PCellSeg*, const PCellSeg*, int, int, long long, double, const T*, T*,   \
                                         hipStream_t);
BT_INST_P(double)
BT_INST_P(float)

// ---- Dq^-1 ---------------------------------------------------------------------------------
// Dq(q_e node) = sum over the cells sharing the node along e of eta/K_c h_e MC(a,a) prod_{f!=e} h_f/2
__global__ __launch_bounds__(256) void dq_kernel(const InstDev* __restrict__ insts, const double* __restrict__ kinv, double* __restrict__ dqinv) {
  const InstDev& I = insts[blockIdx.y];
  const int d = I.dim;
  double* out = dqinv + I.state_off;
  const double* kc = kinv + I.cell_off;
  const long long qend = I.off_p;
  for (long long t = I.off_q[0] + (long long)blockIdx.x * blockDim.x + threadIdx.x; t < qend;
       t += (long long)gridDim.x * blockDim.x) {
    int e = 0;
    for (int c = 1; c < d; ++c)
      if (t >= I.off_q[c]) e = c;
    long long rem = t - I.off_q[e];
    int co[3] = {0, 0, 0};
    for (int f = 0; f < d; ++f) { co[f] = rem % I.sq[e][f]; rem /= I.sq[e][f]; }
    const int m = co[e];
    if (q_fixed(I, e, m)) { out[t] = 0.0; continue; }
    double hp = 1.0;
    for (int f = 0; f < d; ++f)
      if (f != e) hp *= 0.5 * I.h[f];
    int cc[3];
    for (int f = 0; f < d; ++f) cc[f] = co[f] >> 1;
    double dsum = 0.0;
    for (int side = 0; side < 2; ++side) {
      int ce, a;
      if (m & 1) { if (side) break; ce = (m - 1) / 2; a = 1; }
      else { ce = m / 2 - 1 + side; a = side ? 0 : 2; if (ce < 0 || ce >= I.n[e]) continue; }
      cc[e] = ce;
      const long long cell = cc[0] + (long long)I.n[0] * (cc[1] + (long long)I.n[1] * (d == 3 ? cc[2] : 0));
      dsum += kc[cell] * I.h[e] * MC(a, a) * hp;
    }
    out[t] = 1.0 / dsum;
  }
}
void launch_dq(const InstDev* insts, int count, long long maxN, const double* kinv, double* dqinv, hipStream_t s) {
  hipLaunchKernelGGL(dq_kernel, grid3(maxN, count, 1), dim3(kBlk), 0, s, insts, kinv, dqinv);
}

}  // namespace bt
