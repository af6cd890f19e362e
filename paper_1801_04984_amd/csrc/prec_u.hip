// Geometric multigrid for the Q2 elasticity block tau A of the fixed-stress
// mechanics step (u = (tau A)^-1 (r_u + b tau E p)).
//
// Levels are uniform boxes n -> ceil(n/2) per axis; the coarse operator is
// the same bilinear form rediscretised (for even n the spaces are nested and
// this equals the Galerkin product).  Prolongation evaluates the coarse Q2
// function at the fine nodes (tensor product of 1D interpolation tables, valid
// for non-nested meshes too); restriction is its transpose, applied as one
// 1D pass per axis.  Essential rows are identity on every level; all level
// vectors are kept zero there.
#include "common.h"
#include "prec.h"
#include "rows.h"

namespace bt {

// tile variants of the 2D operator: 16x16 threads (15x15 owned cells) or
// 8x8 (7x7); the small tile spreads small levels over more compute units
int uapply_tile(int dim, int variant) { return dim == 2 ? (variant == 1 ? 7 : 15) : -1; }

// y = tau A x (mode 0) or y = b - tau A x (mode 1); essential rows: y = 0 (mode 0), y = b (mode 1).
// One block = UT x UT cells ((UT-1)^2 owned + low-side halo); each owned cell sums
// its lower-left 2x2 nodes (and the top/right boundary nodes of the last
// cells) from the element rows of the cells sharing them, staged in LDS.
// Every global load of a thread (the cell's x values and, for mode 1, its b
// values) is issued before the first use, at clamped in-range indices.
template <typename T, int UT>
__global__ __launch_bounds__(UT * UT) void uapply2d_kernel(const UGridSeg* __restrict__ segs,
                                                           const int4* __restrict__ work, int mode,
                                                           const T* __restrict__ X, const T* __restrict__ Bv,
                                                           T* __restrict__ Y, const T* __restrict__ emat) {
  constexpr int UO = UT - 1;
  __shared__ T E[18][UT * UT];
  const int4 w = work[blockIdx.x];
  const UGridSeg& G = segs[w.x];
  const int j = blockIdx.y;
  const long long vo = G.voff + j * G.vjstride;
  const T* Xl = X + vo;
  const T* Bl = Bv + vo;
  T* Yl = Y + vo;
  const int lx = threadIdx.x, ly = threadIdx.y, tid = ly * UT + lx;
  const int nx = G.n[0], ny = G.n[1];
  const int i = w.y * UO - 1 + lx, jc = w.z * UO - 1 + ly;
  const bool valid = (i >= 0) && (i < nx) && (jc >= 0) && (jc < ny);
  const bool owned = valid && lx >= 1 && ly >= 1;
  const bool lastx = i == nx - 1, lasty = jc == ny - 1;
  const int sux = G.su[0];
  const int nu1 = G.su[0] * G.su[1];
  const int ub = valid ? 2 * i + sux * (2 * jc) : 0;
  T uu[18], bv[18] = {};
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int o = ub + a + sux * b;
      uu[b * 3 + a] = Xl[o];
      uu[9 + b * 3 + a] = Xl[nu1 + o];
    }
  if (mode == 1 && owned) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int o = ub + a + sux * b;
        bv[b * 3 + a] = Bl[o];
        bv[9 + b * 3 + a] = Bl[nu1 + o];
      }
  }
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const bool bot = b == 0 && jc == 0;
      const bool fx = bot || (a == 0 && i == 0) || (a == 2 && lastx);
      if (!valid || fx) uu[b * 3 + a] = T(0);
      if (!valid || bot) uu[9 + b * 3 + a] = T(0);
    }
  {
    const T* AE = emat + G.emat_off;   // tau A_e of this level (18x18)
    // one row per iteration (scalar loads; unrolling all rows would spill the scalar registers)
#pragma unroll 1
    for (int rr = 0; rr < 18; ++rr) {
      T acc = 0;
#pragma unroll
      for (int cc = 0; cc < 18; ++cc) acc += AE[rr * 18 + cc] * uu[cc];
      E[rr][tid] = acc;
    }
  }
  __syncthreads();
  if (!owned) return;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if ((a == 2 && !lastx) || (b == 2 && !lasty)) continue;
        const int mx = 2 * i + a, my = 2 * jc + b;
        const int go = c * nu1 + ub + a + sux * b;
        const bool fixed = my == 0 || (c == 0 && (mx == 0 || mx == 2 * nx));
        T v = 0;
        if (!fixed) {
#pragma unroll
          for (int sy = 0; sy < 2; ++sy) {
            if (b != 0 && sy == 0) continue;
            const int lb = b != 0 ? b : (sy == 0 ? 2 : 0);
            const int dy = (b == 0 && sy == 0) ? -UT : 0;
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
              if (a != 0 && sx == 0) continue;
              const int la = a != 0 ? a : (sx == 0 ? 2 : 0);
              const int dx = (a == 0 && sx == 0) ? -1 : 0;
              v += E[c * 9 + lb * 3 + la][tid + dy + dx];
            }
          }
        }
        Yl[go] = mode == 0 ? v : bv[c * 9 + b * 3 + a] - v;
      }
}

template <typename T>
void launch_uapply(int dim, const UGridSeg* segs, const int4* work, int nwork, int nj, int mode, const T* x,
                   const T* b, T* y, const T* emat, hipStream_t s, int variant) {
  if (dim == 2) {
    if (variant == 1)
      hipLaunchKernelGGL((uapply2d_kernel<T, 8>), dim3(nwork, nj), dim3(8, 8), 0, s, segs, work, mode, x, b, y, emat);
    else
      hipLaunchKernelGGL((uapply2d_kernel<T, 16>), dim3(nwork, nj), dim3(16, 16), 0, s, segs, work, mode, x, b, y,
                         emat);
  } else {
    launch_uapply3d<T>(segs, work, nwork, nj, variant, mode, x, b, y, emat, s);
  }
}
template void launch_uapply<double>(int, const UGridSeg*, const int4*, int, int, int, const double*, const double*,
                                    double*, const double*, hipStream_t, int);
template void launch_uapply<float>(int, const UGridSeg*, const int4*, int, int, int, const float*, const float*,
                                   float*, const float*, hipStream_t, int);

// ---- restriction pass ------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void rpass_kernel(const RPass* __restrict__ segs, const double* __restrict__ tab, const T* __restrict__ in,
                             T* __restrict__ out) {
  const RPass P = segs[blockIdx.y];
  const int j = blockIdx.z;
  const long long ni = (long long)P.din[0] * P.din[1] * P.din[2];
  const long long no = (long long)P.dout[0] * P.dout[1] * P.dout[2];
  const T* I = in + P.ioff + j * P.ijstride;
  T* O = out + P.ooff + j * P.ojstride;
  const long long istr[3] = {1, (long long)P.din[0], (long long)P.din[0] * P.din[1]};
  const int nout = (int)(no * P.dim), no32 = (int)no;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nout; t += gridDim.x * blockDim.x) {
    const int c = t >= no32 ? (t >= 2 * no32 ? 2 : 1) : 0;
    int co[3];
    unrank((unsigned)(t - c * no32), P.dout, co);
    if (P.last && ugrid_fixed(P.dim, P.dout, c, co[0], co[1], co[2])) { O[t] = T(0); continue; }
    long long base = c * ni;
    for (int f = 0; f < 3; ++f)
      if (f != P.axis) base += co[f] * istr[f];
    const double* tr = tab + P.tab + (long long)co[P.axis] * 2 * P.width;
    double s = 0.0;
    for (int k = 0; k < P.width; ++k) {
      const double wgt = tr[2 * k + 1];
      if (wgt == 0.0) continue;
      s += wgt * (double)I[base + (long long)tr[2 * k] * istr[P.axis]];
    }
    O[t] = (T)s;
  }
}
template <typename T>
void launch_rpass(const RPass* segs, int nseg, int nj, long long maxout, const double* tab, const T* in, T* out,
                  hipStream_t s) {
  long long b = (maxout + kBlk - 1) / kBlk;
  hipLaunchKernelGGL((rpass_kernel<T>), dim3((unsigned)(b > 65535 ? 65535 : (b < 1 ? 1 : b)), nseg, nj), dim3(kBlk), 0,
                     s, segs, tab, in, out);
}
template void launch_rpass<double>(const RPass*, int, int, long long, const double*, const double*, double*,
                                   hipStream_t);
template void launch_rpass<float>(const RPass*, int, int, long long, const double*, const float*, float*,
                                  hipStream_t);

// ---- prolongation: x_fine += P e_coarse ---------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void uprolong_kernel(const UProl* __restrict__ segs, const double* __restrict__ tab,
                                const T* __restrict__ e, T* __restrict__ x) {
  const UProl P = segs[blockIdx.y];
  const int j = blockIdx.z;
  const long long nf = (long long)P.sf[0] * P.sf[1] * P.sf[2];
  const long long nc = (long long)P.sc[0] * P.sc[1] * P.sc[2];
  const T* Ec = e + P.coff + j * P.cjstride;
  T* Xf = x + P.foff + j * P.fjstride;
  const int nft = (int)(nf * P.dim), nf32 = (int)nf;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nft; t += gridDim.x * blockDim.x) {
    const int c = t >= nf32 ? (t >= 2 * nf32 ? 2 : 1) : 0;
    int m[3];
    unrank((unsigned)(t - c * nf32), P.sf, m);
    if (ugrid_fixed(P.dim, P.sf, c, m[0], m[1], m[2])) continue;
    const double* tx = tab + P.tab[0] + 4LL * m[0];
    const double* ty = tab + P.tab[1] + 4LL * m[1];
    const int Cx = (int)tx[0], Cy = (int)ty[0];
    double s = 0.0;
    if (P.dim == 2) {
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a)
          s += tx[1 + a] * ty[1 + b] * (double)Ec[c * nc + (2 * Cx + a) + (long long)P.sc[0] * (2 * Cy + b)];
    } else {
      const double* tz = tab + P.tab[2] + 4LL * m[2];
      const int Cz = (int)tz[0];
      for (int cz = 0; cz < 3; ++cz)
        for (int b = 0; b < 3; ++b)
          for (int a = 0; a < 3; ++a)
            s += tx[1 + a] * ty[1 + b] * tz[1 + cz] *
                 (double)Ec[c * nc + (2 * Cx + a) + (long long)P.sc[0] * ((2 * Cy + b) + (long long)P.sc[1] * (2 * Cz + cz))];
    }
    Xf[t] += (T)s;
  }
}
template <typename T>
void launch_uprolong(const UProl* segs, int nseg, int nj, long long maxfine, const double* tab, const T* e, T* x,
                     hipStream_t s) {
  long long b = (maxfine + kBlk - 1) / kBlk;
  hipLaunchKernelGGL((uprolong_kernel<T>), dim3((unsigned)(b > 65535 ? 65535 : (b < 1 ? 1 : b)), nseg, nj), dim3(kBlk),
                     0, s, segs, tab, e, x);
}
template void launch_uprolong<double>(const UProl*, int, int, long long, const double*, const double*, double*,
                                      hipStream_t);
template void launch_uprolong<float>(const UProl*, int, int, long long, const double*, const float*, float*,
                                     hipStream_t);

// ---- y = Dinv x on level segments -------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void muldinv_kernel(const LSeg* __restrict__ segs, const T* __restrict__ dinv, const T* __restrict__ x,
                               T* __restrict__ y) {
  const LSeg sg = segs[blockIdx.y];
  const long long off = sg.off + blockIdx.z * sg.jstride, doff = sg.doff + blockIdx.z * sg.djstride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x)
    y[off + i] = dinv[doff + i] * x[off + i];
}
template <typename T>
void launch_mul_dinv(const LSeg* segs, int nseg, int nj, long long maxlen, const T* dinv, const T* x, T* y,
                     hipStream_t s) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  hipLaunchKernelGGL((muldinv_kernel<T>), dim3((unsigned)(b > 65535 ? 65535 : (b < 1 ? 1 : b)), nseg, nj), dim3(kBlk), 0,
                     s, segs, dinv, x, y);
}
template void launch_mul_dinv<double>(const LSeg*, int, int, long long, const double*, const double*, double*,
                                      hipStream_t);
template void launch_mul_dinv<float>(const LSeg*, int, int, long long, const float*, const float*, float*,
                                     hipStream_t);

}  // namespace bt
