// 3D space-time slab operator Y = A X (or A^T X) and the 3D Q2 elasticity
// operator of the multigrid levels.
//
// u-rows (tau A u - c_p E p, section "Poroelasticity"): one block = an xy
// tile of 8x8 cells (7x7 owned plus a one-cell halo on the low sides) that
// marches through a z-chunk of cell layers.  Each thread evaluates the element
// vector of its cell by sum factorisation through the 3x3x3 Gauss points, one
// z-slice of points at a time (registers stay bounded), and stages it in LDS.
// Node planes are completed layer by layer: plane 2k gets the top slice of
// layer k-1 (carried in LDS) plus the bottom slice of layer k, plane 2k+1 the
// middle slice; every owned node is summed in a fixed order (deterministic,
// no atomics).  q-rows and p-rows are gathers (rows.h) in their own kernels:
//   q-rows: tau (Mq q + B p);   p-rows: -w [tau div q_i + sum_j T_ij (b div u_j + p_j/M)]
//   (A^T: p-rows -w [tau div q_i + tau b div u_i + sum_j T_ji p_j / M], u-rows use sum_j T_ji p_j).
#include "kernels.h"
#include "prec.h"
#include "rows.h"

namespace bt {

constexpr int kT3 = 8;
constexpr int kO3 = kT3 - 1;
constexpr int kZC = 8;

int apply3d_tile_cells_xy() { return kO3; }
int apply3d_tile_cells_z() { return kZC; }

template <typename T>
struct U3Job {
  int n[3], su[3];
  T h[3], tau, lam, mu, cp;
  const T* X;        // u block, components at X + c * nu1
  const T* Bv;       // residual mode right-hand side (same layout) or null
  T* Y;
  const T* P;        // pressure block of the coupling (mixed over time levels) or null
  long long plstride;  // distance between the time levels of P
  T pw[4];           // time-level weights of the coupling pressure
  int npl;
  int sp[2];
  int mode;          // 0: Y = A x (+ coupling); 1: Y = B - A x
};

template <typename T>
__device__ __forceinline__ void u3_run(const U3Job<T>& J, int i0, int j0, int k0) {
  __shared__ T E[81][64];
  __shared__ T C[27][64];
  const int tid = threadIdx.x;
  const int lx = tid % kT3, ly = tid / kT3;
  const int nx = J.n[0], ny = J.n[1], nz = J.n[2];
  const int i = i0 - 1 + lx, j = j0 - 1 + ly;
  const bool vxy = i >= 0 && i < nx && j >= 0 && j < ny;
  const long long nu1 = (long long)J.su[0] * J.su[1] * J.su[2];
  const long long sy = J.su[0], sz = (long long)J.su[0] * J.su[1];
  const T ihx = T(1) / J.h[0], ihy = T(1) / J.h[1], ihz = T(1) / J.h[2];
  const T vol = J.h[0] * J.h[1] * J.h[2];
#pragma unroll
  for (int q = 0; q < 27; ++q) C[q][tid] = T(0);
  const int kbeg = k0 > 0 ? k0 - 1 : 0;
  const int kend = min(k0 + kZC, nz);
  // owned xy node ranges
  const int mxe = (i0 + kO3 >= nx) ? 2 * nx + 1 : 2 * i0 + 2 * kO3;
  const int mye = (j0 + kO3 >= ny) ? 2 * ny + 1 : 2 * j0 + 2 * kO3;
  const int nmx = mxe - 2 * i0, nmy = mye - 2 * j0;
  const int nplane = nmx * nmy;

  for (int k = kbeg; k < kend; ++k) {
    // ---- element vector of cell (i, j, k)
#pragma unroll
    for (int q = 0; q < 81; ++q) E[q][tid] = T(0);
    if (vxy) {
      T pc[8];
      if (J.npl > 0) {
#pragma unroll
        for (int g = 0; g < 8; ++g) {
          const long long o = (2 * i + (g & 1)) + (long long)J.sp[0] *
                              ((2 * j + ((g >> 1) & 1)) + (long long)J.sp[1] * (2 * k + (g >> 2)));
          T s = 0;
          for (int l = 0; l < J.npl; ++l) s += J.pw[l] * J.P[l * J.plstride + o];
          pc[g] = s;
        }
      } else {
#pragma unroll
        for (int g = 0; g < 8; ++g) pc[g] = T(0);
      }
#pragma unroll 1
      for (int kz = 0; kz < 3; ++kz) {
        T zv[3][9], zd[3][9];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int ba = 0; ba < 9; ++ba) {
            const int a = ba % 3, b = ba / 3;
            const int mx = 2 * i + a, my = 2 * j + b;
            T v = 0, dv = 0;
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
              const int mz = 2 * k + kk;
              const T u = ugrid_fixed(3, J.su, c, mx, my, mz) ? T(0) : J.X[c * nu1 + mx + sy * my + sz * mz];
              v += T(VQ(kz, kk)) * u;
              dv += T(DQ(kz, kk)) * u;
            }
            zv[c][ba] = v;
            zd[c][ba] = dv;
          }
        T av[3][9], ad[3][9];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int ba = 0; ba < 9; ++ba) { av[c][ba] = 0; ad[c][ba] = 0; }
#pragma unroll
        for (int ky = 0; ky < 3; ++ky)
#pragma unroll
          for (int kx = 0; kx < 3; ++kx) {
            T g[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              T tx = 0, ty = 0, tz = 0;
#pragma unroll
              for (int b = 0; b < 3; ++b) {
                T sd = 0, sv = 0, szv = 0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                  sd += T(DQ(kx, a)) * zv[c][b * 3 + a];
                  sv += T(VQ(kx, a)) * zv[c][b * 3 + a];
                  szv += T(VQ(kx, a)) * zd[c][b * 3 + a];
                }
                tx += T(VQ(ky, b)) * sd;
                ty += T(DQ(ky, b)) * sv;
                tz += T(VQ(ky, b)) * szv;
              }
              g[c][0] = tx * ihx;
              g[c][1] = ty * ihy;
              g[c][2] = tz * ihz;
            }
            T pq = 0;
#pragma unroll
            for (int gg = 0; gg < 8; ++gg)
              pq += T(PQ(kx, gg & 1) * PQ(ky, (gg >> 1) & 1)) * T(PQ(kz, gg >> 2)) * pc[gg];
            const T W = T(wq(kx) * wq(ky)) * T(wq(kz)) * vol;
            const T div = g[0][0] + g[1][1] + g[2][2];
            const T diag = J.tau * J.lam * div - J.cp * pq;
            T S[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
              for (int e = 0; e < 3; ++e) {
                T s = J.tau * J.mu * (g[c][e] + g[e][c]);
                if (c == e) s += diag;
                S[c][e] = W * s * (e == 0 ? ihx : (e == 1 ? ihy : ihz));
              }
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
              for (int b = 0; b < 3; ++b)
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                  av[c][b * 3 + a] += T(VQ(ky, b) * DQ(kx, a)) * S[c][0] + T(DQ(ky, b) * VQ(kx, a)) * S[c][1];
                  ad[c][b * 3 + a] += T(VQ(ky, b) * VQ(kx, a)) * S[c][2];
                }
          }
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int kk = 0; kk < 3; ++kk)
#pragma unroll
            for (int ba = 0; ba < 9; ++ba)
              E[c * 27 + kk * 9 + ba][tid] += T(VQ(kz, kk)) * av[c][ba] + T(DQ(kz, kk)) * ad[c][ba];
      }
    }
    __syncthreads();
    // ---- owned node planes 2k (bottom slice + carried top slice) and 2k+1
    if (k >= k0) {
      for (int idx = tid; idx < 6 * nplane; idx += 64) {
        const int c = idx / (2 * nplane);
        const int rem = idx - c * 2 * nplane;
        const int zl = rem / nplane;                  // 0: plane 2k, 1: plane 2k+1
        const int r2 = rem - zl * nplane;
        const int mx = 2 * i0 + r2 % nmx, my = 2 * j0 + r2 / nmx, mz = 2 * k + zl;
        const long long go = c * nu1 + mx + sy * my + sz * mz;
        T v;
        if (ugrid_fixed(3, J.su, c, mx, my, mz)) {
          v = J.mode == 0 ? J.X[go] : T(0);
        } else {
          const bool xo = mx & 1, yo = my & 1;
          const int cx0 = xo ? (mx - 1) / 2 : mx / 2 - 1, ax0 = xo ? 1 : 2;
          const int cy0 = yo ? (my - 1) / 2 : my / 2 - 1, ay0 = yo ? 1 : 2;
          const bool vx0 = cx0 >= 0, vx1 = !xo && (mx / 2 < nx);
          const bool vy0 = cy0 >= 0, vy1 = !yo && (my / 2 < ny);
          const int tx0 = cx0 - i0 + 1, ty0 = cy0 - j0 + 1;
          v = 0;
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int qx = q & 1, qy = q >> 1;
            if (!((qy ? vy1 : vy0) && (qx ? vx1 : vx0))) continue;
            const int t = (ty0 + qy) * kT3 + tx0 + qx;
            const int a = qx ? 0 : ax0, b = qy ? 0 : ay0;
            v += E[c * 27 + zl * 9 + b * 3 + a][t];
            if (zl == 0) v += C[c * 9 + b * 3 + a][t];
          }
        }
        J.Y[go] = J.mode == 0 ? v : J.Bv[go] - v;
      }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 27; ++q) C[q][tid] = E[(q / 9) * 27 + 18 + q % 9][tid];
  }
  // ---- top plane 2 nz (only the layer below contributes)
  if (kend == nz) {
    __syncthreads();
    for (int idx = tid; idx < 3 * nplane; idx += 64) {
      const int c = idx / nplane;
      const int r2 = idx - c * nplane;
      const int mx = 2 * i0 + r2 % nmx, my = 2 * j0 + r2 / nmx, mz = 2 * nz;
      const long long go = c * nu1 + mx + sy * my + sz * mz;
      T v;
      if (ugrid_fixed(3, J.su, c, mx, my, mz)) {
        v = J.mode == 0 ? J.X[go] : T(0);
      } else {
        const bool xo = mx & 1, yo = my & 1;
        const int cx0 = xo ? (mx - 1) / 2 : mx / 2 - 1, ax0 = xo ? 1 : 2;
        const int cy0 = yo ? (my - 1) / 2 : my / 2 - 1, ay0 = yo ? 1 : 2;
        const bool vx0 = cx0 >= 0, vx1 = !xo && (mx / 2 < nx);
        const bool vy0 = cy0 >= 0, vy1 = !yo && (my / 2 < ny);
        const int tx0 = cx0 - i0 + 1, ty0 = cy0 - j0 + 1;
        v = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int qx = q & 1, qy = q >> 1;
          if (!((qy ? vy1 : vy0) && (qx ? vx1 : vx0))) continue;
          const int t = (ty0 + qy) * kT3 + tx0 + qx;
          const int a = qx ? 0 : ax0, b = qy ? 0 : ay0;
          v += C[c * 9 + b * 3 + a][t];
        }
      }
      J.Y[go] = J.mode == 0 ? v : J.Bv[go] - v;
    }
  }
}

// operator apply: u-rows of time level blockIdx.y
template <typename T, int NL, bool TR>
__global__ __launch_bounds__(64) void apply3d_u_kernel(const InstDev* __restrict__ insts, const int4* __restrict__ work,
                                                       TimeMat tm, const T* __restrict__ X, T* __restrict__ Y) {
  const int4 w = work[blockIdx.x];
  const InstDev& I = insts[w.x];
  const int lev = blockIdx.y;
  U3Job<T> J;
  for (int e = 0; e < 3; ++e) { J.n[e] = I.n[e]; J.su[e] = I.su[e]; J.h[e] = T(I.h[e]); }
  J.tau = T(I.tau); J.lam = T(I.lam); J.mu = T(I.mu);
  J.X = X + I.x_off + lev * I.N + I.off_u[0];
  J.Y = Y + I.x_off + lev * I.N + I.off_u[0];
  J.Bv = nullptr;
  J.mode = 0;
  J.P = X + I.x_off + I.off_p;
  J.plstride = I.N;
  J.npl = NL;
  J.sp[0] = I.sp[0]; J.sp[1] = I.sp[1];
  for (int l = 0; l < 4; ++l) J.pw[l] = T(0);
  if (!TR) {
    for (int l = 0; l < NL; ++l) J.pw[l] = (l == lev) ? T(1) : T(0);
    J.cp = T(I.tau * I.b);
  } else {
    for (int l = 0; l < NL; ++l) J.pw[l] = T(tm.T[l * 4 + lev]);
    J.cp = T(I.b);
  }
  u3_run<T>(J, w.y * kO3, w.z * kO3, w.w * kZC);
}

// q-rows: tau (Mq q + B p), identity on essential rows
template <typename T>
__global__ __launch_bounds__(256) void qrows_kernel(const InstDev* __restrict__ insts, const T* __restrict__ kinv,
                                                    const T* __restrict__ X, T* __restrict__ Y) {
  const InstDev& I = insts[blockIdx.y];
  const int lev = blockIdx.z;
  const T* Xl = X + I.x_off + lev * I.N;
  T* Yl = Y + I.x_off + lev * I.N;
  const T* kc = kinv + I.cell_off;
  for (long long t = I.off_q[0] + (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.off_p;
       t += (long long)gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode_dof(I, t, blk, comp, co);
    if (q_fixed(I, comp, co[comp])) { Yl[t] = Xl[t]; continue; }
    T dg;
    Yl[t] = mq_node<T>(I, kc, Xl, comp, co, dg) + T(I.tau) * bp_node<T>(I, Xl, comp, co);
  }
}

// p-rows of every time level, one thread per cell
template <typename T, int NL, bool TR, int DIM>
__global__ __launch_bounds__(256) void prows_kernel(const InstDev* __restrict__ insts, TimeMat tm,
                                                    const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int NG = 1 << DIM;
  const InstDev& I = insts[blockIdx.y];
  for (long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x; cell < I.ncells;
       cell += (long long)gridDim.x * blockDim.x) {
    const int ce[3] = {(int)(cell % I.n[0]), (int)((cell / I.n[0]) % I.n[1]),
                       DIM == 3 ? (int)(cell / ((long long)I.n[0] * I.n[1])) : 0};
    long long po[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g)
      po[g] = p_index(I, 2 * ce[0] + (g & 1), 2 * ce[1] + ((g >> 1) & 1), DIM == 3 ? 2 * ce[2] + (g >> 2) : 0);
    T w = 1;
#pragma unroll
    for (int e = 0; e < DIM; ++e) w *= T(0.5 * I.h[e]);
    T acc[NL][NG];
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int g = 0; g < NG; ++g) acc[l][g] = 0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const T* Xj = X + I.x_off + j * I.N;
      T du[NG], dq[NG];
      cell_div<T, DIM>(I, Xj, ce, du, dq);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const T pj = Xj[po[g]];
        if (!TR) {
          const T z = T(I.b) * du[g] + T(I.Minv) * pj;
#pragma unroll
          for (int l = 0; l < NL; ++l) acc[l][g] += T(tm.T[l * 4 + j]) * z + ((l == j) ? T(I.tau) * dq[g] : T(0));
        } else {
#pragma unroll
          for (int l = 0; l < NL; ++l)
            acc[l][g] += T(tm.T[j * 4 + l]) * T(I.Minv) * pj +
                         ((l == j) ? T(I.tau) * (dq[g] + T(I.b) * du[g]) : T(0));
        }
      }
    }
#pragma unroll
    for (int l = 0; l < NL; ++l)
#pragma unroll
      for (int g = 0; g < NG; ++g) Y[I.x_off + l * I.N + po[g]] = -w * acc[l][g];
  }
}

static dim3 g3(long long maxlen, int count, int nj) {
  long long b = (maxlen + 255) / 256;
  return dim3((unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b)), count, nj);
}

template <typename T, int NL>
static void apply3d_nl(const ApplyArgs& a, const void* x, void* y, int tr, long long maxN, long long maxc, int count) {
  const T* X = (const T*)x;
  T* Y = (T*)y;
  if (tr)
    hipLaunchKernelGGL((apply3d_u_kernel<T, NL, true>), dim3(a.nwork, NL), dim3(64), 0, a.stream, a.inst, a.work, *a.tm,
                       X, Y);
  else
    hipLaunchKernelGGL((apply3d_u_kernel<T, NL, false>), dim3(a.nwork, NL), dim3(64), 0, a.stream, a.inst, a.work,
                       *a.tm, X, Y);
  hipLaunchKernelGGL((qrows_kernel<T>), g3(maxN, count, NL), dim3(256), 0, a.stream, a.inst, (const T*)a.kinv, X, Y);
  if (tr)
    hipLaunchKernelGGL((prows_kernel<T, NL, true, 3>), g3(maxc, count, 1), dim3(256), 0, a.stream, a.inst, *a.tm, X, Y);
  else
    hipLaunchKernelGGL((prows_kernel<T, NL, false, 3>), g3(maxc, count, 1), dim3(256), 0, a.stream, a.inst, *a.tm, X,
                       Y);
}

template <typename T>
void launch_apply3d(const ApplyArgs& a, const void* x, void* y, int transpose) {
  switch (a.nl) {
    case 1: apply3d_nl<T, 1>(a, x, y, transpose, a.maxN, a.maxc, a.count); break;
    case 2: apply3d_nl<T, 2>(a, x, y, transpose, a.maxN, a.maxc, a.count); break;
    case 3: apply3d_nl<T, 3>(a, x, y, transpose, a.maxN, a.maxc, a.count); break;
    default: apply3d_nl<T, 4>(a, x, y, transpose, a.maxN, a.maxc, a.count); break;
  }
}
template void launch_apply3d<double>(const ApplyArgs&, const void*, void*, int);
template void launch_apply3d<float>(const ApplyArgs&, const void*, void*, int);

// elasticity multigrid level: y = tau A x (mode 0) or y = b - tau A x (mode 1)
template <typename T>
__global__ __launch_bounds__(64) void uapply3d_kernel(const UGridSeg* __restrict__ segs, const int4* __restrict__ work,
                                                      int mode, const T* __restrict__ X, const T* __restrict__ Bv,
                                                      T* __restrict__ Y) {
  const int4 w = work[blockIdx.x];
  const UGridSeg& G = segs[w.x];
  const long long vo = G.voff + blockIdx.y * G.vjstride;
  U3Job<T> J;
  for (int e = 0; e < 3; ++e) { J.n[e] = G.n[e]; J.su[e] = G.su[e]; J.h[e] = T(G.h[e]); }
  J.tau = T(G.tau); J.lam = T(G.lam); J.mu = T(G.mu); J.cp = T(0);
  J.X = X + vo;
  J.Y = Y + vo;
  J.Bv = Bv ? Bv + vo : nullptr;
  J.mode = mode;
  J.P = nullptr;
  J.plstride = 0;
  J.npl = 0;
  J.sp[0] = 1; J.sp[1] = 1;
  for (int l = 0; l < 4; ++l) J.pw[l] = T(0);
  u3_run<T>(J, w.y * kO3, w.z * kO3, w.w * kZC);
}
template <typename T>
void launch_uapply3d(const UGridSeg* segs, const int4* work, int nwork, int nj, int mode, const T* x, const T* b, T* y,
                     hipStream_t s) {
  hipLaunchKernelGGL((uapply3d_kernel<T>), dim3(nwork, nj), dim3(64), 0, s, segs, work, mode, x, b, y);
}
template void launch_uapply3d<double>(const UGridSeg*, const int4*, int, int, int, const double*, const double*,
                                      double*, hipStream_t);
template void launch_uapply3d<float>(const UGridSeg*, const int4*, int, int, int, const float*, const float*, float*,
                                     hipStream_t);

}  // namespace bt
