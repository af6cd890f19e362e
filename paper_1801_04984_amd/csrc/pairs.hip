// Complex-pair level blocks of the preconditioner (section "Monolithic
// Approach": in the real block eigenbasis of the temporal matrix a complex
// eigenvalue alpha +- i beta gives the coupled 2x2 level block
//   [[L, beta M_t], [-beta M_t, L]],   L = alpha M_t + tau K_s,
// whose off-diagonal blocks are the C^+- of the paper).
//
// The block is solved with its couplings kept by the preconditioned
// square-block factorisation (PRESB; Axelsson, Neytcheva and co-authors):
// with H = (alpha + beta) M_t + tau K_s and right-hand side (f, g),
//   w = H^-1 (f - g),  y = H^-1 (g + beta M_t w),  x = (w + y, y).
// That is the exact inverse of [[L, beta M_t], [-beta M_t, L + 2 beta M_t]],
// which differs from the pair block only in its second diagonal block.  Both
// H solves are the level solves of the fixed-stress preconditioner with the
// shift alpha + beta.
//
// The levels are ordered pair firsts, real levels, pair seconds, so that the
// w solves run in one pass with the real levels (levels 0 .. nl - npairs - 1)
// and the y solves in a second pass over the first npairs level slots: every
// level block costs one level solve.  The kernels below form the right-hand
// sides in place (split: f - g into the first slot; couple: g + beta M_t w
// into the first slot, w saved) and combine the results (join).
#include <hip/hip_runtime.h>

#include "prec.h"
#include "rows.h"

namespace bt {

static dim3 pair_grid(long long maxlen, int count, int npairs) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b)), count, npairs);
}

// first slot: f - g (forward) or f + g (transposed); g stays in the second slot
template <typename T>
__global__ __launch_bounds__(256) void pair_split_kernel(const InstDev* __restrict__ insts, PairSet ps, T sign,
                                                         T* __restrict__ r) {
  const InstDev& I = insts[blockIdx.y];
  const long long l0 = I.x_off + ps.j[blockIdx.z] * I.N, l1 = I.x_off + ps.j2[blockIdx.z] * I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x)
    r[l0 + t] += sign * r[l1 + t];
}

// w (first slot of z) saved; first slot of r = g + beta M_t w, where M_t w has
// p-rows only: -|cell|/2^d (b div u(x_g) + p_g / M) at the Gauss points x_g of
// DG-Q1 (Gauss-nodal mass), essential u values masked.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void pair_couple_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                          const T* __restrict__ z, T* __restrict__ save,
                                                          T* __restrict__ r) {
  constexpr int NG = 1 << DIM;
  const InstDev& I = insts[blockIdx.y];
  const T beta = T(ps.beta[blockIdx.z]);
  const long long l0 = I.x_off + ps.j[blockIdx.z] * I.N, l1 = I.x_off + ps.j2[blockIdx.z] * I.N;
  const long long np = I.off_p, nitems = np + I.ncells;
  const unsigned n0 = I.n[0], n1 = I.n[1];
  const T w = T(DIM == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]);
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nitems;
       t += (long long)gridDim.x * blockDim.x) {
    if (t < np) {   // u and q rows: M_t has none
      save[l0 + t] = z[l0 + t];
      r[l0 + t] = r[l1 + t];
      continue;
    }
    const int cell = (int)(t - np);
    const unsigned q = (unsigned)cell / n0;
    const int ce[3] = {(int)((unsigned)cell - q * n0), (int)(q % n1), DIM == 3 ? (int)(q / n1) : 0};
    const int pb = (int)I.off_p + 2 * ce[0] + I.sp[0] * (2 * ce[1] + I.sp[1] * (DIM == 3 ? 2 * ce[2] : 0));
    T du[NG];
    cell_divu<T, DIM>(I, z + l0, ce, du);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      const int o = pb + (g & 1) + I.sp[0] * (((g >> 1) & 1) + I.sp[1] * ((g >> 2) & 1));
      const T p = z[l0 + o];
      save[l0 + o] = p;
      r[l0 + o] = r[l1 + o] - beta * w * (T(I.b) * du[g] + T(I.Minv) * p);
    }
  }
}

// second slot = y, first slot = w + sign y (y: first slot of z after the second pass)
template <typename T>
__global__ __launch_bounds__(256) void pair_join_kernel(const InstDev* __restrict__ insts, PairSet ps, T sign,
                                                        const T* __restrict__ save, T* __restrict__ z) {
  const InstDev& I = insts[blockIdx.y];
  const long long l0 = I.x_off + ps.j[blockIdx.z] * I.N, l1 = I.x_off + ps.j2[blockIdx.z] * I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N;
       t += (long long)gridDim.x * blockDim.x) {
    const T y = z[l0 + t];
    z[l1 + t] = y;
    z[l0 + t] = save[l0 + t] + sign * y;
  }
}

// ---- transposed pair block [[L^T, -beta M_t^T], [beta M_t^T, L^T]] (the
// slab transpose in the basis Q^-T): with H^T = ((alpha + beta) M_t + tau K_s)^T,
//   w = H^-T (f + g),  y = H^-T (g - beta M_t^T w),  x = (w - y, y).
// M_t^T w = [-b E p_w; 0; -Mp p_w / M]: u-rows from the E p gather (essential
// u rows keep g), p-rows Gauss-nodal; w (first slot of z) saved on the way.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void pair_couple_t_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                            const T* __restrict__ z, T* __restrict__ save,
                                                            T* __restrict__ r) {
  const InstDev& I = insts[blockIdx.y];
  const T beta = T(ps.beta[blockIdx.z]);
  const long long l0 = I.x_off + ps.j[blockIdx.z] * I.N, l1 = I.x_off + ps.j2[blockIdx.z] * I.N;
  const T* P = z + l0 + I.off_p;
  const T w = T(DIM == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]);
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    save[l0 + t] = z[l0 + t];
    T v = r[l1 + t];
    if (t < I.off_q[0]) {
      int blk, comp, co[3];
      decode_dof(I, (int)t, blk, comp, co);
      const T ep = ep_node<T, DIM>(I, P, comp, co);
      if (!u_fixed(I, comp, co[0], co[1], co[2])) v += beta * T(I.b) * ep;
    } else if (t >= I.off_p) {
      v += beta * w * T(I.Minv) * z[l0 + t];
    }
    r[l0 + t] = v;
  }
}

template <typename T>
void launch_pair_split(const InstDev* insts, int count, long long maxN, const PairSet& ps, int transpose, T* r,
                       hipStream_t s) {
  hipLaunchKernelGGL((pair_split_kernel<T>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps,
                     T(transpose ? 1 : -1), r);
}
template <typename T>
void launch_pair_couple(int dim, const InstDev* insts, int count, long long maxN, const PairSet& ps, int transpose,
                        const T* z, T* save, T* r, hipStream_t s) {
  const dim3 g = pair_grid(maxN, count, ps.n);
  if (transpose) {
    if (dim == 2) hipLaunchKernelGGL((pair_couple_t_kernel<T, 2>), g, dim3(kBlk), 0, s, insts, ps, z, save, r);
    else hipLaunchKernelGGL((pair_couple_t_kernel<T, 3>), g, dim3(kBlk), 0, s, insts, ps, z, save, r);
  } else {
    if (dim == 2) hipLaunchKernelGGL((pair_couple_kernel<T, 2>), g, dim3(kBlk), 0, s, insts, ps, z, save, r);
    else hipLaunchKernelGGL((pair_couple_kernel<T, 3>), g, dim3(kBlk), 0, s, insts, ps, z, save, r);
  }
}
template <typename T>
void launch_pair_join(const InstDev* insts, int count, long long maxN, const PairSet& ps, int transpose, const T* save,
                      T* z, hipStream_t s) {
  hipLaunchKernelGGL((pair_join_kernel<T>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps,
                     T(transpose ? -1 : 1), save, z);
}

#define BT_INST_PAIRS(T)                                                                                          \
  template void launch_pair_split<T>(const InstDev*, int, long long, const PairSet&, int, T*, hipStream_t);       \
  template void launch_pair_couple<T>(int, const InstDev*, int, long long, const PairSet&, int, const T*, T*, T*, \
                                      hipStream_t);                                                               \
  template void launch_pair_join<T>(const InstDev*, int, long long, const PairSet&, int, const T*, T*, hipStream_t);
BT_INST_PAIRS(double)
BT_INST_PAIRS(float)

}  // namespace bt
