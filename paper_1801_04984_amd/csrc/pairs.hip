// Complex-pair level blocks of the preconditioner (section "Monolithic
// Approach": in the real block eigenbasis of the temporal matrix a complex
// eigenvalue alpha +- i beta gives the coupled 2x2 level block
//   [[L, beta M_t], [-beta M_t, L]],   L = alpha M_t + tau K_s,
// whose off-diagonal blocks are the C^+- of the paper).
//
// The block is solved with its couplings kept by the preconditioned
// square-block factorisation (PRESB; Axelsson, Neytcheva and co-authors):
// with H = (alpha + beta) M_t + tau K_s and right-hand side (f, g),
//   w = H^-1 (f - g),  y = H^-1 (g + beta M_t w),  x = w + y.
// That is the exact inverse of [[L, beta M_t], [-beta M_t, L + 2 beta M_t]],
// which differs from the pair block only in its second diagonal block.  Both
// H solves are the level solves of the fixed-stress preconditioner with the
// shift alpha + beta; the three kernels below form the right-hand sides
// between them and combine the results.
#include <hip/hip_runtime.h>

#include "prec.h"
#include "rows.h"

namespace bt {

static dim3 pair_grid(long long maxlen, int count, int npairs) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b)), count, npairs);
}

// save g (level j+1) and form f - g in level j
template <typename T>
__global__ __launch_bounds__(256) void pair_split_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                         T* __restrict__ r, T* __restrict__ save) {
  const InstDev& I = insts[blockIdx.y];
  const int j = ps.j[blockIdx.z];
  const long long l0 = I.x_off + j * I.N, l1 = l0 + I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    const T g = r[l1 + t];
    save[l1 + t] = g;
    r[l0 + t] -= g;
  }
}

// w (level j of z) saved; level j+1 right-hand side g + beta M_t w, where
// M_t w has p-rows only: -|cell|/2^d (b div u(x_g) + p_g / M) at the Gauss
// points x_g of DG-Q1 (Gauss-nodal mass), essential u values masked.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void pair_couple_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                          const T* __restrict__ z, T* __restrict__ save,
                                                          T* __restrict__ r) {
  constexpr int NG = 1 << DIM;
  const InstDev& I = insts[blockIdx.y];
  const int j = ps.j[blockIdx.z];
  const T beta = T(ps.beta[blockIdx.z]);
  const long long l0 = I.x_off + j * I.N, l1 = l0 + I.N;
  const long long np = I.off_p, nitems = np + I.ncells;
  const unsigned n0 = I.n[0], n1 = I.n[1];
  const T w = T(DIM == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]);
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nitems;
       t += (long long)gridDim.x * blockDim.x) {
    if (t < np) {   // u and q rows: M_t has none
      save[l0 + t] = z[l0 + t];
      r[l1 + t] = save[l1 + t];
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
      r[l1 + o] = save[l1 + o] - beta * w * (T(I.b) * du[g] + T(I.Minv) * p);
    }
  }
}

// x = w + y in level j (y stays in level j+1)
template <typename T>
__global__ __launch_bounds__(256) void pair_join_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                        const T* __restrict__ save, T* __restrict__ z) {
  const InstDev& I = insts[blockIdx.y];
  const int j = ps.j[blockIdx.z];
  const long long l0 = I.x_off + j * I.N, l1 = l0 + I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x)
    z[l0 + t] = save[l0 + t] + z[l1 + t];
}

// ---- transposed pair block [[L^T, -beta M_t^T], [beta M_t^T, L^T]] (the
// slab transpose in the basis Q^-T): with H^T = ((alpha + beta) M_t + tau K_s)^T,
//   w = H^-T (f + g),  y = H^-T (g - beta M_t^T w),  x = w - y.
template <typename T>
__global__ __launch_bounds__(256) void pair_split_t_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                           T* __restrict__ r, T* __restrict__ save) {
  const InstDev& I = insts[blockIdx.y];
  const int j = ps.j[blockIdx.z];
  const long long l0 = I.x_off + j * I.N, l1 = l0 + I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    const T g = r[l1 + t];
    save[l1 + t] = g;
    r[l0 + t] += g;
  }
}

// M_t^T w = [-b E p_w; 0; -Mp p_w / M]: u-rows from the E p gather (essential
// u rows keep g), p-rows Gauss-nodal; w (level j of z) saved on the way.
template <typename T, int DIM>
__global__ __launch_bounds__(256) void pair_couple_t_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                            const T* __restrict__ z, T* __restrict__ save,
                                                            T* __restrict__ r) {
  const InstDev& I = insts[blockIdx.y];
  const int j = ps.j[blockIdx.z];
  const T beta = T(ps.beta[blockIdx.z]);
  const long long l0 = I.x_off + j * I.N, l1 = l0 + I.N;
  const T* P = z + l0 + I.off_p;
  const T w = T(DIM == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]);
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    save[l0 + t] = z[l0 + t];
    T v = save[l1 + t];
    if (t < I.off_q[0]) {
      int blk, comp, co[3];
      decode_dof(I, (int)t, blk, comp, co);
      const T ep = ep_node<T, DIM>(I, P, comp, co);
      if (!u_fixed(I, comp, co[0], co[1], co[2])) v += beta * T(I.b) * ep;
    } else if (t >= I.off_p) {
      v += beta * w * T(I.Minv) * z[l0 + t];
    }
    r[l1 + t] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void pair_join_t_kernel(const InstDev* __restrict__ insts, PairSet ps,
                                                          const T* __restrict__ save, T* __restrict__ z) {
  const InstDev& I = insts[blockIdx.y];
  const int j = ps.j[blockIdx.z];
  const long long l0 = I.x_off + j * I.N, l1 = l0 + I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x)
    z[l0 + t] = save[l0 + t] - z[l1 + t];
}

template <typename T>
void launch_pair_split(const InstDev* insts, int count, long long maxN, const PairSet& ps, T* r, T* save,
                       hipStream_t s) {
  hipLaunchKernelGGL((pair_split_kernel<T>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, r, save);
}
template <typename T>
void launch_pair_couple(int dim, const InstDev* insts, int count, long long maxN, const PairSet& ps, const T* z,
                        T* save, T* r, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL((pair_couple_kernel<T, 2>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, z, save,
                       r);
  else
    hipLaunchKernelGGL((pair_couple_kernel<T, 3>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, z, save,
                       r);
}
template <typename T>
void launch_pair_join(const InstDev* insts, int count, long long maxN, const PairSet& ps, const T* save, T* z,
                      hipStream_t s) {
  hipLaunchKernelGGL((pair_join_kernel<T>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, save, z);
}

template <typename T>
void launch_pair_split_t(const InstDev* insts, int count, long long maxN, const PairSet& ps, T* r, T* save,
                         hipStream_t s) {
  hipLaunchKernelGGL((pair_split_t_kernel<T>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, r, save);
}
template <typename T>
void launch_pair_couple_t(int dim, const InstDev* insts, int count, long long maxN, const PairSet& ps, const T* z,
                          T* save, T* r, hipStream_t s) {
  if (dim == 2)
    hipLaunchKernelGGL((pair_couple_t_kernel<T, 2>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, z,
                       save, r);
  else
    hipLaunchKernelGGL((pair_couple_t_kernel<T, 3>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, z,
                       save, r);
}
template <typename T>
void launch_pair_join_t(const InstDev* insts, int count, long long maxN, const PairSet& ps, const T* save, T* z,
                        hipStream_t s) {
  hipLaunchKernelGGL((pair_join_t_kernel<T>), pair_grid(maxN, count, ps.n), dim3(kBlk), 0, s, insts, ps, save, z);
}

#define BT_INST_PAIRS_T(T)                                                                                       \
  template void launch_pair_split_t<T>(const InstDev*, int, long long, const PairSet&, T*, T*, hipStream_t);     \
  template void launch_pair_couple_t<T>(int, const InstDev*, int, long long, const PairSet&, const T*, T*, T*,  \
                                        hipStream_t);                                                            \
  template void launch_pair_join_t<T>(const InstDev*, int, long long, const PairSet&, const T*, T*, hipStream_t);
BT_INST_PAIRS_T(double)
BT_INST_PAIRS_T(float)

template void launch_pair_split<double>(const InstDev*, int, long long, const PairSet&, double*, double*, hipStream_t);
template void launch_pair_split<float>(const InstDev*, int, long long, const PairSet&, float*, float*, hipStream_t);
template void launch_pair_couple<double>(int, const InstDev*, int, long long, const PairSet&, const double*, double*,
                                         double*, hipStream_t);
template void launch_pair_couple<float>(int, const InstDev*, int, long long, const PairSet&, const float*, float*,
                                        float*, hipStream_t);
template void launch_pair_join<double>(const InstDev*, int, long long, const PairSet&, const double*, double*,
                                       hipStream_t);
template void launch_pair_join<float>(const InstDev*, int, long long, const PairSet&, const float*, float*,
                                      hipStream_t);

}  // namespace bt
