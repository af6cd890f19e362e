// Sub-system operators of the fixed-stress iterative coupling (section
// "Iterative Coupling Approach": the flow problem is solved with the volumetric
// mean stress held fixed, the mechanics problem with the new pressure, in turn).
//
// On a slab the flow sub-system acts on (q, p) of every time level.  Its
// operator is the slab operator with the displacement set to zero and the
// missing displacement response of the fluid content replaced by the
// fixed-stress term: in the mass rows (multiplied by -1, as everywhere here)
//   sum_j T_ij ( -(1/M) Mp p_j ) + tau B^T q_i   becomes
//   sum_j T_ij ( -(1/M + L) Mp p_j ) + tau B^T q_i.
// The apply kernels compute the first form for x with zero u; the kernel
// below adds -L Mp (T p)_i (Mp is Gauss-nodal: |cell| / 2^d per DoF) and
// clears the u-rows.  The mechanics sub-system is tau A per level (u-rows
// only); zero_rows clears the rows a sub-system does not own.
#include <hip/hip_runtime.h>

#include "prec.h"

namespace bt {

static dim3 fs_grid(long long maxlen, int count) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b < 1 ? 1 : (b > 4096 ? 4096 : b)), count);
}

template <typename T, int NL>
__global__ __launch_bounds__(256) void fs_flow_fix_kernel(const InstDev* __restrict__ insts, TimeMat tm,
                                                          const T* __restrict__ x, T* __restrict__ y) {
  const InstDev& I = insts[blockIdx.y];
  const int dim = I.dim;
  const T wl = T(-I.Lfs * (dim == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]));
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    if (t < I.off_q[0]) {
#pragma unroll
      for (int i = 0; i < NL; ++i) y[I.x_off + i * I.N + t] = T(0);
    } else if (t >= I.off_p) {
      T p[NL];
#pragma unroll
      for (int j = 0; j < NL; ++j) p[j] = x[I.x_off + j * I.N + t];
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        T s = 0;
#pragma unroll
        for (int j = 0; j < NL; ++j) s += T(tm.T[i * 4 + j]) * p[j];
        y[I.x_off + i * I.N + t] += wl * s;
      }
    }
  }
}

// which = 0: clear the u-rows; 1: clear the q- and p-rows (every level)
template <typename T>
__global__ __launch_bounds__(256) void zero_rows_kernel(const InstDev* __restrict__ insts, int nl, int which,
                                                        T* __restrict__ y) {
  const InstDev& I = insts[blockIdx.y];
  const long long lo = which == 0 ? 0 : I.off_q[0], hi = which == 0 ? I.off_q[0] : I.N;
  const long long len = hi - lo;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < nl * len;
       t += (long long)gridDim.x * blockDim.x) {
    const long long j = t / len, r = t - j * len;
    y[I.x_off + j * I.N + lo + r] = T(0);
  }
}

template <typename T>
void launch_fs_flow_fix(const InstDev* insts, int count, long long maxN, int nl, const TimeMat& tm, const T* x, T* y,
                        hipStream_t s) {
  const dim3 g = fs_grid(maxN, count);
  switch (nl) {
    case 1: hipLaunchKernelGGL((fs_flow_fix_kernel<T, 1>), g, dim3(kBlk), 0, s, insts, tm, x, y); break;
    case 2: hipLaunchKernelGGL((fs_flow_fix_kernel<T, 2>), g, dim3(kBlk), 0, s, insts, tm, x, y); break;
    case 3: hipLaunchKernelGGL((fs_flow_fix_kernel<T, 3>), g, dim3(kBlk), 0, s, insts, tm, x, y); break;
    default: hipLaunchKernelGGL((fs_flow_fix_kernel<T, 4>), g, dim3(kBlk), 0, s, insts, tm, x, y); break;
  }
}
template <typename T>
void launch_zero_rows(const InstDev* insts, int count, long long maxN, int nl, int which, T* y, hipStream_t s) {
  hipLaunchKernelGGL((zero_rows_kernel<T>), fs_grid(maxN * nl, count), dim3(kBlk), 0, s, insts, nl, which, y);
}
template void launch_fs_flow_fix<double>(const InstDev*, int, long long, int, const TimeMat&, const double*, double*,
                                         hipStream_t);
template void launch_fs_flow_fix<float>(const InstDev*, int, long long, int, const TimeMat&, const float*, float*,
                                        hipStream_t);
template void launch_zero_rows<double>(const InstDev*, int, long long, int, int, double*, hipStream_t);
template void launch_zero_rows<float>(const InstDev*, int, long long, int, int, float*, hipStream_t);

}  // namespace bt
