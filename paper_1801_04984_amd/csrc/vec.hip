// Segmented vector kernels: every vector is a concatenation of segments
// (one per instance, or per instance and multigrid level), each with r+1
// time levels at a fixed stride.  Reductions are two-stage with a fixed
// partition (deterministic: the same inputs give the same bits).
#include "vec.h"

namespace bt {

// ---- fill / copy / cast ------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void fill_kernel(T* __restrict__ x, T v, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    x[i] = v;
}
template <typename A, typename B>
__global__ __launch_bounds__(256) void cast_kernel(const A* __restrict__ x, B* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = (B)x[i];
}
static unsigned nblocks(long long n) {
  long long b = (n + 255) / 256;
  return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}
template <typename T>
void vfill(T* x, T v, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(fill_kernel<T>, dim3(nblocks(n)), dim3(256), 0, s, x, v, n);
}
template void vfill<double>(double*, double, long long, hipStream_t);
template void vfill<float>(float*, float, long long, hipStream_t);
void vcast(const double* x, float* y, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((cast_kernel<double, float>), dim3(nblocks(n)), dim3(256), 0, s, x, y, n);
}
void vcast(const float* x, double* y, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((cast_kernel<float, double>), dim3(nblocks(n)), dim3(256), 0, s, x, y, n);
}

// ---- y = a x + b y over whole vectors ---------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void axpby_kernel(T a, const T* __restrict__ x, T b, T* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i] + b * y[i];
}
template <typename T>
void vaxpby(double a, const T* x, double b, T* y, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL((axpby_kernel<T>), dim3(nblocks(n)), dim3(256), 0, s, T(a), x, T(b), y, n);
}
template void vaxpby<double>(double, const double*, double, double*, long long, hipStream_t);
template void vaxpby<float>(double, const float*, double, float*, long long, hipStream_t);
// y += x (mixed precision accumulate: double += float)
__global__ __launch_bounds__(256) void acc_f32_kernel(const float* __restrict__ x, double* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] += (double)x[i];
}
void vacc(const float* x, double* y, long long n, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(acc_f32_kernel, dim3(nblocks(n)), dim3(256), 0, s, x, y, n);
}

// ---- segmented multi-dot: out[seg][k] = <V_k, w> over segment seg ------------
// stage 1: block b of segment s reduces a fixed chunk for KB vectors
constexpr int kDotThreads = 256;
constexpr int kKBMax = 32;   // vectors per stage-1 launch: w is read once per 32
// the values V[(k0 + k) * ldv + i] of one element for k < nk (0 beyond), in FP64,
// with every load issued before any is used, so that they stay in flight together.
// FP64 rows past nk are skipped by uniform branches.  For FP32 rows the compiler
// moves the conversion into such a branch and waits there, so every row is loaded
// (rows past nk repeat row nk - 1, which the cache serves) and masked afterwards.
template <typename TV, int K>
__device__ __forceinline__ void load_column(const TV* __restrict__ V, long long ldv, int k0, int nk, long long i,
                                            double (&v)[K]) {
  if constexpr (sizeof(TV) == sizeof(double)) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = k < nk ? (double)V[(long long)(k0 + k) * ldv + i] : 0.0;
  } else {
    const int last = nk > 0 ? nk - 1 : 0;
    TV raw[K];
#pragma unroll
    for (int k = 0; k < K; ++k) raw[k] = V[(long long)(k0 + (k < last ? k : last)) * ldv + i];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = k < nk ? (double)raw[k] : 0.0;
  }
}

template <typename TV, typename TW, int kKB>
__global__ __launch_bounds__(kDotThreads) void mdot_stage1(const TV* __restrict__ V, long long ldv, int k0, int nk,
                                                           const TW* __restrict__ w, const VSeg* __restrict__ segs,
                                                           int nchunk, double* __restrict__ partial) {
  const VSeg sg = segs[blockIdx.y];
  const int chunk = blockIdx.x;
  const long long len = sg.len;
  const long long per = (len + nchunk - 1) / nchunk;
  const long long beg = chunk * per, end = beg + per < len ? beg + per : len;
  double acc[kKB];
#pragma unroll
  for (int k = 0; k < kKB; ++k) acc[k] = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += kDotThreads) {
    double v[kKB];
    load_column<TV, kKB>(V, ldv, k0, nk, sg.off + i, v);
    const double wi = (double)w[sg.off + i];
#pragma unroll
    for (int k = 0; k < kKB; ++k) acc[k] += v[k] * wi;
  }
  __shared__ double red[kKB][kDotThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kKB; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < kKB && threadIdx.x < nk) {
    double v = 0.0;
    for (int q = 0; q < kDotThreads / 64; ++q) v += red[threadIdx.x][q];
    partial[((long long)blockIdx.y * 64 + k0 + threadIdx.x) * nchunk + chunk] = v;
  }
}
// stage 2: one block per (vector k, segment); fixed-order tree over the chunk partials
__global__ __launch_bounds__(256) void mdot_stage2(const double* __restrict__ partial, int nchunk,
                                                   double* __restrict__ out, double* __restrict__ hout) {
  const int k = blockIdx.x, s = blockIdx.y;
  const double* p = partial + ((long long)s * 64 + k) * nchunk;
  double v = 0.0;
  for (int c = threadIdx.x; c < nchunk; c += 256) v += p[c];
  __shared__ double red[4];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double r = (red[0] + red[1]) + (red[2] + red[3]);
    out[s * 64 + k] = r;
    if (hout) hout[s * 64 + k] = r;   // host-mapped copy (read after the stream completes)
  }
}

int dot_chunks(long long maxlen) {
  long long c = (maxlen + 1023) / 1024;
  return (int)(c < 1 ? 1 : (c > kMaxChunks ? kMaxChunks : c));
}

template <typename TV, typename TW>
void seg_mdot(const TV* V, long long ldv, int nk, const TW* w, const VSeg* segs, int nseg, int nchunk,
              double* partial, double* out, hipStream_t s, double* hout) {
  // groups of up to 32 vectors; the unrolled width is the smallest of 8, 16, 32 that holds the group
  for (int k0 = 0; k0 < nk; k0 += kKBMax) {
    int kk = nk - k0 < kKBMax ? nk - k0 : kKBMax;
    if (kk <= 8)
      hipLaunchKernelGGL((mdot_stage1<TV, TW, 8>), dim3(nchunk, nseg), dim3(kDotThreads), 0, s, V, ldv, k0, kk, w,
                         segs, nchunk, partial);
    else if (kk <= 16)
      hipLaunchKernelGGL((mdot_stage1<TV, TW, 16>), dim3(nchunk, nseg), dim3(kDotThreads), 0, s, V, ldv, k0, kk, w,
                         segs, nchunk, partial);
    else
      hipLaunchKernelGGL((mdot_stage1<TV, TW, kKBMax>), dim3(nchunk, nseg), dim3(kDotThreads), 0, s, V, ldv, k0, kk,
                         w, segs, nchunk, partial);
  }
  hipLaunchKernelGGL(mdot_stage2, dim3(nk, nseg), dim3(256), 0, s, partial, nchunk, out, hout);
}
template void seg_mdot<double, double>(const double*, long long, int, const double*, const VSeg*, int, int, double*,
                                       double*, hipStream_t, double*);
template void seg_mdot<float, float>(const float*, long long, int, const float*, const VSeg*, int, int, double*,
                                     double*, hipStream_t, double*);

// ---- fused Gram-Schmidt passes (K = nk <= kFuseK basis vectors) -----------------
// pass 2 of classical Gram-Schmidt twice, fused with the update of pass 1:
//   w <- w - sum_k c1[k] V_k,   partial dots <V_k, w> (k < K) and <w, w> (slot K)
// over the same fixed chunks as mdot_stage1 (the V_k values of an element are
// read once for both), reduced by mdot_stage2.
template <typename TV, typename TW, int kFuseK>
__global__ __launch_bounds__(kDotThreads) void gs_update_dot_kernel(const TV* __restrict__ V, long long ldv, int nk,
                                                                    const double* __restrict__ c1,
                                                                    TW* __restrict__ w, const VSeg* __restrict__ segs,
                                                                    int nchunk, double* __restrict__ partial) {
  const VSeg sg = segs[blockIdx.y];
  const int chunk = blockIdx.x;
  const long long len = sg.len;
  const long long per = (len + nchunk - 1) / nchunk;
  const long long beg = chunk * per, end = beg + per < len ? beg + per : len;
  __shared__ double cs[kFuseK];
  if (threadIdx.x < kFuseK) cs[threadIdx.x] = threadIdx.x < nk ? c1[blockIdx.y * 64 + threadIdx.x] : 0.0;
  __syncthreads();
  double acc[kFuseK + 1];
#pragma unroll
  for (int k = 0; k <= kFuseK; ++k) acc[k] = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += kDotThreads) {
    double v[kFuseK];
    load_column<TV, kFuseK>(V, ldv, 0, nk, sg.off + i, v);
    double wi = (double)w[sg.off + i];
#pragma unroll
    for (int k = 0; k < kFuseK; ++k) wi -= cs[k] * v[k];
    const TW wt = (TW)wi;
    w[sg.off + i] = wt;
    const double wn = (double)wt;
#pragma unroll
    for (int k = 0; k < kFuseK; ++k) acc[k] += v[k] * wn;
    acc[kFuseK] += wn * wn;
  }
  __shared__ double red[kFuseK + 1][kDotThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k <= kFuseK; ++k) {
    double v = acc[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  for (int k = threadIdx.x; k <= nk; k += kDotThreads) {
    const int src = k < nk ? k : kFuseK;
    double v = 0.0;
    for (int q = 0; q < kDotThreads / 64; ++q) v += red[src][q];
    partial[((long long)blockIdx.y * 64 + k) * nchunk + chunk] = v;
  }
}
// update of pass 2 and normalisation in one sweep:
//   w <- f (w - sum_k c2[k] V_k),  f = 1 / sqrt(c2[K] - sum_k c2[k]^2)  (0 for a zero norm)
// (c2[K] = |w|^2 before the update; the removed components are orthogonal, so the
// norm after it follows by Pythagoras)
template <typename TV, typename TW, int kFuseK>
__global__ __launch_bounds__(256) void gs_update_scale_kernel(const TV* __restrict__ V, long long ldv, int nk,
                                                              const double* __restrict__ c2, TW* __restrict__ w,
                                                              const VSeg* __restrict__ segs) {
  const VSeg sg = segs[blockIdx.y];
  __shared__ double cs[kFuseK];
  __shared__ double fs;
  const double* c = c2 + blockIdx.y * 64;
  if (threadIdx.x < kFuseK) cs[threadIdx.x] = threadIdx.x < nk ? c[threadIdx.x] : 0.0;
  if (threadIdx.x == 0) {
    double n2 = c[nk];
    for (int k = 0; k < nk; ++k) n2 -= c[k] * c[k];
    fs = n2 > 0.0 ? 1.0 / sqrt(n2) : 0.0;
  }
  __syncthreads();
  const double f = fs;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x) {
    double v[kFuseK];
    load_column<TV, kFuseK>(V, ldv, 0, nk, sg.off + i, v);
    double wi = (double)w[sg.off + i];
#pragma unroll
    for (int k = 0; k < kFuseK; ++k) wi -= cs[k] * v[k];
    const TW wt = (TW)wi;   // rounded to the storage type before the scaling, as a separate pass would
    w[sg.off + i] = (TW)(f * (double)wt);
  }
}
template <typename TV, typename TW>
void gs_update_dot(const TV* V, long long ldv, int nk, const double* c1, TW* w, const VSeg* segs, int nseg, int nchunk,
                   double* partial, double* out, hipStream_t s, double* hout) {
  // the unrolled width is the smallest of 8, 16, 32 that holds nk
  if (nk <= 8)
    hipLaunchKernelGGL((gs_update_dot_kernel<TV, TW, 8>), dim3(nchunk, nseg), dim3(kDotThreads), 0, s, V, ldv, nk,
                       c1, w, segs, nchunk, partial);
  else if (nk <= 16)
    hipLaunchKernelGGL((gs_update_dot_kernel<TV, TW, 16>), dim3(nchunk, nseg), dim3(kDotThreads), 0, s, V, ldv, nk,
                       c1, w, segs, nchunk, partial);
  else
    hipLaunchKernelGGL((gs_update_dot_kernel<TV, TW, kFuseK>), dim3(nchunk, nseg), dim3(kDotThreads), 0, s, V, ldv,
                       nk, c1, w, segs, nchunk, partial);
  hipLaunchKernelGGL(mdot_stage2, dim3(nk + 1, nseg), dim3(256), 0, s, partial, nchunk, out, hout);
}
template <typename TV, typename TW>
void gs_update_scale(const TV* V, long long ldv, int nk, const double* c2, TW* w, const VSeg* segs, int nseg,
                     long long maxlen, hipStream_t s) {
  long long b = (maxlen + 255) / 256;
  unsigned gx = (unsigned)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
  if (nk <= 8)
    hipLaunchKernelGGL((gs_update_scale_kernel<TV, TW, 8>), dim3(gx, nseg), dim3(256), 0, s, V, ldv, nk, c2, w, segs);
  else if (nk <= 16)
    hipLaunchKernelGGL((gs_update_scale_kernel<TV, TW, 16>), dim3(gx, nseg), dim3(256), 0, s, V, ldv, nk, c2, w,
                       segs);
  else
    hipLaunchKernelGGL((gs_update_scale_kernel<TV, TW, kFuseK>), dim3(gx, nseg), dim3(256), 0, s, V, ldv, nk, c2, w,
                       segs);
}
template void gs_update_dot<double, double>(const double*, long long, int, const double*, double*, const VSeg*, int,
                                            int, double*, double*, hipStream_t, double*);
template void gs_update_dot<float, float>(const float*, long long, int, const double*, float*, const VSeg*, int, int,
                                          double*, double*, hipStream_t, double*);
template void gs_update_scale<double, double>(const double*, long long, int, const double*, double*, const VSeg*, int,
                                              long long, hipStream_t);
template void gs_update_scale<float, float>(const float*, long long, int, const double*, float*, const VSeg*, int,
                                            long long, hipStream_t);

// ---- classical Gram-Schmidt twice with delayed reorthogonalisation ---------------
// (one reduction and one update sweep over the basis per Arnoldi step instead of
// two and three).  Step nk: basis slots 0..nk-1 hold the final orthonormal vectors,
// slot nk the candidate u of the next one (projected once, not normalised), slot
// nk+1 the operator applied to u, w.  The reduction gives a = V^T u, b = V^T w,
// alpha = u.u and gamma = u.w:
//   out[seg*64 + k] = a_k, out[seg*64 + nk + k] = b_k (k < nk),
//   out[seg*64 + 2 nk] = alpha, out[seg*64 + 2 nk + 1] = gamma.
// The update then writes the final vector of slot nk, v = (u - V a) / nu with
// nu = sqrt(alpha - |a|^2) (the removed components are orthogonal: Pythagoras), and
// the next candidate into slot nk+1, u' = (w - V b - e v) / nu with e = v.w =
// (gamma - a.b) / nu: w projected once on the complement of the basis including
// v, scaled by 1/nu, which is the once-projected A P^-1 v (A P^-1 V a lies in the
// span of the basis).  |u'|^2 is reduced on the way.
template <typename TV, int K>
__global__ __launch_bounds__(kDotThreads) void dcgs_dots_kernel(const TV* __restrict__ V, long long ldv, int nk,
                                                                const VSeg* __restrict__ segs, int nchunk,
                                                                double* __restrict__ partial) {
  const VSeg sg = segs[blockIdx.y];
  const int chunk = blockIdx.x;
  const long long len = sg.len;
  const long long per = (len + nchunk - 1) / nchunk;
  const long long beg = chunk * per, end = beg + per < len ? beg + per : len;
  const TV* u = V + (long long)nk * ldv;
  const TV* w = u + ldv;
  double acc[2 * K + 2];
#pragma unroll
  for (int k = 0; k < 2 * K + 2; ++k) acc[k] = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += kDotThreads) {
    double v[K];
    load_column<TV, K>(V, ldv, 0, nk, sg.off + i, v);
    const double ui = (double)u[sg.off + i], wi = (double)w[sg.off + i];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      acc[k] += v[k] * ui;
      acc[K + k] += v[k] * wi;
    }
    acc[2 * K] += ui * ui;
    acc[2 * K + 1] += ui * wi;
  }
  __shared__ double red[2 * K + 2][kDotThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 2 * K + 2; ++k) {
    double x = acc[k];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) red[k][wv] = x;
  }
  __syncthreads();
  // output slot q < 2 nk + 2 from accumulator: a_k at k, b_k at K + k, alpha, gamma at 2K, 2K+1
  for (int q = threadIdx.x; q < 2 * nk + 2; q += kDotThreads) {
    const int src = q < nk ? q : (q < 2 * nk ? K + q - nk : 2 * K + q - 2 * nk);
    double x = 0.0;
    for (int r = 0; r < kDotThreads / 64; ++r) x += red[src][r];
    partial[((long long)blockIdx.y * 64 + q) * nchunk + chunk] = x;
  }
}

template <typename TV, int K>
__global__ __launch_bounds__(kDotThreads) void dcgs_update_kernel(TV* __restrict__ V, long long ldv, int nk,
                                                                  const double* __restrict__ c,
                                                                  const VSeg* __restrict__ segs, int nchunk,
                                                                  double* __restrict__ partial) {
  const VSeg sg = segs[blockIdx.y];
  const int chunk = blockIdx.x;
  const long long len = sg.len;
  const long long per = (len + nchunk - 1) / nchunk;
  const long long beg = chunk * per, end = beg + per < len ? beg + per : len;
  __shared__ double ca[K], cb[K];
  __shared__ double fs, es;
  const double* cs = c + blockIdx.y * 64;
  if (threadIdx.x < K) {
    ca[threadIdx.x] = threadIdx.x < nk ? cs[threadIdx.x] : 0.0;
    cb[threadIdx.x] = threadIdx.x < nk ? cs[nk + threadIdx.x] : 0.0;
  }
  if (threadIdx.x == 0) {
    double n2 = cs[2 * nk], ab = 0.0;
    for (int k = 0; k < nk; ++k) {
      n2 -= cs[k] * cs[k];
      ab += cs[k] * cs[nk + k];
    }
    const double nu = n2 > 0.0 ? sqrt(n2) : 0.0;
    fs = nu > 0.0 ? 1.0 / nu : 0.0;      // a zero norm (breakdown) gives zero vectors
    es = (cs[2 * nk + 1] - ab) * fs;
  }
  __syncthreads();
  const double f = fs, e = es;
  TV* u = V + (long long)nk * ldv;
  TV* w = u + ldv;
  double nacc = 0.0;
  for (long long i = beg + threadIdx.x; i < end; i += kDotThreads) {
    double v[K];
    load_column<TV, K>(V, ldv, 0, nk, sg.off + i, v);
    double ui = (double)u[sg.off + i], wi = (double)w[sg.off + i];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ui -= ca[k] * v[k];
      wi -= cb[k] * v[k];
    }
    const TV vt = (TV)(f * ui);          // the final vector, in the storage type
    const TV ut = (TV)(f * (wi - e * (double)vt));
    u[sg.off + i] = vt;
    w[sg.off + i] = ut;
    nacc += (double)ut * (double)ut;
  }
  __shared__ double red[kDotThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int o = 32; o > 0; o >>= 1) nacc += __shfl_down(nacc, o, 64);
  if (lane == 0) red[wv] = nacc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0;
    for (int r = 0; r < kDotThreads / 64; ++r) x += red[r];
    partial[((long long)blockIdx.y * 64) * nchunk + chunk] = x;
  }
}

template <typename T>
void dcgs_step(T* V, long long ldv, int nk, const VSeg* segs, int nseg, int nchunk, double* partial, double* dots,
               double* norm, hipStream_t s, double* hdots, double* hnorm) {
  const dim3 g(nchunk, nseg), b(kDotThreads);
  if (nk <= 8) {
    hipLaunchKernelGGL((dcgs_dots_kernel<T, 8>), g, b, 0, s, V, ldv, nk, segs, nchunk, partial);
  } else if (nk <= 16) {
    hipLaunchKernelGGL((dcgs_dots_kernel<T, 16>), g, b, 0, s, V, ldv, nk, segs, nchunk, partial);
  } else {
    hipLaunchKernelGGL((dcgs_dots_kernel<T, kLowSyncMax>), g, b, 0, s, V, ldv, nk, segs, nchunk, partial);
  }
  hipLaunchKernelGGL(mdot_stage2, dim3(2 * nk + 2, nseg), dim3(256), 0, s, partial, nchunk, dots, hdots);
  if (nk <= 8) {
    hipLaunchKernelGGL((dcgs_update_kernel<T, 8>), g, b, 0, s, V, ldv, nk, dots, segs, nchunk, partial);
  } else if (nk <= 16) {
    hipLaunchKernelGGL((dcgs_update_kernel<T, 16>), g, b, 0, s, V, ldv, nk, dots, segs, nchunk, partial);
  } else {
    hipLaunchKernelGGL((dcgs_update_kernel<T, kLowSyncMax>), g, b, 0, s, V, ldv, nk, dots, segs, nchunk, partial);
  }
  hipLaunchKernelGGL(mdot_stage2, dim3(1, nseg), dim3(256), 0, s, partial, nchunk, norm, hnorm);
}
template void dcgs_step<double>(double*, long long, int, const VSeg*, int, int, double*, double*, double*, hipStream_t,
                                double*, double*);
template void dcgs_step<float>(float*, long long, int, const VSeg*, int, int, double*, double*, double*, hipStream_t,
                               double*, double*);

// ---- plain copy (a kernel, so that it can sit in a captured graph) ----------------
template <typename T>
__global__ __launch_bounds__(256) void vcopy_kernel(const T* __restrict__ x, T* __restrict__ y, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    y[i] = x[i];
}
template <typename T>
void vcopy(const T* x, T* y, long long n, hipStream_t s) {
  long long b = (n + 255) / 256;
  unsigned gx = (unsigned)(b > 4096 ? 4096 : (b < 1 ? 1 : b));
  hipLaunchKernelGGL((vcopy_kernel<T>), dim3(gx), dim3(256), 0, s, x, y, n);
}
template void vcopy<double>(const double*, double*, long long, hipStream_t);
template void vcopy<float>(const float*, float*, long long, hipStream_t);

// ---- segmented multi-axpy: w[seg] += sum_k c[seg][k] V_k[seg] -----------------
template <typename TV, typename TW>
__global__ __launch_bounds__(256) void maxpy_kernel(const TV* __restrict__ V, long long ldv, int nk, const double* __restrict__ c,
                             double csign, TW* __restrict__ w, const VSeg* __restrict__ segs) {
  const VSeg sg = segs[blockIdx.y];
  const double* cs = c + blockIdx.y * 64;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x) {
    double v = (double)w[sg.off + i];
    for (int k = 0; k < nk; ++k) v += csign * cs[k] * (double)V[(long long)k * ldv + sg.off + i];
    w[sg.off + i] = (TW)v;
  }
}
template <typename TV, typename TW>
void seg_maxpy(const TV* V, long long ldv, int nk, const double* c, double csign, TW* w, const VSeg* segs, int nseg,
               long long maxlen, hipStream_t s) {
  long long b = (maxlen + 255) / 256;
  unsigned gx = (unsigned)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
  hipLaunchKernelGGL((maxpy_kernel<TV, TW>), dim3(gx, nseg), dim3(256), 0, s, V, ldv, nk, c, csign, w, segs);
}
template void seg_maxpy<double, double>(const double*, long long, int, const double*, double, double*, const VSeg*,
                                        int, long long, hipStream_t);
template void seg_maxpy<float, float>(const float*, long long, int, const double*, double, float*, const VSeg*, int,
                                      long long, hipStream_t);
template void seg_maxpy<float, double>(const float*, long long, int, const double*, double, double*, const VSeg*, int,
                                       long long, hipStream_t);

// ---- segmented scale: y[seg] = s[seg*64 + idx] * x[seg] (idx-th coefficient) ----------
template <typename TX, typename TY>
__global__ __launch_bounds__(256) void sscale_kernel(const TX* __restrict__ x, TY* __restrict__ y, const double* __restrict__ sc, int idx,
                              int inv, const VSeg* __restrict__ segs) {
  const VSeg sg = segs[blockIdx.y];
  double f = sc[blockIdx.y * 64 + idx];
  if (inv == 3) {
    // squared norm by Pythagoras: sc[idx] = |w|^2 before removing the components
    // sc[0..idx-1] along orthonormal vectors
    const double* c = sc + blockIdx.y * 64;
    for (int i = 0; i < idx; ++i) f -= c[i] * c[i];
    inv = 2;
  }
  if (inv == 1) f = f > 0.0 ? 1.0 / f : 0.0;
  else if (inv == 2) f = f > 0.0 ? 1.0 / sqrt(f) : 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x)
    y[sg.off + i] = (TY)(f * (double)x[sg.off + i]);
}
template <typename TX, typename TY>
void seg_scale(const TX* x, TY* y, const double* sc, int idx, int inv, const VSeg* segs, int nseg, long long maxlen,
               hipStream_t s) {
  long long b = (maxlen + 255) / 256;
  unsigned gx = (unsigned)(b > 2048 ? 2048 : (b < 1 ? 1 : b));
  hipLaunchKernelGGL((sscale_kernel<TX, TY>), dim3(gx, nseg), dim3(256), 0, s, x, y, sc, idx, inv, segs);
}
template void seg_scale<double, double>(const double*, double*, const double*, int, int, const VSeg*, int, long long,
                                        hipStream_t);
template void seg_scale<float, float>(const float*, float*, const double*, int, int, const VSeg*, int, long long,
                                      hipStream_t);
template void seg_scale<double, float>(const double*, float*, const double*, int, int, const VSeg*, int, long long,
                                       hipStream_t);

// ---- time transform: y_i = sum_j M_ij x_j per spatial DoF (all instances) -----
template <typename T, int NL>
__global__ __launch_bounds__(256) void ttrans_kernel(const InstDev* __restrict__ insts, const T* __restrict__ x, T* __restrict__ y, Mat4 M) {
  const InstDev& I = insts[blockIdx.y];
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < I.N; k += (long long)gridDim.x * blockDim.x) {
    T v[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) v[j] = x[I.x_off + j * I.N + k];
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      T s = 0;
#pragma unroll
      for (int j = 0; j < NL; ++j) s += T(M.m[i * 4 + j]) * v[j];
      y[I.x_off + i * I.N + k] = s;
    }
  }
}
template <typename T>
void time_transform(const InstDev* insts, int count, long long maxN, int nl, const Mat4& M, const T* x, T* y,
                    hipStream_t s) {
  long long b = (maxN + 255) / 256;
  dim3 g((unsigned)(b > 4096 ? 4096 : b), count);
  switch (nl) {
    case 1: hipLaunchKernelGGL((ttrans_kernel<T, 1>), g, dim3(256), 0, s, insts, x, y, M); break;
    case 2: hipLaunchKernelGGL((ttrans_kernel<T, 2>), g, dim3(256), 0, s, insts, x, y, M); break;
    case 3: hipLaunchKernelGGL((ttrans_kernel<T, 3>), g, dim3(256), 0, s, insts, x, y, M); break;
    default: hipLaunchKernelGGL((ttrans_kernel<T, 4>), g, dim3(256), 0, s, insts, x, y, M); break;
  }
}
template void time_transform<double>(const InstDev*, int, long long, int, const Mat4&, const double*, double*,
                                     hipStream_t);
template void time_transform<float>(const InstDev*, int, long long, int, const Mat4&, const float*, float*,
                                    hipStream_t);

// ---- Chebyshev update on level segments -------------------------------------------
// x += d; r -= y; d = rho d + sig Dinv r      (y = A d computed by the caller)
// first step (init != 0): r = b - y0 is not touched; d = sig Dinv r; x untouched.
template <typename T, int MODE>
__global__ __launch_bounds__(256) void cheb_kernel(const LSeg* __restrict__ segs, double rho, double sig, T* __restrict__ x,
                            T* __restrict__ r, T* __restrict__ d, const T* __restrict__ y,
                            const T* __restrict__ dinv, const T* __restrict__ b) {
  const LSeg sg = segs[blockIdx.y];
  const int j = blockIdx.z;
  const long long off = sg.off + j * sg.jstride, doff = sg.doff + j * sg.djstride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x) {
    const T di = dinv[doff + i];
    if constexpr (MODE == 0) {         // init: d = sig Dinv r
      d[off + i] = T(sig) * di * r[off + i];
    } else if constexpr (MODE == 2) {  // init from x = 0: x = 0, r = b, d = sig Dinv b
      const T bb = b[off + i];
      x[off + i] = T(0);
      r[off + i] = bb;
      d[off + i] = T(sig) * di * bb;
    } else {                 // regular step
      const T dd = d[off + i];
      x[off + i] += dd;
      const T rr = r[off + i] - y[off + i];
      r[off + i] = rr;
      d[off + i] = T(rho) * dd + T(sig) * di * rr;
    }
  }
}
// final: x += d
template <typename T>
__global__ __launch_bounds__(256) void addseg_kernel(const LSeg* __restrict__ segs, const T* __restrict__ d, T* __restrict__ x, double a) {
  const LSeg sg = segs[blockIdx.y];
  const long long off = sg.off + blockIdx.z * sg.jstride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x)
    x[off + i] += T(a) * d[off + i];
}
static dim3 lgrid(long long maxlen, int nseg, int nj) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b)), nseg, nj);
}
template <typename T>
void cheb_update(const LSeg* segs, int nseg, int nj, long long maxlen, int mode, double rho, double sig, T* x, T* r,
                 T* d, const T* y, const T* dinv, const T* b, hipStream_t s) {
  const dim3 g = lgrid(maxlen, nseg, nj);
  if (mode == 0)
    hipLaunchKernelGGL((cheb_kernel<T, 0>), g, dim3(kBlk), 0, s, segs, rho, sig, x, r, d, y, dinv, b);
  else if (mode == 2)
    hipLaunchKernelGGL((cheb_kernel<T, 2>), g, dim3(kBlk), 0, s, segs, rho, sig, x, r, d, y, dinv, b);
  else
    hipLaunchKernelGGL((cheb_kernel<T, 1>), g, dim3(kBlk), 0, s, segs, rho, sig, x, r, d, y, dinv, b);
}
template <typename T>
void seg_add(const LSeg* segs, int nseg, int nj, long long maxlen, const T* d, T* x, double a, hipStream_t s) {
  hipLaunchKernelGGL((addseg_kernel<T>), lgrid(maxlen, nseg, nj), dim3(kBlk), 0, s, segs, d, x, a);
}
template void cheb_update<double>(const LSeg*, int, int, long long, int, double, double, double*, double*, double*,
                                  const double*, const double*, const double*, hipStream_t);
template void cheb_update<float>(const LSeg*, int, int, long long, int, double, double, float*, float*, float*,
                                 const float*, const float*, const float*, hipStream_t);
template void seg_add<double>(const LSeg*, int, int, long long, const double*, double*, double, hipStream_t);
template void seg_add<float>(const LSeg*, int, int, long long, const float*, float*, double, hipStream_t);

// zero a level segment set
template <typename T>
__global__ __launch_bounds__(256) void zseg_kernel(const LSeg* __restrict__ segs, T* __restrict__ x) {
  const LSeg sg = segs[blockIdx.y];
  const long long off = sg.off + blockIdx.z * sg.jstride;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < sg.len;
       i += (long long)gridDim.x * blockDim.x)
    x[off + i] = T(0);
}
template <typename T>
void seg_zero(const LSeg* segs, int nseg, int nj, long long maxlen, T* x, hipStream_t s) {
  hipLaunchKernelGGL((zseg_kernel<T>), lgrid(maxlen, nseg, nj), dim3(kBlk), 0, s, segs, x);
}
template void seg_zero<double>(const LSeg*, int, int, long long, double*, hipStream_t);
template void seg_zero<float>(const LSeg*, int, int, long long, float*, hipStream_t);

// ---- dense coarse solve: x_seg = Ainv_seg b_seg (FP64 matrices, any T vectors) -----
// one block per (segment, time level); Ainv row-major n x n at segs[].moff (+ j*mjstride)
template <typename T>
__global__ __launch_bounds__(256) void dense_kernel(const DSeg* __restrict__ segs, const double* __restrict__ Ainv,
                                                    const T* __restrict__ b, T* __restrict__ x) {
  const DSeg sg = segs[blockIdx.y];
  const int j = blockIdx.z;
  const double* A = Ainv + sg.moff + (long long)j * sg.mjstride;
  const long long vo = sg.off + j * sg.jstride;
  const int n = sg.n;
  extern __shared__ double sb[];
  for (int i = threadIdx.x; i < n; i += blockDim.x) sb[i] = (double)b[vo + i];
  __syncthreads();
  for (int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); row < n; row += gridDim.x * (blockDim.x / 64)) {
    double s = 0.0;
    for (int c = threadIdx.x & 63; c < n; c += 64) s += A[(long long)row * n + c] * sb[c];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) x[vo + row] = (T)s;
  }
}
// one wave per row, all levels at once (the matrix is read once per row)
template <typename T, int NJ>
__global__ __launch_bounds__(256) void dense_shared_kernel(const DSeg* __restrict__ segs,
                                                           const double* __restrict__ Ainv, const T* __restrict__ b,
                                                           T* __restrict__ x) {
  const DSeg sg = segs[blockIdx.y];
  const double* A = Ainv + sg.moff;
  const int n = sg.n;
  const int lane = threadIdx.x & 63;
  for (int row = blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); row < n; row += gridDim.x * (blockDim.x / 64)) {
    const double* Ar = A + (long long)row * n;
    double s[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j) s[j] = 0.0;
    for (int c = lane; c < n; c += 64) {
      const double a = Ar[c];
#pragma unroll
      for (int j = 0; j < NJ; ++j) s[j] += a * (double)b[sg.off + j * sg.jstride + c];
    }
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      double v = s[j];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
      if (lane == 0) x[sg.off + j * sg.jstride + row] = (T)v;
    }
  }
}

template <typename T>
void dense_solve(const DSeg* segs, int nseg, int nj, int maxn, bool shared, const double* Ainv, const T* b, T* x,
                 hipStream_t s) {
  unsigned gx = (unsigned)((maxn + 3) / 4);   // one wave per row
  if (gx > 2048) gx = 2048;
  if (shared) {
    switch (nj) {
      case 1: hipLaunchKernelGGL((dense_shared_kernel<T, 1>), dim3(gx, nseg), dim3(256), 0, s, segs, Ainv, b, x); break;
      case 2: hipLaunchKernelGGL((dense_shared_kernel<T, 2>), dim3(gx, nseg), dim3(256), 0, s, segs, Ainv, b, x); break;
      case 3: hipLaunchKernelGGL((dense_shared_kernel<T, 3>), dim3(gx, nseg), dim3(256), 0, s, segs, Ainv, b, x); break;
      default: hipLaunchKernelGGL((dense_shared_kernel<T, 4>), dim3(gx, nseg), dim3(256), 0, s, segs, Ainv, b, x); break;
    }
    return;
  }
  hipLaunchKernelGGL((dense_kernel<T>), dim3(gx, nseg, nj), dim3(256), maxn * sizeof(double), s, segs, Ainv, b, x);
}
template void dense_solve<double>(const DSeg*, int, int, int, bool, const double*, const double*, double*, hipStream_t);
template void dense_solve<float>(const DSeg*, int, int, int, bool, const double*, const float*, float*, hipStream_t);

// Gauss-Jordan exchange step k on every matrix of the batch.  With p = a_kk:
//   a_kk <- 1/p,  a_kj <- -a_kj/p,  a_ik <- a_ik/p,  a_ij <- a_ij - a_ik a_kj/p,
// which exchanges unknown k with equation k; after all n steps the array holds
// the inverse.  Row and column k are read from a snapshot taken by the previous
// step (parity k & 1), so every element is read and written by its own thread
// only; the threads of row/column k+1 store the snapshot for the next step.
__global__ __launch_bounds__(256) void gj_init_kernel(const GJMat* __restrict__ mats, const double* __restrict__ A,
                                                      double* __restrict__ snap) {
  const GJMat m = mats[blockIdx.y];
  const double* a = A + m.moff;
  double* S = snap + m.soff;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < m.n; t += gridDim.x * blockDim.x) {
    S[t] = a[t];                              // row 0
    S[m.n + t] = a[(long long)t * m.n];       // column 0
  }
}

__global__ __launch_bounds__(256) void gj_step_kernel(const GJMat* __restrict__ mats, int k, double* __restrict__ A,
                                                      double* __restrict__ snap, int* __restrict__ bad) {
  const GJMat m = mats[blockIdx.z];
  const int n = m.n;
  const int i = blockIdx.y;
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || i >= n || j >= n) return;
  const double* Rs = snap + m.soff + (k & 1) * 2 * (long long)n;
  const double* Cs = Rs + n;
  double* Rn = snap + m.soff + ((k & 1) ^ 1) * 2 * (long long)n;
  double* Cn = Rn + n;
  const double p = Cs[k];
  const double ip = 1.0 / p;
  double* a = A + m.moff + (long long)i * n + j;
  double v;
  if (i == k) v = (j == k) ? ip : -Rs[j] * ip;
  else if (j == k) v = Cs[i] * ip;
  else v = *a - Cs[i] * Rs[j] * ip;
  *a = v;
  if (k + 1 < n) {
    if (i == k + 1) Rn[j] = v;
    if (j == k + 1) Cn[i] = v;
  }
  if (i == k && j == k && !(p != 0.0 && isfinite(p))) *bad = 1;
}

void dense_invert(const GJMat* mats, int nmats, int maxn, double* A, double* snap, int* bad, hipStream_t s) {
  if (nmats <= 0 || maxn <= 0) return;
  const unsigned gx = (unsigned)((maxn + 255) / 256);
  hipLaunchKernelGGL(gj_init_kernel, dim3(gx, nmats), dim3(256), 0, s, mats, (const double*)A, snap);
  for (int k = 0; k < maxn; ++k)
    hipLaunchKernelGGL(gj_step_kernel, dim3(gx, maxn, nmats), dim3(256), 0, s, mats, k, A, snap, bad);
}

}  // namespace bt
