// Segmented vector kernels (vec.hip).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace bt {

struct VSeg {          // a contiguous segment of a vector (one instance)
  long long off, len;
};
struct LSeg {          // a multigrid-level field segment with r+1 time levels
  long long off, jstride, len;
  long long doff, djstride;  // matching diagonal-inverse segment
};
struct DSeg {          // dense coarse solve segment
  long long off, jstride;
  int n, pad;
  long long moff, mjstride;
};
struct GJMat {         // one dense matrix to invert in place: offset, snapshot offset, order
  long long moff, soff;
  int n, pad;
};
struct Mat4 { double m[16]; };

constexpr int kMaxChunks = 2048;  // dot-product partial sums per segment (upper bound)
int dot_chunks(long long maxlen);

template <typename T> void vfill(T* x, T v, long long n, hipStream_t s);
void vcast(const double* x, float* y, long long n, hipStream_t s);
void vcast(const float* x, double* y, long long n, hipStream_t s);
template <typename T>
void vaxpby(double a, const T* x, double b, T* y, long long n, hipStream_t s);
void vacc(const float* x, double* y, long long n, hipStream_t s);
// out[seg * 64 + k] = V_k[seg] . w[seg]; hout (optional): the same values also
// written to host-mapped pinned memory
template <typename TV, typename TW>
void seg_mdot(const TV* V, long long ldv, int nk, const TW* w, const VSeg* segs, int nseg, int nchunk,
              double* partial, double* out, hipStream_t s, double* hout = nullptr);
template <typename T> void vcopy(const T* x, T* y, long long n, hipStream_t s);
// fused classical Gram-Schmidt passes for nk <= kFuseK basis vectors (see vec.hip):
// w -= V c1 with out[seg*64 + k] = <V_k, w> (k < nk), out[seg*64 + nk] = <w, w>;
// then w = (w - V c2) / sqrt(c2[nk] - |c2[0..nk)|^2)
constexpr int kFuseK = 32;
template <typename TV, typename TW>
void gs_update_dot(const TV* V, long long ldv, int nk, const double* c1, TW* w, const VSeg* segs, int nseg, int nchunk,
                   double* partial, double* out, hipStream_t s, double* hout = nullptr);
template <typename TV, typename TW>
void gs_update_scale(const TV* V, long long ldv, int nk, const double* c2, TW* w, const VSeg* segs, int nseg,
                     long long maxlen, hipStream_t s);
// one Arnoldi step of classical Gram-Schmidt twice with delayed reorthogonalisation
// (vec.hip), nk <= kLowSyncMax final basis vectors: slot nk (candidate u) becomes
// final, slot nk+1 (w = A P^-1 u) the next candidate.  dots[seg*64 + ...]:
// V^T u (nk), V^T w (nk), u.u, u.w; norm[seg*64] = |next candidate|^2; hdots,
// hnorm: host-mapped copies.
constexpr int kLowSyncMax = 31;
template <typename T>
void dcgs_step(T* V, long long ldv, int nk, const VSeg* segs, int nseg, int nchunk, double* partial, double* dots,
               double* norm, hipStream_t s, double* hdots, double* hnorm);
template <typename TV, typename TW>
void seg_maxpy(const TV* V, long long ldv, int nk, const double* c, double csign, TW* w, const VSeg* segs, int nseg,
               long long maxlen, hipStream_t s);
template <typename TX, typename TY>
// y[seg] = f x[seg] with f = sc[seg*64+idx] (inv 0), its inverse (1), its inverse
// square root (2), or 1 / sqrt(sc[idx] - sum_{i<idx} sc[i]^2) (3); zero for a
// non-positive argument (1-3)
void seg_scale(const TX* x, TY* y, const double* sc, int idx, int inv, const VSeg* segs, int nseg, long long maxlen,
               hipStream_t s);
template <typename T>
void time_transform(const InstDev* insts, int count, long long maxN, int nl, const Mat4& M, const T* x, T* y,
                    hipStream_t s);
template <typename T>
void cheb_update(const LSeg* segs, int nseg, int nj, long long maxlen, int mode, double rho, double sig, T* x, T* r,
                 T* d, const T* y, const T* dinv, const T* b, hipStream_t s);
template <typename T>
void seg_add(const LSeg* segs, int nseg, int nj, long long maxlen, const T* d, T* x, double a, hipStream_t s);
template <typename T>
void seg_zero(const LSeg* segs, int nseg, int nj, long long maxlen, T* x, hipStream_t s);
// x_j = Ainv_j b_j per segment and level j; shared = every segment's matrix is
// the same for all levels (mjstride 0): one pass over each row serves all j
template <typename T>
void dense_solve(const DSeg* segs, int nseg, int nj, int maxn, bool shared, const double* Ainv, const T* b, T* x,
                 hipStream_t s);
// In-place inversion of a batch of dense matrices (symmetric positive definite,
// or identity rows/columns plus an SPD block) by Gauss-Jordan exchange steps
// without pivoting; snap holds 4 n doubles per matrix; *bad is set to 1 if a
// pivot is zero or not finite (the caller clears it first).
void dense_invert(const GJMat* mats, int nmats, int maxn, double* A, double* snap, int* bad, hipStream_t s);

}  // namespace bt
