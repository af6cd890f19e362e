// Preconditioner kernels: level descriptors and launchers (prec_*.hip).
//
// Section "Preconditioning technology": GMRES is preconditioned level-blockwise
// (the L_j blocks of the real block form of the temporal matrix, couplings
// dropped) by a truncated fixed-stress split of every L_j:
//   p = -S_j^-1 r_p,          S_j = alpha_j (1/M + L) Mp + tau B^T diag(Mq)^-1 B
//   q = (tau Mq)^-1 (r_q - tau B p)
//   u = (tau A)^-1 (r_u + b tau E p)
// with inexact inner solves: an aggregation multigrid V-cycle for S_j, a
// Chebyshev-Jacobi polynomial for Mq, a geometric Q2 multigrid V-cycle for A.
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"
#include "vec.h"

namespace bt {

// Chebyshev modes of the fused stencil kernels
enum ChebMode { kResInit = 0, kResInitZero = 1, kStep = 2, kApplyDinv = 3 };

struct ChebCoef {      // one launch: init scale or step coefficients
  double s0;           // init: d = s0 Dinv r
  double rho, sig;     // step: d_out = rho d_in + sig Dinv r
  double bsign;        // init: r = bsign * b (- S x)
};

// complex-pair level blocks: Q^-1 T Q = [[alpha, beta], [-beta, alpha]] on the
// levels (j, j2) of a pair, beta > 0 (pairs.hip)
struct PairSet {
  int n;               // number of pairs (0..2)
  int j[2];            // first level of each pair
  int j2[2];           // its second level
  double beta[2];
};
// transpose selects the block of the slab transpose in the basis Q^-T
template <typename T>
void launch_pair_split(const InstDev* insts, int count, long long maxN, const PairSet& ps, int transpose, T* r,
                       hipStream_t s);
template <typename T>
void launch_pair_couple(int dim, const InstDev* insts, int count, long long maxN, const PairSet& ps, int transpose,
                        const T* z, T* save, T* r, hipStream_t s);
template <typename T>
void launch_pair_join(const InstDev* insts, int count, long long maxN, const PairSet& ps, int transpose, const T* save,
                      T* z, hipStream_t s);

// fixed-stress sub-systems (fixed_stress.hip): y += -L Mp (T p) on the p-rows with the
// u-rows cleared; zero_rows clears the u-rows (which = 0) or the q- and p-rows (1)
template <typename T>
void launch_fs_flow_fix(const InstDev* insts, int count, long long maxN, int nl, const TimeMat& tm, const T* x, T* y,
                        hipStream_t s);
template <typename T>
void launch_zero_rows(const InstDev* insts, int count, long long maxN, int nl, int which, T* y, hipStream_t s);


// pressure Schur, fine DG level: one segment per instance (all time levels)
struct PDgSeg {
  int inst;            // index into InstDev table
  int pad;
  long long voff, vjstride;    // work vectors (slab layout): p-block of level j
  long long dqoff;             // Dq^-1 (state layout) of this instance
  long long doff, djstride;    // Dinv of S_j (normalised), per time level
  double cm[4];                // alpha_j (1/M + L) for each time level
  InstDev I;                   // copy of the instance descriptor (one indirection less per launch)
};
// pressure Schur, cell levels
struct PCellSeg {
  int n[3];
  int dim;
  long long ncells;
  long long voff, vjstride;    // work vectors [inst][j][cell]
  long long coff;              // coefficient block: 5 * ncells (t0, t1, t2, ttop, m)
  long long doff, djstride;
  double cm[4];
};

template <typename T>
void launch_pdg(int dim, const InstDev* insts, const PDgSeg* segs, int nseg, int nj, long long maxnp, int mode,
                ChebCoef cc, const T* dqinv, const T* dinv, const T* b, T* x, T* r, const T* din, T* dout,
                hipStream_t s);
void launch_pdg_diag(int dim, const InstDev* insts, const PDgSeg* segs, int nseg, int nj, long long maxnp,
                     const double* dqinv, double* dinv, hipStream_t s);
template <typename T>
void launch_pcell(const PCellSeg* segs, int nseg, int nj, long long maxc, int mode, ChebCoef cc, const T* coef,
                  const T* dinv, const T* b, T* x, T* r, const T* din, T* dout, hipStream_t s);
void launch_pcell_diag(const PCellSeg* segs, int nseg, int nj, long long maxc, const double* coef, double* dinv,
                       hipStream_t s);
// Galerkin coefficients: level 1 from Dq^-1, coarser levels by aggregation
void launch_pcoef_first(const InstDev* insts, const PDgSeg* fine, const PCellSeg* lev1, int nseg, long long maxc,
                        const double* dqinv, double* coef, hipStream_t s);
void launch_pcoef_coarsen(const PCellSeg* fine, const PCellSeg* coarse, int nseg, long long maxc, const double* coef_f,
                          double* coef_c, hipStream_t s);
// transfers: restrict residual (sum over children), prolongate correction (x += w e)
template <typename T>
void launch_p_restrict_dg(const InstDev* insts, const PDgSeg* fine, const PCellSeg* coarse, int nseg, int nj,
                          long long maxc, const T* r, T* b, hipStream_t s);
template <typename T>
void launch_p_prolong_dg(const InstDev* insts, const PDgSeg* fine, const PCellSeg* coarse, int nseg, int nj,
                         long long maxnp, double w, const T* e, T* x, hipStream_t s);
template <typename T>
void launch_p_restrict_cell(const PCellSeg* fine, const PCellSeg* coarse, int nseg, int nj, long long maxc,
                            const T* r, T* b, hipStream_t s);
template <typename T>
void launch_p_prolong_cell(const PCellSeg* fine, const PCellSeg* coarse, int nseg, int nj, long long maxc, double w,
                           const T* e, T* x, hipStream_t s);

// Dq (diagonal of the flux mass with K) inverse, 0 on essential flux DoFs
void launch_dq(const InstDev* insts, int count, long long maxN, const double* kinv, double* dqinv, hipStream_t s);

// flux block: coupling right-hand sides from p, and tau Mq Chebyshev
// per time level coefficient of the displacement right-hand side f_u = r_u + c_j b E p
// (c_j = tau for L_j, c_j = the level shift for L_j^T)
struct LevelCoef { double c[4]; };
template <typename T>
void launch_coupling(int dim, const InstDev* insts, int count, int nj, long long maxN, const LevelCoef& cu,
                     const T* rt, const T* zp, T* fu, T* fq, hipStream_t s);
template <typename T>
void launch_mq(int dim, const InstDev* insts, int count, int nj, long long maxN, int mode, ChebCoef cc,
               const T* kinv, const T* dinvq, const T* b, T* x, T* r, const T* din, T* dout, hipStream_t s);

// elasticity multigrid levels
struct UGridSeg {
  int dim;
  int n[3];
  int su[3];
  int pad;
  double h[3];
  double tau, lam, mu;
  long long voff, vjstride;    // u block of time level j: voff + j*vjstride, components contiguous
  long long doff;              // Dinv (normalised), shared by all time levels
  long long nu;                // dim * prod(su)
  long long emat_off;          // tau*A_e of the level (2D 18x18; 3D matrix-core fragments)
};
// one separable restriction pass along `axis` (input dims din -> output dims dout)
struct RPass {
  int dim, axis, width, last;  // width: pairs per coarse node; last: mask essential rows of the output grid
  int din[3], dout[3];
  long long ioff, ijstride, ooff, ojstride;
  long long tab;               // restriction table: per output coordinate along axis: width (fine, weight) pairs
};
// prolongation fine <- coarse (tensor product of 1D interpolation)
struct UProl {
  int dim, pad;
  int sf[3], sc[3];            // fine / coarse nodal sizes
  long long foff, fjstride, coff, cjstride;
  long long tab[3];            // per axis: per fine node (coarse cell, w0, w1, w2)
};
// 2D: variant 0 = 16x16-thread tiles, 1 = 8x8 (owned cells per tile edge:
// uapply_tile(2, variant)); 3D: the variant is the z-chunk (cell layers per block)
template <typename T>
void launch_uapply(int dim, const UGridSeg* segs, const int4* work, int nwork, int nj, int mode, const T* x,
                   const T* b, T* y, const T* emat, hipStream_t s, int variant);
int uapply_tile(int dim, int variant);
// exact line solve of tau Mq x = b (q blocks of every level; w: q-sized scratch).
// maxcells_line = the largest cell count along any axis of any instance: lines
// of up to kPcrMaxCells cells are solved by one wavefront each (parallel cyclic
// reduction), longer lines by one thread each (Thomas sweep).
constexpr int kPcrMaxCells = 511;
template <typename T>
void launch_mq_lines(int dim, const InstDev* insts, int count, int nj, long long maxlines, int maxcells_line,
                     const T* kinv, const T* b, T* x, T* w, hipStream_t s);
template <typename T>
void launch_uapply3d(const UGridSeg* segs, const int4* work, int nwork, int nj, int zc, int mode, const T* x,
                     const T* b, T* y, const T* emat, hipStream_t s);
// one Chebyshev step of the 3D elasticity smoother with its operator product in the same
// sweep: x += d, r -= tau A d, dnext = rho d + sig Dinv r (dnext must not be d)
template <typename T>
void launch_uapply3d_cheb(const UGridSeg* segs, const int4* work, int nwork, int nj, int zc, const T* d, T* x, T* r,
                          T* dnext, const T* dinv, double rho, double sig, const T* emat, hipStream_t s);
template <typename T>
void launch_rpass(const RPass* segs, int nseg, int nj, long long maxout, const double* tab, const T* in, T* out,
                  hipStream_t s);
template <typename T>
void launch_uprolong(const UProl* segs, int nseg, int nj, long long maxfine, const double* tab, const T* e, T* x,
                     hipStream_t s);
template <typename T>
void launch_mul_dinv(const LSeg* segs, int nseg, int nj, long long maxlen, const T* dinv, const T* x, T* y,
                     hipStream_t s);

// finalize: z = (Q kron I) zt on free DoFs, z = r on essential DoFs
template <typename T>
void launch_prec_finalize(const InstDev* insts, int count, long long maxN, int nl, const Mat4& Q, const T* zt,
                          const T* r, T* z, hipStream_t s);

}  // namespace bt
