// 3D space-time slab operator Y = A X (or A^T X) and the 3D Q2 elasticity
// operator of the multigrid levels.
//
// u-rows (tau A u - c_p E p, section "Poroelasticity"): on the uniform box
// mesh every cell of an instance (or multigrid level) has the same element
// matrices tau A_e (81x81) and E_e (81x8).  The element products of a layer
// of cells are therefore one dense contraction
//     [tau A_e | E_e] (81 x 89)  x  [u_e ; -c_p p_e] (89 x cells),
// done on the matrix cores (16x16x4 MFMA, FP64 or FP32): twelve waves, three
// per SIMD, each keep one 16-row tile of the element matrix in registers for
// the whole launch and multiply it with one half of the layer's gathered
// element vectors staged in LDS.  The node loads of a layer are issued two
// layers ahead and stay in flight across the matrix-core phase in between
// (software pipeline).
//
// Work decomposition: one block = an xy tile of 8x8 cells (7x7 owned plus a
// one-cell halo on the low sides) marching through a z-chunk of cell layers.
// The element rows of layer k are staged in LDS and every owned node of planes
// 2k (bottom slice of layer k plus the top slice of layer k-1, carried in
// LDS) and 2k+1 (middle slice) is summed in a fixed order, in the next layer's
// first phase: deterministic, no atomics.  q-rows and p-rows are gathers (rows.h) in their own kernels:
//   q-rows: tau (Mq q + B p);   p-rows: -w [tau div q_i + sum_j T_ij (b div u_j + p_j/M)]
//   (A^T: p-rows -w [tau div q_i + tau b div u_i + sum_j T_ji p_j / M], u-rows use sum_j T_ji p_j).
#include "kernels.h"
#include "prec.h"
#include "rows.h"

namespace bt {

constexpr int kT3 = 8;        // xy tile edge in cells (64 cells per layer)
constexpr int kO3 = kT3 - 1;  // owned cells per tile edge
constexpr int kZC = 8;        // cell layers per z-chunk
constexpr int kRT3 = 6;       // 16-row tiles of the 96 padded element rows
constexpr int kW3 = 12;       // waves per block: (row tile, half of the 64 cells) each, three per SIMD
constexpr int kLD3 = 80;      // LDS row stride (elements): 16-lane groups of one half-wave hit disjoint banks

int apply3d_tile_cells_xy() { return kO3; }
// z-chunk variants of the operator apply (tile autotuner; identical results): 8, 4, 16 layers
int apply3d_variants() { return 3; }
int apply3d_tile_cells_z(int variant) { return variant == 1 ? 4 : (variant == 2 ? 16 : kZC); }

typedef double mf_d4 __attribute__((ext_vector_type(4)));
typedef float mf_f4 __attribute__((ext_vector_type(4)));

// 16x16x4 MFMA: A operand lane l holds A[l % 16][l / 16], B operand B[l / 16][l % 16];
// output value v of lane l is D[row(l, v)][l % 16].
template <typename T> struct Mfma16;
template <> struct Mfma16<double> {
  using V = mf_d4;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * v + (l >> 4); }
};
template <> struct Mfma16<float> {
  using V = mf_f4;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

template <typename T>
struct U3Job {
  int n[3], su[3];
  const T* A;        // element-matrix fragments: [wave][k-step][lane] (see elast_fragments3d)
  T cp;              // coupling weight: element rows are tau A_e u - cp E_e p
  const T* X;        // u block, components at X + c * nu1
  const T* Bv;       // residual mode right-hand side (same layout) or null
  T* Y;
  const T* P;        // pressure block of the coupling (mixed over time levels) or null
  long long plstride;  // distance between the time levels of P
  T pw[4];           // time-level weights of the coupling pressure
  int npl;
  int sp[2];
  int mode;          // 0: Y = A x (+ coupling); 1: Y = B - A x; 2: Chebyshev step (below)
  bool copy_fixed;   // mode 0, essential rows: copy x (slab operator) or 0 (multigrid level operator)
  // mode 2, with y = A d for d = X (essential rows 0): Xs += d, Rs -= y,
  // Y = rho d + sig Dv Rs (the next direction; Y must not be X)
  T* Xs;
  T* Rs;
  const T* Dv;
  T rho, sig;
};

// KS = k-steps of 4 columns: 23 with the 8 coupling columns, 21 without.
//
// Two phases per cell layer k, one barrier after each:
//   A: the node sums of layer k-1 (element rows in Rw, the carried top slice of
//      layer k-2 in Cc[k & 1]) and the carry of layer k-1's top slice into
//      Cc[(k & 1) ^ 1], then the element rows of layer k on the matrix cores
//      (gathered vectors in Ul);
//   B: the rows of layer k into Rw, the node planes of layer k+1 scattered into
//      Ul, the loads of layer k+2 issued, the right-hand side of layer k's node
//      sums (residual mode) prefetched.
// (Against one phase per step, with five barriers per layer, this is 3-5% faster
// at 48^3; letting some waves of a SIMD multiply before they sum was slower.)
template <typename T, int KS>
__device__ __forceinline__ void u3_run(const U3Job<T>& J, int i0, int j0, int k0, int zc) {
  constexpr int NC = kT3 * kT3, NT = 64 * kW3, KR = 4 * KS;
  __shared__ T Ul[KR * kLD3];     // gathered element vectors of the layer on the matrix cores [k][cell]
  __shared__ T Rw[81 * kLD3];     // element rows of the layer whose nodes are summed [comp*27 + node][cell]
  __shared__ T Cc[2][27 * NC];    // carried top slices, by layer parity [comp*9 + node][cell]
  using M = Mfma16<T>;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nx = J.n[0], ny = J.n[1], nz = J.n[2];
  const int nu1 = J.su[0] * J.su[1] * J.su[2];
  const int sy = J.su[0], sz = J.su[0] * J.su[1];
  const int kbeg = k0 > 0 ? k0 - 1 : 0;
  const int kend = min(k0 + zc, nz);
  const int mxe = (i0 + kO3 >= nx) ? 2 * nx + 1 : 2 * i0 + 2 * kO3;
  const int mye = (j0 + kO3 >= ny) ? 2 * ny + 1 : 2 * j0 + 2 * kO3;
  const int nmx = mxe - 2 * i0, nmy = mye - 2 * j0;
  const int nplane = nmx * nmy;
  // this wave's 16-row tile of the element matrix, resident for the whole launch,
  // and its half of the layer's 64 cells (column tiles 2 ch, 2 ch + 1)
  const int rt = wv % kRT3, ch = wv / kRT3;
  T af[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s) af[s] = J.A[(rt * KS + s) * 64 + lane];
  for (int idx = tid; idx < 2 * 27 * NC; idx += NT) Cc[idx / (27 * NC)][idx % (27 * NC)] = T(0);
  // node-plane gather: 3 planes x 3 components of 17 x 17 nodes per layer.  All
  // of a thread's loads are issued before the LDS scatter; their offsets (less
  // the layer term) and masks do not depend on the layer and are computed here.
  constexpr int NX = 2 * kT3 + 1, NP = NX * NX, NGA = 9 * NP;
  constexpr int NIT = (NGA + NT - 1) / NT;
  // per load: bits 0..29 the in-range offset, bit 30 = plane z 0 (bottom face at
  // k = 0), bit 31 = masked (outside the tile's node range or essential).  The
  // offset is below the size of one level's u block, which the host's limit of
  // 2^31 slab unknowns keeps under 2^30.
  unsigned gcode[NIT];
  {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = min(tid + it * NT, NGA - 1);
      const int cz = idx / NP;                 // comp * 3 + plane
      const int r = idx - cz * NP;
      const int c2 = cz / 3, z = cz - 3 * c2;
      const int ny_ = r / NX, nx_ = r - NX * ny_;
      const int mx = 2 * (i0 - 1) + nx_, my = 2 * (j0 - 1) + ny_;
      const int mxc = min(max(mx, 0), J.su[0] - 1), myc = min(max(my, 0), J.su[1] - 1);
      // in the tile's node range and not on an essential lateral face (mz = 1 is never the bottom)
      const bool ok = tid + it * NT < NGA && mx >= 0 && mx < J.su[0] && my >= 0 && my < J.su[1] &&
                      !ugrid_fixed(3, J.su, c2, mx, my, 1);
      gcode[it] = (unsigned)(c2 * nu1 + mxc + sy * myc + sz * z) | (z == 0 ? 1u << 30 : 0u) | (ok ? 0u : 1u << 31);
    }
  }

  T gv[NIT];
  // ---- the element vectors of layer k into Ul: the three node planes 2k..2k+2
  // of the tile (17 x 17 nodes per plane and component, loaded into gv, read
  // once, coalesced along x); every node is written to the element-vector slot
  // of each cell that shares it (essential u masked).  Cells outside the mesh get
  // partial vectors; their rows are never summed into an owned node.  Then the
  // coupling columns (scaled mixed pressure at the cell's Gauss points) and padding.
  auto scatter_layer = [&](int k) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      // bottom face (plane mz = 0) is essential for every component
      const unsigned g = gcode[it];
      const bool in = !(g >> 31) && !(k == 0 && ((g >> 30) & 1u));
      gv[it] = in ? gv[it] : T(0);
    }
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
      const int idx = tid + it * NT;
      if (idx >= NGA) break;
      const int cz = idx / NP;
      const int r = idx - cz * NP;
      const int c2 = cz / 3, z = cz - 3 * c2;
      const int ny_ = r / NX, nx_ = r - NX * ny_;
      const T v = gv[it];
      // cells of the tile sharing the node along x and y (local node a, b)
#pragma unroll
      for (int sj = 0; sj < 2; ++sj) {
        int ly, b;
        if (ny_ & 1) { if (sj) break; ly = ny_ >> 1; b = 1; }
        else { ly = (ny_ >> 1) - sj; b = sj ? 2 : 0; if (ly < 0 || ly >= kT3) continue; }
#pragma unroll
        for (int si = 0; si < 2; ++si) {
          int lx, a;
          if (nx_ & 1) { if (si) break; lx = nx_ >> 1; a = 1; }
          else { lx = (nx_ >> 1) - si; a = si ? 2 : 0; if (lx < 0 || lx >= kT3) continue; }
          Ul[(c2 * 27 + z * 9 + b * 3 + a) * kLD3 + ly * kT3 + lx] = v;
        }
      }
    }
    for (int idx = tid; idx < (KR - 81) * NC; idx += NT) {
      const int kr = 81 + (idx >> 6), cell = idx & 63;
      const int i = i0 - 1 + (cell & 7), j = j0 - 1 + (cell >> 3);
      T v = 0;
      if (kr < 89 && J.npl > 0 && i >= 0 && i < nx && j >= 0 && j < ny) {
        const int g = kr - 81;
        const long long o = (2 * i + (g & 1)) + (long long)J.sp[0] *
                            ((2 * j + ((g >> 1) & 1)) + (long long)J.sp[1] * (2 * k + (g >> 2)));
        T s = 0;
        for (int l = 0; l < J.npl; ++l) s += J.pw[l] * J.P[l * J.plstride + o];
        v = -J.cp * s;
      }
      Ul[kr * kLD3 + cell] = v;
    }
  };
  // the node loads of layer k (in flight until the scatter that consumes them)
  auto load_layer = [&](int k) {
#pragma unroll
    for (int it = 0; it < NIT; ++it) gv[it] = J.X[(int)(gcode[it] & 0x3fffffffu) + sz * (2 * k)];
  };

  // ---- owned node planes 2k (bottom slice of Rw + carried top slice cb) and 2k+1
  // FP64 residual mode and Chebyshev step: the values of the owned nodes that the
  // sums need are prefetched into pf (residual: the right-hand side; Chebyshev
  // step: d, x, r, Dinv); FP32 keeps the single loop, as for the gather
  constexpr int NOW = sizeof(T) == 8 ? (6 * (2 * kO3 + 1) * (2 * kO3 + 1) + NT - 1) / NT : 1;
  T pf[4][NOW];
  auto prefetch_nodes = [&](int k) {
    if (sizeof(T) == 8 && J.mode != 0) {
#pragma unroll
      for (int it = 0; it < NOW; ++it) {
        const int idx = min(tid + it * NT, 6 * nplane - 1);
        const int c = idx / (2 * nplane);
        const int rem = idx - c * 2 * nplane;
        const int zl = rem >= nplane;
        const int r2 = rem - zl * nplane;
        const int go = c * nu1 + (2 * i0 + r2 % nmx) + sy * (2 * j0 + r2 / nmx) + sz * (2 * k + zl);
        if (J.mode == 1) {
          pf[0][it] = J.Bv[go];
        } else {
          pf[0][it] = J.X[go];
          pf[1][it] = J.Xs[go];
          pf[2][it] = J.Rs[go];
          pf[3][it] = J.Dv[go];
        }
      }
    }
  };
  // the result v of an owned node (y = A x of mode 0 and 2, b - A x of mode 1)
  auto store_node = [&](int go, T v, int it) {
    if (J.mode != 2) {
      J.Y[go] = v;
      return;
    }
    const bool pre = sizeof(T) == 8;
    const T dd = pre ? pf[0][it] : J.X[go];
    const T rr = (pre ? pf[2][it] : J.Rs[go]) - v;
    J.Xs[go] = (pre ? pf[1][it] : J.Xs[go]) + dd;
    J.Rs[go] = rr;
    J.Y[go] = J.rho * dd + J.sig * (pre ? pf[3][it] : J.Dv[go]) * rr;
  };
  auto node_sums = [&](int k, const T* __restrict__ cb) {
#pragma unroll
    for (int it = 0; it < NOW; ++it)
    for (int idx = tid + it * NT; idx < 6 * nplane; idx += (sizeof(T) == 8 ? 6 * nplane : NT)) {
      const int c = idx / (2 * nplane);
      const int rem = idx - c * 2 * nplane;
      const int zl = rem >= nplane;
      const int r2 = rem - zl * nplane;
      const int mx = 2 * i0 + r2 % nmx, my = 2 * j0 + r2 / nmx, mz = 2 * k + zl;
      const int go = c * nu1 + mx + sy * my + sz * mz;
      T v;
      if (ugrid_fixed(3, J.su, c, mx, my, mz)) {
        v = J.mode == 1 ? (sizeof(T) == 8 ? pf[0][it] : J.Bv[go]) : (J.copy_fixed ? J.X[go] : T(0));
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
          const int cell = (ty0 + qy) * kT3 + tx0 + qx;
          const int nd = (qy ? 0 : ay0) * 3 + (qx ? 0 : ax0);
          v += Rw[(c * 27 + zl * 9 + nd) * kLD3 + cell];
          if (zl == 0) v += cb[(c * 9 + nd) * NC + cell];
        }
        if (J.mode == 1) v = (sizeof(T) == 8 ? pf[0][it] : J.Bv[go]) - v;
      }
      store_node(go, v, it);
    }
  };
  // top slice of the rows in Rw (comp * 9 + node) into the carry buffer cn
  auto carry = [&](T* __restrict__ cn) {
    for (int idx = tid; idx < 27 * NC; idx += NT) {
      const int r = idx >> 6, cell = idx & 63;
      const int c = r / 9;
      cn[idx] = Rw[(c * 27 + 18 + (r - 9 * c)) * kLD3 + cell];
    }
  };
  // phase A of the layer below (its node sums when owned, and its carry)
  auto finish_below = [&](int k) {
    if (k > kbeg) {
      if (k - 1 >= k0) node_sums(k - 1, Cc[k & 1]);
      carry(Cc[(k & 1) ^ 1]);
    }
  };

  // prologue: layer kbeg gathered into Ul, the loads of layer kbeg + 1 in flight
  load_layer(kbeg);
  scatter_layer(kbeg);
  load_layer(kbeg + 1 < kend ? kbeg + 1 : kbeg);
  __syncthreads();
  for (int k = kbeg; k < kend; ++k) {
    // ---- phase A: the layer below; element rows of layer k: rows of tile rt x cells 32 ch .. 32 ch + 31
    finish_below(k);
    typename M::V acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) acc[t] = typename M::V{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const T* Bs = Ul + (4 * s + (lane >> 4)) * kLD3 + 32 * ch + (lane & 15);
#pragma unroll
      for (int t = 0; t < 2; ++t) acc[t] = M::mma(af[s], Bs[16 * t], acc[t]);
    }
    __syncthreads();
    // ---- phase B: rows of layer k into Rw; layer k+1 into Ul, loads of layer k+2
    {
      const int c = rt >> 1, h = rt & 1;
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int pr = 16 * h + M::row(lane, v);
          if (pr < 27) Rw[(c * 27 + pr) * kLD3 + 32 * ch + 16 * t + (lane & 15)] = acc[t][v];
        }
    }
    if (k + 1 < kend) {
      scatter_layer(k + 1);
      // (the last layer re-reads its own planes: in range, unused)
      load_layer(k + 2 < kend ? k + 2 : k + 1);
    }
    if (k >= k0) prefetch_nodes(k);
    __syncthreads();
  }
  // the last layer's node sums and carry
  finish_below(kend);
  __syncthreads();
  // ---- top plane 2 nz (only the layer below contributes)
  if (kend == nz) {
    const T* cb = Cc[(kend & 1) ^ 1];
    for (int idx = tid; idx < 3 * nplane; idx += NT) {
      const int c = idx / nplane;
      const int r2 = idx - c * nplane;
      const int mx = 2 * i0 + r2 % nmx, my = 2 * j0 + r2 / nmx, mz = 2 * nz;
      const int go = c * nu1 + mx + sy * my + sz * mz;
      T v;
      if (ugrid_fixed(3, J.su, c, mx, my, mz)) {
        v = J.mode == 1 ? J.Bv[go] : (J.copy_fixed ? J.X[go] : T(0));
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
          const int cell = (ty0 + qy) * kT3 + tx0 + qx;
          v += cb[(c * 9 + (qy ? 0 : ay0) * 3 + (qx ? 0 : ax0)) * NC + cell];
        }
        if (J.mode == 1) v = J.Bv[go] - v;
      }
      if (J.mode == 2) {
        const T dd = J.X[go];
        const T rr = J.Rs[go] - v;
        J.Xs[go] += dd;
        J.Rs[go] = rr;
        J.Y[go] = J.rho * dd + J.sig * J.Dv[go] * rr;
      } else {
        J.Y[go] = v;
      }
    }
  }
}

// operator apply: u-rows of time level blockIdx.y
template <typename T, int NL, bool TR>
__global__ __launch_bounds__(64 * kW3) void apply3d_u_kernel(const InstDev* __restrict__ insts,
                                                             const int4* __restrict__ work, int zc, TimeMat tm,
                                                             const T* __restrict__ emat, const T* __restrict__ X,
                                                             T* __restrict__ Y) {
  const int4 w = work[blockIdx.x];
  const InstDev& I = insts[w.x];
  const int lev = blockIdx.y;
  U3Job<T> J;
  for (int e = 0; e < 3; ++e) { J.n[e] = I.n[e]; J.su[e] = I.su[e]; }
  J.A = emat + I.emat_off;
  J.X = X + I.x_off + lev * I.N + I.off_u[0];
  J.Y = Y + I.x_off + lev * I.N + I.off_u[0];
  J.Bv = nullptr;
  J.mode = 0;
  J.copy_fixed = true;
  J.P = X + I.x_off + I.off_p;
  J.plstride = I.N;
  J.sp[0] = I.sp[0]; J.sp[1] = I.sp[1];
  for (int l = 0; l < 4; ++l) J.pw[l] = T(0);
  if (!TR) {
    // forward: the coupling uses the pressure of the same level only
    J.P += lev * I.N;
    J.npl = 1;
    J.pw[0] = T(1);
    J.cp = T(I.tau * I.b);
  } else {
    J.npl = NL;
    for (int l = 0; l < NL; ++l) J.pw[l] = T(tm.T[l * 4 + lev]);
    J.cp = T(I.b);
  }
  u3_run<T, 23>(J, w.y * kO3, w.z * kO3, w.w * zc, zc);
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
  const int q0 = (int)I.off_q[0], q1 = (int)I.off_p;
  for (int t = q0 + blockIdx.x * blockDim.x + threadIdx.x; t < q1; t += gridDim.x * blockDim.x) {
    int blk, comp, co[3];
    decode_dof(I, t, blk, comp, co);
    if (q_fixed(I, comp, co[comp])) { Yl[t] = Xl[t]; continue; }
    T mq, dg, bp;
    flux_row<T>(I, kc, Xl, comp, co, t - (int)I.off_q[comp], mq, dg, bp);
    Yl[t] = mq + T(I.tau) * bp;
  }
}

// p-rows in two passes (few live registers per thread):
//  pass 1, one thread per (cell, level l):
//    forward:    Y_l(p) = b div u_l + p_l / M           (zeta_l, staged in Y)
//    transposed: Y_l(p) = -w tau (div q_l + b div u_l)
//  pass 2, one thread per cell, all levels:
//    forward:    Y_l(p) = -w (tau div q_l + sum_j T_lj zeta_j)
//    transposed: Y_l(p) += -w sum_j T_jl p_j / M
template <typename T, bool TR, int DIM>
__global__ __launch_bounds__(256) void prows_local_kernel(const InstDev* __restrict__ insts, const T* __restrict__ X,
                                                          T* __restrict__ Y) {
  constexpr int NG = 1 << DIM;
  const InstDev& I = insts[blockIdx.y];
  const int l = blockIdx.z;
  const int nc = (int)I.ncells;
  const unsigned n0 = I.n[0], n1 = I.n[1];
  const T* Xl = X + I.x_off + l * I.N;
  T* Yl = Y + I.x_off + l * I.N;
  const T w = T(DIM == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]);
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < nc; cell += gridDim.x * blockDim.x) {
    const unsigned q = (unsigned)cell / n0;
    const int ce[3] = {(int)((unsigned)cell - q * n0), (int)(q % n1), DIM == 3 ? (int)(q / n1) : 0};
    const int pb = (int)I.off_p + 2 * ce[0] + I.sp[0] * (2 * ce[1] + I.sp[1] * (DIM == 3 ? 2 * ce[2] : 0));
    T du[NG];
    cell_divu<T, DIM>(I, Xl, ce, du);
    if (!TR) {
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const int o = pb + (g & 1) + I.sp[0] * (((g >> 1) & 1) + I.sp[1] * ((g >> 2) & 1));
        Yl[o] = T(I.b) * du[g] + T(I.Minv) * Xl[o];
      }
    } else {
      T dq[NG];
      cell_divq<T, DIM>(I, Xl, ce, dq);
#pragma unroll
      for (int g = 0; g < NG; ++g) {
        const int o = pb + (g & 1) + I.sp[0] * (((g >> 1) & 1) + I.sp[1] * ((g >> 2) & 1));
        Yl[o] = -w * T(I.tau) * (dq[g] + T(I.b) * du[g]);
      }
    }
  }
}

template <typename T, int NL, bool TR, int DIM>
__global__ __launch_bounds__(256) void prows_mix_kernel(const InstDev* __restrict__ insts, TimeMat tm,
                                                        const T* __restrict__ X, T* __restrict__ Y) {
  constexpr int NG = 1 << DIM;
  const InstDev& I = insts[blockIdx.y];
  const int nc = (int)I.ncells;
  const unsigned n0 = I.n[0], n1 = I.n[1];
  const T w = T(DIM == 3 ? 0.125 * I.h[0] * I.h[1] * I.h[2] : 0.25 * I.h[0] * I.h[1]);
  for (int cell = blockIdx.x * blockDim.x + threadIdx.x; cell < nc; cell += gridDim.x * blockDim.x) {
    const unsigned q = (unsigned)cell / n0;
    const int ce[3] = {(int)((unsigned)cell - q * n0), (int)(q % n1), DIM == 3 ? (int)(q / n1) : 0};
    const int pb = (int)I.off_p + 2 * ce[0] + I.sp[0] * (2 * ce[1] + I.sp[1] * (DIM == 3 ? 2 * ce[2] : 0));
    int po[NG];
#pragma unroll
    for (int g = 0; g < NG; ++g) po[g] = pb + (g & 1) + I.sp[0] * (((g >> 1) & 1) + I.sp[1] * ((g >> 2) & 1));
    T v[NL][NG];   // forward: zeta_j; transposed: p_j / M
#pragma unroll
    for (int j = 0; j < NL; ++j)
#pragma unroll
      for (int g = 0; g < NG; ++g)
        v[j][g] = TR ? T(I.Minv) * X[I.x_off + j * I.N + po[g]] : Y[I.x_off + j * I.N + po[g]];
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      T* Yl = Y + I.x_off + l * I.N;
      if (!TR) {
        T dq[NG];
        cell_divq<T, DIM>(I, X + I.x_off + l * I.N, ce, dq);
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          T s = T(I.tau) * dq[g];
#pragma unroll
          for (int j = 0; j < NL; ++j) s += T(tm.T[l * 4 + j]) * v[j][g];
          Yl[po[g]] = -w * s;
        }
      } else {
#pragma unroll
        for (int g = 0; g < NG; ++g) {
          T s = 0;
#pragma unroll
          for (int j = 0; j < NL; ++j) s += T(tm.T[j * 4 + l]) * v[j][g];
          Yl[po[g]] += -w * s;
        }
      }
    }
  }
}

static dim3 g3(long long maxlen, int count, int nj) {
  long long b = (maxlen + kBlk - 1) / kBlk;
  return dim3((unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b)), count, nj);
}

template <typename T, int NL>
static void apply3d_nl(const ApplyArgs& a, const void* x, void* y, int tr, long long maxN, long long maxc, int count) {
  const T* X = (const T*)x;
  T* Y = (T*)y;
  const T* em = (const T*)a.emat;
  if (tr)
    hipLaunchKernelGGL((apply3d_u_kernel<T, NL, true>), dim3(a.nwork, NL), dim3(64 * kW3), 0, a.stream, a.inst,
                       a.work, apply3d_tile_cells_z(a.variant), *a.tm, em, X, Y);
  else
    hipLaunchKernelGGL((apply3d_u_kernel<T, NL, false>), dim3(a.nwork, NL), dim3(64 * kW3), 0, a.stream, a.inst,
                       a.work, apply3d_tile_cells_z(a.variant), *a.tm, em, X, Y);
  hipLaunchKernelGGL((qrows_kernel<T>), g3(maxN, count, NL), dim3(kBlk), 0, a.stream, a.inst, (const T*)a.kinv, X, Y);
  if (tr) {
    hipLaunchKernelGGL((prows_local_kernel<T, true, 3>), g3(maxc, count, NL), dim3(kBlk), 0, a.stream, a.inst, X, Y);
    hipLaunchKernelGGL((prows_mix_kernel<T, NL, true, 3>), g3(maxc, count, 1), dim3(kBlk), 0, a.stream, a.inst, *a.tm,
                       X, Y);
  } else {
    hipLaunchKernelGGL((prows_local_kernel<T, false, 3>), g3(maxc, count, NL), dim3(kBlk), 0, a.stream, a.inst, X, Y);
    hipLaunchKernelGGL((prows_mix_kernel<T, NL, false, 3>), g3(maxc, count, 1), dim3(kBlk), 0, a.stream, a.inst,
                       *a.tm, X, Y);
  }
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

// elasticity multigrid level: y = tau A x (mode 0; essential rows 0), y = b - tau A x
// (mode 1; essential rows b), or one Chebyshev step with the operator applied to the
// direction d = x (mode 2: xs += d, rs -= tau A d, y = rho d + sig Dinv rs)
template <typename T>
__global__ __launch_bounds__(64 * kW3) void uapply3d_kernel(const UGridSeg* __restrict__ segs,
                                                            const int4* __restrict__ work, int zc, int mode,
                                                            const T* __restrict__ emat, const T* __restrict__ X,
                                                            const T* __restrict__ Bv, T* __restrict__ Y,
                                                            T* __restrict__ Xs, T* __restrict__ Rs,
                                                            const T* __restrict__ dinv, double rho, double sig) {
  const int4 w = work[blockIdx.x];
  const UGridSeg& G = segs[w.x];
  const long long vo = G.voff + blockIdx.y * G.vjstride;
  U3Job<T> J;
  for (int e = 0; e < 3; ++e) { J.n[e] = G.n[e]; J.su[e] = G.su[e]; }
  J.A = emat + G.emat_off;
  J.cp = T(0);
  J.X = X + vo;
  J.Y = Y + vo;
  J.Bv = Bv ? Bv + vo : nullptr;
  J.mode = mode;
  J.copy_fixed = false;
  J.P = nullptr;
  J.plstride = 0;
  J.npl = 0;
  J.sp[0] = 1; J.sp[1] = 1;
  for (int l = 0; l < 4; ++l) J.pw[l] = T(0);
  J.Xs = Xs ? Xs + vo : nullptr;
  J.Rs = Rs ? Rs + vo : nullptr;
  J.Dv = dinv ? dinv + G.doff : nullptr;
  J.rho = T(rho);
  J.sig = T(sig);
  u3_run<T, 21>(J, w.y * kO3, w.z * kO3, w.w * zc, zc);
}
template <typename T>
void launch_uapply3d(const UGridSeg* segs, const int4* work, int nwork, int nj, int zc, int mode, const T* x,
                     const T* b, T* y, const T* emat, hipStream_t s) {
  hipLaunchKernelGGL((uapply3d_kernel<T>), dim3(nwork, nj), dim3(64 * kW3), 0, s, segs, work, zc, mode, emat, x, b,
                     y, (T*)nullptr, (T*)nullptr, (const T*)nullptr, 0.0, 0.0);
}
template <typename T>
void launch_uapply3d_cheb(const UGridSeg* segs, const int4* work, int nwork, int nj, int zc, const T* d, T* x, T* r,
                          T* dnext, const T* dinv, double rho, double sig, const T* emat, hipStream_t s) {
  hipLaunchKernelGGL((uapply3d_kernel<T>), dim3(nwork, nj), dim3(64 * kW3), 0, s, segs, work, zc, 2, emat, d,
                     (const T*)nullptr, dnext, x, r, dinv, rho, sig);
}
template void launch_uapply3d<double>(const UGridSeg*, const int4*, int, int, int, int, const double*, const double*,
                                      double*, const double*, hipStream_t);
template void launch_uapply3d<float>(const UGridSeg*, const int4*, int, int, int, int, const float*, const float*,
                                     float*, const float*, hipStream_t);
template void launch_uapply3d_cheb<double>(const UGridSeg*, const int4*, int, int, int, const double*, double*, double*,
                                           double*, const double*, double, double, const double*, hipStream_t);
template void launch_uapply3d_cheb<float>(const UGridSeg*, const int4*, int, int, int, const float*, float*, float*,
                                          float*, const float*, double, double, const float*, hipStream_t);

}  // namespace bt
