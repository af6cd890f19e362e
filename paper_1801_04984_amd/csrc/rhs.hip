// Slab right-hand side (section "Discretisation in Time", dG jump term):
//   rhs_i = tau F(t_start + tau s_i) + g_i M_t X^-,   essential rows 0.
// F: compressive top traction -sigma(t) on the vertical displacement of the
// top face, int_top phi_node = prod_e h_e w(m_e) with the Simpson-type
// weights of the closed quadratic basis (1/6 at a boundary vertex, 1/3 at an
// interior vertex shared by two cells, 2/3 at an edge mid node).
// M_t X^- is non-zero only in the p-rows, where it is the Gauss-2 point
// value -w (b div u^- + p^-/M) (exact, see the operator kernels).
#include "kernels_aux.h"

namespace bt {

__device__ __forceinline__ double sigma_of_t(const InstDev& I, double t) {
  if (I.load_kind == 0) return t > 0.0 ? I.s0 : 0.0;
  double s = t / I.t_ramp;
  s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
  return I.s0 * s;
}

__device__ __forceinline__ double face_w(int m, int n) {
  if (m & 1) return 2.0 / 3.0;
  return (m == 0 || m == 2 * n) ? 1.0 / 6.0 : 1.0 / 3.0;
}

// div u of the state at the Gauss-2 points of cell (i,j,k); out[gz][gy][gx]
__device__ void divu_cell(const InstDev& I, const double* S, int i, int j, int k, double out[2][2][2]) {
  const int d = I.dim;
  for (int g = 0; g < 8; ++g) out[g >> 2][(g >> 1) & 1][g & 1] = 0.0;
  const int nz = d == 3 ? 3 : 1;
  for (int c = 0; c < d; ++c) {
    const double ih = 1.0 / I.h[c];
    for (int az = 0; az < nz; ++az)
      for (int ay = 0; ay < 3; ++ay)
        for (int ax = 0; ax < 3; ++ax) {
          const int mx = 2 * i + ax, my = 2 * j + ay, mz = d == 3 ? 2 * k + az : 0;
          if (u_fixed(I, c, mx, my, mz)) continue;
          const double v = S[I.off_u[c] + mx + (long long)I.su[0] * (my + (long long)I.su[1] * mz)];
          for (int gz = 0; gz < (d == 3 ? 2 : 1); ++gz)
            for (int gy = 0; gy < 2; ++gy)
              for (int gx = 0; gx < 2; ++gx) {
                double fx = c == 0 ? DG(gx, ax) : VG(gx, ax);
                double fy = c == 1 ? DG(gy, ay) : VG(gy, ay);
                double fz = d == 3 ? (c == 2 ? DG(gz, az) : VG(gz, az)) : 1.0;
                out[gz][gy][gx] += ih * fx * fy * fz * v;
              }
        }
  }
}

__global__ void rhs_kernel(const InstDev* __restrict__ insts, TimeMat tm, int nl, double t_start,
                           const double* __restrict__ state, double* __restrict__ rhs) {
  const InstDev& I = insts[blockIdx.y];
  const long long cell = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= I.ncells) return;
  const int d = I.dim;
  const int i = cell % I.n[0];
  const int j = (cell / I.n[0]) % I.n[1];
  const int k = d == 3 ? (int)(cell / ((long long)I.n[0] * I.n[1])) : 0;
  const double* S = state + I.state_off;
  double* R = rhs + I.x_off;
  double du[2][2][2];
  divu_cell(I, S, i, j, k, du);
  double w = I.h[0] * I.h[1] * 0.25;
  if (d == 3) w *= I.h[2] * 0.5;
  const int ngz = d == 3 ? 2 : 1;
  for (int gz = 0; gz < ngz; ++gz)
    for (int gy = 0; gy < 2; ++gy)
      for (int gx = 0; gx < 2; ++gx) {
        const long long po = I.off_p + (2 * i + gx) + (long long)I.sp[0] * ((2 * j + gy) + (long long)I.sp[1] * (d == 3 ? 2 * k + gz : 0));
        const double zeta = I.b * du[gz][gy][gx] + I.Minv * S[po];
        for (int l = 0; l < nl; ++l) R[l * I.N + po] = -w * tm.g[l] * zeta;
      }
  // top traction on the vertical displacement component (never essential on top)
  const int top_axis = d - 1;
  const bool top = (d == 2) ? (j == I.n[1] - 1) : (k == I.n[2] - 1);
  if (!top) return;
  const int nax = (i == I.n[0] - 1) ? 3 : 2;
  const int nay = (d == 3) ? ((j == I.n[1] - 1) ? 3 : 2) : 1;
  for (int ay = 0; ay < nay; ++ay)
    for (int ax = 0; ax < nax; ++ax) {
      const int mx = 2 * i + ax;
      double wf = I.h[0] * face_w(mx, I.n[0]);
      long long o;
      if (d == 2) {
        o = I.off_u[1] + mx + (long long)I.su[0] * (2 * I.n[1]);
      } else {
        const int my = 2 * j + ay;
        wf *= I.h[1] * face_w(my, I.n[1]);
        o = I.off_u[2] + mx + (long long)I.su[0] * (my + (long long)I.su[1] * (2 * I.n[2]));
      }
      for (int l = 0; l < nl; ++l) R[l * I.N + o] = -I.tau * sigma_of_t(I, t_start + I.tau * tm.s[l]) * wf;
    }
  (void)top_axis;
}

void launch_rhs(const InstDev* d_inst, int count, long long max_cells, const TimeMat& tm, int nl, double t_start,
                const double* state, double* rhs, hipStream_t s) {
  dim3 grid((unsigned)((max_cells + 255) / 256), count);
  hipLaunchKernelGGL(rhs_kernel, grid, dim3(256), 0, s, d_inst, tm, nl, t_start, state, rhs);
}

}  // namespace bt
