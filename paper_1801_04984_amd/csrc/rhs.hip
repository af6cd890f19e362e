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

__global__ __launch_bounds__(256) void rhs_kernel(const InstDev* __restrict__ insts, TimeMat tm, int nl, double t_start,
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

namespace bt {

// x_l = state for every time level l (initial guess of a slab)
__global__ __launch_bounds__(256) void bcast_kernel(const InstDev* __restrict__ insts, int nl, const double* __restrict__ state,
                             double* __restrict__ x) {
  const InstDev& I = insts[blockIdx.y];
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    const double v = state[I.state_off + t];
    for (int l = 0; l < nl; ++l) x[I.x_off + l * I.N + t] = v;
  }
}
// state = level `lev` of x
__global__ __launch_bounds__(256) void extract_kernel(const InstDev* __restrict__ insts, int lev, const double* __restrict__ x,
                               double* __restrict__ state) {
  const InstDev& I = insts[blockIdx.y];
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x)
    state[I.state_off + t] = x[I.x_off + lev * I.N + t];
}
void launch_bcast(const InstDev* insts, int count, long long maxN, int nl, const double* state, double* x,
                  hipStream_t s) {
  long long b = (maxN + 255) / 256;
  hipLaunchKernelGGL(bcast_kernel, dim3((unsigned)(b > 4096 ? 4096 : b), count), dim3(256), 0, s, insts, nl, state, x);
}
void launch_extract(const InstDev* insts, int count, long long maxN, int lev, const double* x, double* state,
                    hipStream_t s) {
  long long b = (maxN + 255) / 256;
  hipLaunchKernelGGL(extract_kernel, dim3((unsigned)(b > 4096 ? 4096 : b), count), dim3(256), 0, s, insts, lev, x,
                     state);
}

// sensor residuals: res[k][s] = sum_g w_g p_g (level `lev` of X) - obs[k][s]
__global__ __launch_bounds__(256) void sensor_kernel(const InstDev* __restrict__ insts, int lev, int nsens, const SensorW* __restrict__ sw,
                              const double* __restrict__ X, const double* __restrict__ obs, double* __restrict__ res) {
  const int k = blockIdx.y;
  const InstDev& I = insts[k];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsens) return;
  const SensorW& W = sw[(long long)k * nsens + s];
  const double* P = X + I.x_off + lev * I.N + I.off_p;
  double v = 0.0;
  for (int g = 0; g < 8; ++g) v += W.w[g] * P[W.idx[g]];
  res[(long long)k * nsens + s] = v - obs[(long long)k * nsens + s];
}
void launch_sensor(const InstDev* insts, int count, int lev, int nsens, const SensorW* sw, const double* X,
                   const double* obs, double* res, hipStream_t s) {
  hipLaunchKernelGGL(sensor_kernel, dim3((nsens + 63) / 64, count), dim3(64), 0, s, insts, lev, nsens, sw, X, obs, res);
}

// the same residuals read straight from state n of a state sequence (one
// spatial level per instance) and from p_obs[k][n][s]
__global__ __launch_bounds__(256) void sensor_state_kernel(const InstDev* __restrict__ insts, int n, int nslabs,
                                                           int nsens, const SensorW* __restrict__ sw,
                                                           const double* __restrict__ state,
                                                           const double* __restrict__ p_obs, double* __restrict__ res) {
  const int k = blockIdx.y;
  const InstDev& I = insts[k];
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsens) return;
  const SensorW& W = sw[(long long)k * nsens + s];
  const double* P = state + I.state_off + I.off_p;
  double v = 0.0;
  for (int g = 0; g < 8; ++g) v += W.w[g] * P[W.idx[g]];
  res[(long long)k * nsens + s] = v - p_obs[((long long)k * nslabs + n) * nsens + s];
}
void launch_sensor_state(const InstDev* insts, int count, int n, int nslabs, int nsens, const SensorW* sw,
                         const double* state, const double* p_obs, double* res, hipStream_t s) {
  hipLaunchKernelGGL(sensor_state_kernel, dim3((nsens + 63) / 64, count), dim3(64), 0, s, insts, n, nslabs, nsens, sw,
                     state, p_obs, res);
}

// adjoint right-hand side: a = 0 except
//   level r p-rows:  sum_s res_s psi(x_s)  (sensor scatter, sequential per instance)
//                    - (1/M) w_p c_p
//   level r u-rows:  - b E c_p   (free rows)
// with c_p = sum_i g_i lam_next_i (p-block), the transpose of the dG jump coupling.
__global__ __launch_bounds__(256) void adjrhs_jump_kernel(const InstDev* __restrict__ insts, TimeMat tm, int nl, int has_next,
                                   const double* __restrict__ lam_next, double* __restrict__ a) {
  const InstDev& I = insts[blockIdx.y];
  const int d = I.dim;
  const long long lo = I.x_off + (nl - 1) * I.N;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < I.N; t += (long long)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (has_next) {
      if (t >= I.off_p) {
        double c = 0.0;
        for (int l = 0; l < nl; ++l) c += tm.g[l] * lam_next[I.x_off + l * I.N + t];
        double wp = 1.0;
        for (int e = 0; e < d; ++e) wp *= 0.5 * I.h[e];
        v = -I.Minv * wp * c;
      } else if (t < I.off_q[0]) {
        int comp = 0;
        for (int c2 = 1; c2 < d; ++c2)
          if (t >= I.off_u[c2]) comp = c2;
        long long rem = t - I.off_u[comp];
        int co[3] = {0, 0, 0};
        for (int f = 0; f < 3; ++f) { co[f] = rem % I.su[f]; rem /= I.su[f]; }
        if (!u_fixed(I, comp, co[0], co[1], co[2])) {
          // (E c)(node) = sum over cells of the node, Gauss-2 collocation
          int cl[3][2], al[3][2], nlf[3];
          for (int f = 0; f < 3; ++f) {
            nlf[f] = 0;
            if (f >= d) { cl[f][0] = 0; al[f][0] = 0; nlf[f] = 1; continue; }
            const int m = co[f];
            if (m & 1) { cl[f][0] = (m - 1) / 2; al[f][0] = 1; nlf[f] = 1; }
            else {
              if (m / 2 - 1 >= 0) { cl[f][nlf[f]] = m / 2 - 1; al[f][nlf[f]] = 2; ++nlf[f]; }
              if (m / 2 < I.n[f]) { cl[f][nlf[f]] = m / 2; al[f][nlf[f]] = 0; ++nlf[f]; }
            }
          }
          double s = 0.0;
          for (int iz = 0; iz < nlf[2]; ++iz)
            for (int iy = 0; iy < nlf[1]; ++iy)
              for (int ix = 0; ix < nlf[0]; ++ix) {
                const int cc[3] = {cl[0][ix], cl[1][iy], cl[2][iz]};
                const int aa[3] = {al[0][ix], al[1][iy], al[2][iz]};
                for (int g = 0; g < (d == 3 ? 8 : 4); ++g) {
                  const int gg[3] = {g & 1, (g >> 1) & 1, (g >> 2) & 1};
                  double w = 1.0;
                  for (int f = 0; f < d; ++f) w *= (f == comp) ? GB(aa[f], gg[f]) : 0.5 * I.h[f] * VG(gg[f], aa[f]);
                  const long long po = I.off_p + (2 * cc[0] + gg[0]) +
                                       (long long)I.sp[0] * ((2 * cc[1] + gg[1]) + (long long)I.sp[1] * (d == 3 ? 2 * cc[2] + gg[2] : 0));
                  double cp = 0.0;
                  for (int l = 0; l < nl; ++l) cp += tm.g[l] * lam_next[I.x_off + l * I.N + po];
                  s += w * cp;
                }
              }
          v = -I.b * s;
        }
      }
    }
    for (int l = 0; l < nl - 1; ++l) a[I.x_off + l * I.N + t] = 0.0;
    a[lo + t] = v;
  }
}
__global__ __launch_bounds__(256) void adjrhs_sensor_kernel(const InstDev* __restrict__ insts, int nl, int nsens, const SensorW* __restrict__ sw,
                                     const double* __restrict__ res, double* __restrict__ a) {
  const int k = blockIdx.x;
  const InstDev& I = insts[k];
  if (threadIdx.x != 0) return;
  double* P = a + I.x_off + (nl - 1) * I.N + I.off_p;
  for (int s = 0; s < nsens; ++s) {
    const SensorW& W = sw[(long long)k * nsens + s];
    const double rv = res[(long long)k * nsens + s];
    for (int g = 0; g < 8; ++g)
      if (W.w[g] != 0.0) P[W.idx[g]] += W.w[g] * rv;
  }
}
void launch_adjrhs(const InstDev* insts, int count, long long maxN, const TimeMat& tm, int nl, int has_next,
                   const double* lam_next, int nsens, const SensorW* sw, const double* res, double* a, hipStream_t s) {
  long long b = (maxN + 255) / 256;
  hipLaunchKernelGGL(adjrhs_jump_kernel, dim3((unsigned)(b > 4096 ? 4096 : b), count), dim3(256), 0, s, insts, tm, nl,
                     has_next, lam_next, a);
  hipLaunchKernelGGL(adjrhs_sensor_kernel, dim3(count), dim3(64), 0, s, insts, nl, nsens, sw, res, a);
}

// grad_c += tau eta/K_c sum_i lam_i^T Mq1_c X_i  (free flux DoFs), K == 1 flux mass Mq1
__global__ __launch_bounds__(256) void grad_kernel(const InstDev* __restrict__ insts, int nl, const double* __restrict__ kinv,
                            const double* __restrict__ lam, const double* __restrict__ X, double* __restrict__ grad) {
  const InstDev& I = insts[blockIdx.y];
  const int d = I.dim;
  for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < I.ncells;
       c += (long long)gridDim.x * blockDim.x) {
    const int ce[3] = {(int)(c % I.n[0]), (int)((c / I.n[0]) % I.n[1]), d == 3 ? (int)(c / ((long long)I.n[0] * I.n[1])) : 0};
    double acc = 0.0;
    for (int e = 0; e < d; ++e) {
      double hp = 1.0;
      for (int f = 0; f < d; ++f)
        if (f != e) hp *= 0.5 * I.h[f];
      const int nopen = d == 3 ? 4 : 2;
      for (int go = 0; go < nopen; ++go) {
        long long base = I.off_q[e], s = 1, str_e = 1;
        int bit = 0;
        for (int f = 0; f < d; ++f) {
          if (f == e) str_e = s;
          else { base += (long long)(2 * ce[f] + ((go >> bit) & 1)) * s; ++bit; }
          s *= I.sq[e][f];
        }
        for (int l = 0; l < nl; ++l) {
          const double* L = lam + I.x_off + l * I.N;
          const double* Xl = X + I.x_off + l * I.N;
          for (int a = 0; a < 3; ++a) {
            const int m = 2 * ce[e] + a;
            if (q_fixed(I, e, m)) continue;
            const double la = L[base + m * str_e];
            double mx = 0.0;
            for (int a2 = 0; a2 < 3; ++a2) {
              const int m2 = 2 * ce[e] + a2;
              if (q_fixed(I, e, m2)) continue;
              mx += MC(a, a2) * Xl[base + m2 * str_e];
            }
            acc += la * I.h[e] * hp * mx;
          }
        }
      }
    }
    grad[I.cell_off + c] += I.tau * kinv[I.cell_off + c] * acc;
  }
}
void launch_grad(const InstDev* insts, int count, long long maxc, int nl, const double* kinv, const double* lam,
                 const double* X, double* grad, hipStream_t s) {
  long long b = (maxc + 255) / 256;
  hipLaunchKernelGGL(grad_kernel, dim3((unsigned)(b > 4096 ? 4096 : b), count), dim3(256), 0, s, insts, nl, kinv, lam, X,
                     grad);
}

}  // namespace bt
