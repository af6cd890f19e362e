// Launchers of the auxiliary kernels (right-hand side, marching, adjoint helpers).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace bt {
struct SensorW {         // DG-Q1 evaluation weights of one sensor (unused entries have w = 0)
  long long idx[8];      // p index within the p-block of a level
  double w[8];
};
void launch_rhs(const InstDev* d_inst, int count, long long max_cells, const TimeMat& tm, int nl, double t_start,
                const double* state, double* rhs, hipStream_t s);
void launch_bcast(const InstDev* insts, int count, long long maxN, int nl, const double* state, double* x,
                  hipStream_t s);
void launch_extract(const InstDev* insts, int count, long long maxN, int lev, const double* x, double* state,
                    hipStream_t s);
void launch_sensor_state(const InstDev* insts, int count, int n, int nslabs, int nsens, const SensorW* sw,
                         const double* state, const double* p_obs, double* res, hipStream_t s);
void launch_sensor(const InstDev* insts, int count, int lev, int nsens, const SensorW* sw, const double* X,
                   const double* obs, double* res, hipStream_t s);
void launch_adjrhs(const InstDev* insts, int count, long long maxN, const TimeMat& tm, int nl, int has_next,
                   const double* lam_next, int nsens, const SensorW* sw, const double* res, double* a, hipStream_t s);
void launch_grad(const InstDev* insts, int count, long long maxc, int nl, const double* kinv, const double* lam,
                 const double* X, double* grad, hipStream_t s);
}  // namespace bt
