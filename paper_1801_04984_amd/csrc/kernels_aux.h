// Launchers of the auxiliary kernels (right-hand side, vector ops, preconditioner).
#pragma once
#include <hip/hip_runtime.h>
#include "common.h"

namespace bt {
void launch_rhs(const InstDev* d_inst, int count, long long max_cells, const TimeMat& tm, int nl, double t_start,
                const double* state, double* rhs, hipStream_t s);
}  // namespace bt
