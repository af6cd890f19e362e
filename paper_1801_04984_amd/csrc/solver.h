// Solver-side entry points used by the runtime (solver.cpp).
#pragma once
#include "runtime.h"

namespace bt {
void plan_solver_layout(biot_problem_s* h, Layout& L, bool carve);
void setup_solver(biot_problem_s* h, hipStream_t s);
void refresh_solver(biot_problem_s* h, hipStream_t s);
void destroy_solver(biot_problem_s* h);
void launch_apply(const biot_problem_s* h, const void* x, void* y, int transpose, int dtype, hipStream_t s);
// device address of the static scratch of biot_misfit_noalloc on the current device
void* scratch_ptr();
}  // namespace bt
