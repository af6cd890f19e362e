// Slab solver: right-hand side, GMRES driver, marching and adjoint sweep.
#include "solver.h"

#include <cmath>
#include <string>

#include "kernels_aux.h"

namespace bt {
void plan_solver_layout(biot_problem_s*, Layout&, bool) {}
void setup_solver(biot_problem_s*, hipStream_t) {}
void refresh_solver(biot_problem_s*, hipStream_t) {}
void destroy_solver(biot_problem_s*) {}

static long long max_cells(const biot_problem_s* h) {
  long long m = 0;
  for (auto& I : h->inst) m = I.ncells > m ? I.ncells : m;
  return m;
}

void launch_slab_rhs(const biot_problem_s* h, const double* state, double t_start, double* rhs, hipStream_t s) {
  hip_check(hipMemsetAsync(rhs, 0, sizeof(double) * h->slab_len, s), "rhs clear");
  launch_rhs(h->d_inst, h->count, max_cells(h), h->tm, h->nl, t_start, state, rhs, s);
  hip_check(hipGetLastError(), "rhs launch");
}
}  // namespace bt

using namespace bt;

#define BIOT_TRY try {
#define BIOT_CATCH                                         \
  }                                                        \
  catch (const BiotError& e) {                             \
    set_error(e.msg);                                      \
    return e.st;                                           \
  }                                                        \
  catch (const std::exception& e) {                        \
    set_error(std::string("internal error: ") + e.what()); \
    return BIOT_ERR_ARG;                                   \
  }                                                        \
  return BIOT_OK;

static void need(bool c, const char* m) {
  if (!c) throw BiotError{BIOT_ERR_ARG, m};
}

extern "C" {

biot_status slab_rhs(biot_problem h, const double* state, double t_start, double* rhs, void* stream) {
  BIOT_TRY
  need(h, "handle is null");
  need(state && rhs, "state and rhs must be device pointers");
  need(std::isfinite(t_start), "t_start must be finite");
  launch_slab_rhs(h, state, t_start, rhs, (hipStream_t)stream);
  BIOT_CATCH
}

biot_status solve_slab(biot_problem, const double*, double*, const biot_solve_opts*, biot_solve_info*, void*) {
  set_error("solve_slab: not built yet");
  return BIOT_ERR_ARG;
}
biot_status solve_slab_transposed(biot_problem, const double*, double*, const biot_solve_opts*, biot_solve_info*,
                                  void*) {
  set_error("solve_slab_transposed: not built yet");
  return BIOT_ERR_ARG;
}
biot_status step(biot_problem, int32_t, double, double*, double*, double*, const biot_solve_opts*, biot_solve_info*,
                 void*) {
  set_error("step: not built yet");
  return BIOT_ERR_ARG;
}
biot_status adjoint_sweep(biot_problem, int32_t, double, const double*, const double*, int32_t, const double*,
                          const biot_solve_opts*, double*, double*, void*) {
  set_error("adjoint_sweep: not built yet");
  return BIOT_ERR_ARG;
}
}
