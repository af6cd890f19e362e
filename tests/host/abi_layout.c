/* Prints the size and field offsets of every struct include/biotst.h
 * declares, one JSON object per line, for comparison with the ctypes
 * mirrors of the Python binding. */
#include <stdio.h>

#include "biotst.h"

#define F(S, f) printf("%s\"%s\": %zu", first ? "" : ", ", #f, offsetof(S, f)), first = 0

int main(void) {
  int first;
  first = 1;
  printf("{\"name\": \"biot_problem_desc\", \"size\": %zu, \"fields\": {", sizeof(biot_problem_desc));
  F(biot_problem_desc, dim); F(biot_problem_desc, n); F(biot_problem_desc, length); F(biot_problem_desc, r);
  F(biot_problem_desc, tau); F(biot_problem_desc, lambda); F(biot_problem_desc, mu); F(biot_problem_desc, b);
  F(biot_problem_desc, M); F(biot_problem_desc, eta); F(biot_problem_desc, L_fs);
  F(biot_problem_desc, load_kind); F(biot_problem_desc, load_s0); F(biot_problem_desc, load_t_ramp);
  F(biot_problem_desc, pair_mode);
  printf("}}\n");
  first = 1;
  printf("{\"name\": \"biot_solve_opts\", \"size\": %zu, \"fields\": {", sizeof(biot_solve_opts));
  F(biot_solve_opts, rtol); F(biot_solve_opts, maxit); F(biot_solve_opts, restart);
  F(biot_solve_opts, precision); F(biot_solve_opts, inner_rtol); F(biot_solve_opts, max_refine);
  F(biot_solve_opts, cheb_degree); F(biot_solve_opts, graph);
  printf("}}\n");
  first = 1;
  printf("{\"name\": \"biot_solve_info\", \"size\": %zu, \"fields\": {", sizeof(biot_solve_info));
  F(biot_solve_info, iterations); F(biot_solve_info, restarts); F(biot_solve_info, ir_sweeps);
  F(biot_solve_info, status); F(biot_solve_info, rel_residual);
  printf("}}\n");
  first = 1;
  printf("{\"name\": \"biot_tuning\", \"size\": %zu, \"fields\": {", sizeof(biot_tuning));
  F(biot_tuning, apply_variant); F(biot_tuning, n_variants); F(biot_tuning, apply_us);
  printf("}}\n");
  first = 1;
  printf("{\"name\": \"biot_fs_opts\", \"size\": %zu, \"fields\": {", sizeof(biot_fs_opts));
  F(biot_fs_opts, rtol); F(biot_fs_opts, max_outer); F(biot_fs_opts, inner_rtol); F(biot_fs_opts, inner_maxit);
  printf("}}\n");
  first = 1;
  printf("{\"name\": \"biot_fs_info\", \"size\": %zu, \"fields\": {", sizeof(biot_fs_info));
  F(biot_fs_info, outer); F(biot_fs_info, flow_iterations); F(biot_fs_info, mech_iterations);
  F(biot_fs_info, status); F(biot_fs_info, rel_residual);
  printf("}}\n");
  return 0;
}
