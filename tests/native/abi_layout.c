/* Prints sizeof and field offsets of the structs of include/ffth.h as
 * "struct.field offset" lines, for comparison with the Python binding. */
#include <stddef.h>
#include <stdio.h>

#include "ffth.h"

#define F(S, f) printf(#S "." #f " %zu\n", offsetof(S, f))
#define Z(S) printf(#S ".sizeof %zu\n", sizeof(S))

int main(void) {
  Z(ffth_problem);
  F(ffth_problem, n); F(ffth_problem, nphases); F(ffth_problem, phase); F(ffth_problem, lame);
  F(ffth_problem, stiffness); F(ffth_problem, lambda0); F(ffth_problem, mu0);
  Z(ffth_opts);
  F(ffth_opts, scheme); F(ffth_opts, precision); F(ffth_opts, tol); F(ffth_opts, max_iter);
  F(ffth_opts, inner_tol); F(ffth_opts, max_outer); F(ffth_opts, check_every); F(ffth_opts, autotune); F(ffth_opts, spectrum16);
  Z(ffth_result);
  F(ffth_result, status); F(ffth_result, iters); F(ffth_result, outer_iters); F(ffth_result, fp64_applications);
  F(ffth_result, projections); F(ffth_result, residual); F(ffth_result, mean_stress); F(ffth_result, g_mean);
  F(ffth_result, seconds);
  return 0;
}
