/* Prints the size and field offsets of every structure the C ABI declares, for
 * the comparison with the Python binding's ctypes layouts (tests/test_abi.py). */
#include <stddef.h>
#include <stdio.h>

#include "plcg.h"

#define S(T) printf(#T " size %zu\n", sizeof(T))
#define F(T, f) printf(#T " " #f " %zu\n", offsetof(T, f))

int main(void) {
  S(plcg_operator_desc);
  F(plcg_operator_desc, kind); F(plcg_operator_desc, nx); F(plcg_operator_desc, ny);
  F(plcg_operator_desc, nz); F(plcg_operator_desc, diag); F(plcg_operator_desc, nnz);
  F(plcg_operator_desc, rowptr); F(plcg_operator_desc, colind); F(plcg_operator_desc, vals);
  F(plcg_operator_desc, jacobi); F(plcg_operator_desc, cx); F(plcg_operator_desc, cy);
  F(plcg_operator_desc, cz);
  S(plcg_config);
  F(plcg_config, method); F(plcg_config, l); F(plcg_config, lambda_min);
  F(plcg_config, lambda_max); F(plcg_config, shifts); F(plcg_config, check_every);
  F(plcg_config, max_restarts); F(plcg_config, history_cap); F(plcg_config, precision);
  F(plcg_config, inner_tol); F(plcg_config, launch_mode); F(plcg_config, x_update);
  S(plcg_result);
  F(plcg_result, iters); F(plcg_result, spmvs); F(plcg_result, restarts); F(plcg_result, reason);
  F(plcg_result, rnorm0); F(plcg_result, rec_relres); F(plcg_result, true_relres);
  F(plcg_result, seconds); F(plcg_result, sweep_ms); F(plcg_result, sweeps); F(plcg_result, outer);
  F(plcg_result, host_waits); F(plcg_result, launch_mode); F(plcg_result, x_update_every);
  S(plcg_batch_config);
  F(plcg_batch_config, l); F(plcg_batch_config, lambda_min); F(plcg_batch_config, lambda_max);
  F(plcg_batch_config, max_slots); F(plcg_batch_config, arena_bytes);
  F(plcg_batch_config, chunks_per_block); F(plcg_batch_config, max_restarts);
  F(plcg_batch_config, use_graph); F(plcg_batch_config, precision); F(plcg_batch_config, inner_tol);
  S(plcg_system_desc);
  F(plcg_system_desc, kind); F(plcg_system_desc, nx); F(plcg_system_desc, ny);
  F(plcg_system_desc, nz); F(plcg_system_desc, cx); F(plcg_system_desc, cy); F(plcg_system_desc, cz);
  S(plcg_request);
  F(plcg_request, arrival_s); F(plcg_request, system); F(plcg_request, maxit); F(plcg_request, tol);
  F(plcg_request, x);
  S(plcg_request_outcome);
  F(plcg_request_outcome, admit_s); F(plcg_request_outcome, finish_s); F(plcg_request_outcome, result);
  return 0;
}
