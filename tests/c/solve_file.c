/* A plain C caller of libplcg: reads n doubles of b from a file, solves the 2D
 * 5-point Poisson system on an nx x ny grid with the given method and l, writes
 * x, and prints one line of results.  Also checks two error paths of the ABI.
 *
 *   solve_file nx ny method(cg|plcg) l tol b.bin x.bin
 *
 * Exit status 0 when the solve converged and the error paths behaved. */
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "plcg.h"

static int check_hip(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    fprintf(stderr, "%s: %s\n", what, hipGetErrorString(e));
    return 1;
  }
  return 0;
}

int main(int argc, char **argv) {
  if (argc != 8 && argc != 10) {
    fprintf(stderr, "usage: %s nx ny cg|plcg l tol b.bin x.bin [cx.bin cy.bin]\n", argv[0]);
    return 2;
  }
  /* with cx.bin, cy.bin: the variable-coefficient operator, Jacobi-scaled, shifts on [0, 2] */
  const int var = argc == 10;
  const int nx = atoi(argv[1]), ny = atoi(argv[2]), l = atoi(argv[4]);
  const int method = strcmp(argv[3], "cg") == 0 ? PLCG_METHOD_CG : PLCG_METHOD_PLCG;
  const double tol = atof(argv[5]);
  const size_t n = (size_t)nx * (size_t)ny;

  double *hb = (double *)malloc(n * sizeof(double));
  double *hx = (double *)calloc(n, sizeof(double));
  FILE *f = fopen(argv[6], "rb");
  if (!f || fread(hb, sizeof(double), n, f) != n) {
    fprintf(stderr, "cannot read %s\n", argv[6]);
    return 2;
  }
  fclose(f);

  /* error paths: an invalid l, and a NULL handle */
  plcg_operator_desc op;
  memset(&op, 0, sizeof(op));
  op.kind = PLCG_OP_STENCIL2D5;
  op.nx = nx;
  op.ny = ny;
  op.nz = 1;
  plcg_config cfg;
  memset(&cfg, 0, sizeof(cfg));
  cfg.method = PLCG_METHOD_PLCG;   /* l is checked for p(l)-CG (CG ignores it) */
  cfg.l = 99;
  cfg.lambda_min = 0.0;
  cfg.lambda_max = 8.0;
  plcg_handle *h = NULL;
  if (plcg_create(&op, &cfg, &h) != PLCG_E_INVALID || h != NULL || plcg_last_error()[0] == 0) {
    fprintf(stderr, "invalid l was not rejected\n");
    return 1;
  }
  plcg_result res;
  if (plcg_solve(NULL, NULL, NULL, tol, 10, NULL, &res) != PLCG_E_INVALID) {
    fprintf(stderr, "NULL handle was not rejected\n");
    return 1;
  }

  cfg.method = method;
  cfg.l = l;
  double *dcx = NULL, *dcy = NULL;
  if (var) {
    const size_t ncx = (size_t)(nx + 1) * ny, ncy = (size_t)nx * (ny + 1);
    double *hcx = (double *)malloc(ncx * sizeof(double));
    double *hcy = (double *)malloc(ncy * sizeof(double));
    FILE *fx = fopen(argv[8], "rb"), *fy = fopen(argv[9], "rb");
    if (!fx || !fy || fread(hcx, sizeof(double), ncx, fx) != ncx ||
        fread(hcy, sizeof(double), ncy, fy) != ncy) {
      fprintf(stderr, "cannot read the coefficient files\n");
      return 2;
    }
    fclose(fx);
    fclose(fy);
    if (check_hip(hipMalloc((void **)&dcx, ncx * sizeof(double)), "hipMalloc") ||
        check_hip(hipMalloc((void **)&dcy, ncy * sizeof(double)), "hipMalloc") ||
        check_hip(hipMemcpy(dcx, hcx, ncx * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy") ||
        check_hip(hipMemcpy(dcy, hcy, ncy * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy"))
      return 1;
    free(hcx);
    free(hcy);
    op.cx = dcx;
    op.cy = dcy;
    op.jacobi = 1;
    cfg.lambda_max = 2.0;
  }
  if (plcg_create(&op, &cfg, &h) != PLCG_OK) {
    fprintf(stderr, "plcg_create: %s\n", plcg_last_error());
    return 1;
  }
  double *db = NULL, *dx = NULL;
  hipStream_t s;
  if (check_hip(hipStreamCreate(&s), "hipStreamCreate") ||
      check_hip(hipMalloc((void **)&db, n * sizeof(double)), "hipMalloc") ||
      check_hip(hipMalloc((void **)&dx, n * sizeof(double)), "hipMalloc") ||
      check_hip(hipMemcpy(db, hb, n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy") ||
      check_hip(hipMemcpy(dx, hx, n * sizeof(double), hipMemcpyHostToDevice), "hipMemcpy"))
    return 1;
  const plcg_status st = plcg_solve(h, db, dx, tol, 100000, (void *)s, &res);
  if (st != PLCG_OK) {
    fprintf(stderr, "plcg_solve: %s\n", plcg_last_error());
    return 1;
  }
  if (check_hip(hipMemcpy(hx, dx, n * sizeof(double), hipMemcpyDeviceToHost), "hipMemcpy"))
    return 1;
  f = fopen(argv[7], "wb");
  if (!f || fwrite(hx, sizeof(double), n, f) != n) {
    fprintf(stderr, "cannot write %s\n", argv[7]);
    return 2;
  }
  fclose(f);
  printf("iters %d reason %d restarts %d true_relres %.6e rec_relres %.6e\n", res.iters,
         res.reason, res.restarts, res.true_relres, res.rec_relres);
  plcg_destroy(h);
  /* the library copied the coefficients at plcg_create */
  if (var) {
    (void)hipFree(dcx);
    (void)hipFree(dcy);
  }
  (void)hipFree(db);
  (void)hipFree(dx);
  (void)hipStreamDestroy(s);
  free(hb);
  free(hx);
  return res.reason == PLCG_REASON_CONVERGED ? 0 : 1;
}
