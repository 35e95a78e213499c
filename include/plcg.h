/*
 * libplcg - deep pipelined Conjugate Gradients, p(l)-CG, and classic CG on one
 * AMD Instinct MI355X (gfx950), behind a plain C ABI.
 *
 * Method: Cools, Cornelis, Ghysels, Vanroose, "Improving strong scaling of the
 * Conjugate Gradient method for solving large linear systems using global
 * reduction pipelining" (EuroMPI'19), Alg. 1 with the identity preconditioner.
 * Each p(l)-CG iteration applies the operator once to the auxiliary basis
 * vector z^{(l)}_i (shifted by sigma_i during the first l iterations), updates
 * the l+1 bases Z^{(0..l)} with three-term recurrences (Eqs. all_z_rec2 and
 * specific_z_rec), updates the search direction p and the iterate x
 * (Eqs. pdir, x_a2), and starts the l+1 dot products that form column i+1 of
 * the banded basis transformation G (Sec. 2.2, "Number of dot products").  The
 * dot products of iteration i are consumed l iterations later.
 *
 * Conventions shared by every call:
 *  - Vectors are contiguous float64 arrays in device memory, 16-byte aligned,
 *    indexed row-major with x fastest (index = x + nx*(y + ny*z)).  Values
 *    outside the grid are zero (homogeneous Dirichlet boundary eliminated).
 *  - A system has at most 2^31 - 2^23 unknowns (larger: PLCG_E_INVALID).
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *    device work of a call is enqueued on that stream.
 *  - The library allocates its own workspace at plcg_create and frees it at
 *    plcg_destroy.  Caller buffers are never retained after a call returns
 *    (plcg_submit: until plcg_poll reports completion).
 *  - Errors are returned as negative plcg_status codes; plcg_last_error()
 *    gives a message for the calling thread.  Nothing aborts the process.
 *  - A handle serves one caller at a time: while a solve runs on it
 *    (plcg_solve, or plcg_submit until plcg_poll reports completion) other
 *    solves return PLCG_E_BUSY; plcg_destroy waits for a submitted solve.
 *    Calls on one batch are not safe to make from several threads at once.
 */
#ifndef PLCG_H
#define PLCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct plcg_handle plcg_handle;
typedef int32_t plcg_status;

enum {
  PLCG_OK = 0,
  PLCG_NOT_READY = 1,      /* plcg_poll: the solve is still running */
  PLCG_E_INVALID = -1,     /* bad argument: NULL pointer, size, l, alignment */
  PLCG_E_NOMEM = -2,       /* device or pinned-host allocation failed */
  PLCG_E_HIP = -3,         /* a HIP runtime call failed (message has the code) */
  PLCG_E_BUSY = -4,        /* the handle already has a solve in flight */
  PLCG_E_NONFINITE = -5    /* the initial residual is not finite (NaN/Inf in b or x0) */
};

/* Operator kinds: unscaled integer Dirichlet Laplacians (spectrum inside (0, 8)
 * in 2D and (0, 12) in 3D), a general sparse matrix, and a diagonal matrix - the
 * "one-point stencil" of the paper's communication-bound toy problem (Sec. 4.2),
 * whose diagonal holds the 2D Laplacian's eigenvalues so that CG sees the same
 * spectrum with an SpMV that costs no more than a vector update. */
enum {
  PLCG_OP_STENCIL2D5 = 1,  /* (Au) = 4u - u(x-1) - u(x+1) - u(y-1) - u(y+1) */
  PLCG_OP_STENCIL3D7 = 2,  /* (Au) = 6u - sum of the six face neighbours    */
  PLCG_OP_CSR = 3,         /* a general sparse matrix in compressed sparse rows (the
                              assembled matrices the paper's PETSc runs use); it must be
                              symmetric positive definite */
  PLCG_OP_DIAG = 4         /* (Au)_p = d_p u_p, d given in plcg_operator_desc.diag */
};

enum { PLCG_METHOD_CG = 0, PLCG_METHOD_PLCG = 1 };

/* Arithmetic of p(l)-CG.  FP32_REFINED: iterative refinement in FP64 around an
 * inner p(l)-CG whose vectors (bases, p, correction) are stored in FP32 and whose
 * dot products, G, T and LU scalars are FP64; each refinement step recomputes
 * r_k = b - A x in FP64, solves A d = r_k to |zeta| < max(inner_tol ||r_k||,
 * tol ||r_0|| / 2), and adds x += d in FP64, until ||r_k|| < tol ||r_0||. */
enum { PLCG_PREC_FP64 = 0, PLCG_PREC_FP32_REFINED = 1 };

/* How the iterations are launched.
 * STREAMING: one launch per iteration of Alg. 1 (two per CG iteration) over as
 *   many workgroups as the system fills; the products of each iteration are
 *   reduced across workgroups by a later launch (Sec. 3.1 overlap).
 * RESIDENT: a whole run of Alg. 1 (or all of CG) in one launch of one
 *   1024-thread workgroup that keeps the vectors in registers and reduces inside
 *   the workgroup - for small systems, whose iterations would otherwise be
 *   dominated by launch and device-wide reduction latency.  Available for FP64
 *   with n <= PLCG_RESIDENT_MAX unknowns and, for p(l)-CG, the pipeline lengths
 *   that fit the registers (PLCG_E_INVALID at create otherwise; see
 *   plcg_resident_supported).
 * AUTO (default): RESIDENT where it is available, else STREAMING. */
enum { PLCG_LAUNCH_AUTO = 0, PLCG_LAUNCH_STREAMING = 1, PLCG_LAUNCH_RESIDENT = 2 };
#define PLCG_RESIDENT_MAX 4800

/* When the streaming p(l)-CG sweeps write the iterate x_t = x_{t-1} + zeta_{t-1} p_{t-1}
 * (Eq. x_a2), and classic CG's second sweep x_{k+1} = x_k + alpha_k p_k:
 * EVERY: in every sweep (one p buffer).
 * PAIRED: in every second sweep, both steps at once: p is kept in two buffers, an odd
 *   sweep leaves x alone and an even one adds zeta_{t-2} p_{t-2} and zeta_{t-1} p_{t-1}
 *   with the same two roundings, so x is bit for bit the one EVERY gives; a run that
 *   ends after an odd step adds the last step in one more small kernel.  Half a vector
 *   pass less per iteration, one more vector of device memory.
 * AUTO (default): PAIRED where a vector is at least 16 MiB (below that the sweeps are
 *   bound by launch and reduction latency, which the even sweep's extra loads
 *   lengthen) and the second p buffer does not push a working set that fits the
 *   256 MiB memory-side cache out of it; else EVERY.
 * Classic CG pairs the same way with the two p buffers it has anyway (no extra memory;
 *   AUTO: always).  The resident launches and the batches ignore it. */
enum { PLCG_X_AUTO = 0, PLCG_X_EVERY = 1, PLCG_X_PAIRED = 2 };

enum {
  PLCG_REASON_NONE = 0,
  PLCG_REASON_CONVERGED = 1,        /* recursive residual below tol            */
  PLCG_REASON_MAXIT = 2,            /* maxit x-updates made                    */
  PLCG_REASON_BREAKDOWN_LIMIT = 3,  /* more than max_restarts restarts needed  */
  PLCG_REASON_NONFINITE = 4,        /* initial residual not finite             */
  PLCG_REASON_BREAKDOWN = 5         /* CG only: (p, Ap) <= 0, operator not SPD */
};

typedef struct {
  int32_t kind;           /* PLCG_OP_* */
  int32_t nx, ny, nz;     /* grid extents, each >= 1; nz ignored for 2D (use 1);
                             PLCG_OP_DIAG: n = nx * ny * nz unknowns */
  const double *diag;     /* PLCG_OP_DIAG only (else ignored): device array of n
                             FP64 entries, each finite and > 0 (else
                             PLCG_E_INVALID).  Copied at plcg_create; the caller
                             keeps ownership and may free it afterwards. */
  int64_t nnz;            /* PLCG_OP_CSR only: stored entries */
  const int64_t *rowptr;  /* PLCG_OP_CSR, device: n + 1 offsets, rowptr[0] = 0,
                             nondecreasing, rowptr[n] = nnz */
  const int32_t *colind;  /* PLCG_OP_CSR, device: nnz column indices in [0, n) */
  const double *vals;     /* PLCG_OP_CSR, device: nnz finite FP64 values.  The three
                             arrays are checked and copied at plcg_create (violations
                             give PLCG_E_INVALID); symmetry and definiteness are not
                             checked: a matrix that is not SPD shows up as breakdowns
                             (restart limit) or, for CG, PLCG_REASON_BREAKDOWN. */
  int32_t jacobi;         /* PLCG_OP_CSR, or a stencil kind with edge coefficients (else
                             must be 0): 1 = Jacobi-preconditioned solve, which is Alg. 1
                             with M = diag(A) (Sec. 2.2) in its symmetrically scaled form:
                             the library stores D^{-1/2} A D^{-1/2} (d_p = a_pp > 0, else
                             PLCG_E_INVALID), solves for y = D^{1/2} x from D^{-1/2} b (x is
                             transformed in place on entry and back on exit), stops on the
                             scaled residual |zeta_t| < tol ||D^{-1/2}(b - A x0)|| and
                             reports rec_relres in that norm, rnorm0 and true_relres in the
                             original one.  The Chebyshev interval refers to the scaled
                             matrix ([0, 2] holds its spectrum when A is a weakly diagonally
                             dominant M-matrix, e.g. every variable-coefficient stencil). */
  const double *cx;       /* PLCG_OP_STENCIL2D5 / 3D7 only: NULL for the constant integer
                             stencil; else device arrays of edge coefficients c > 0 of the
                             variable-coefficient operator (A u)_p = sum over the grid edges
                             (p, q) incident to p of c_pq (u_p - u_q), u = 0 outside (edges
                             to the boundary included, so A is an SPD M-matrix; the paper's
                             Sec. 4 problems are of this operator class).  cx: per row
                             (y, z) nx+1 values, the first and last being boundary edges,
                             x fastest; */
  const double *cy;       /* per plane z: ny+1 rows of nx values (edge below row y at row
                             y); required with cx; */
  const double *cz;       /* 3D: nz+1 planes of nx*ny values (edge below plane z at plane
                             z); required with cx in 3D, ignored in 2D.  Checked (finite,
                             > 0; else PLCG_E_INVALID) and copied at plcg_create; the
                             caller keeps ownership.  Each SpMV then reads 2 (2D) or 3 (3D)
                             arrays of edge weights, plus the diagonal when jacobi = 0.
                             The resident launch mode is not offered for these operators,
                             and plcg_apply applies the operator the solver iterates with
                             (the scaled one when jacobi = 1). */
} plcg_operator_desc;

typedef struct {
  int32_t method;         /* PLCG_METHOD_CG or PLCG_METHOD_PLCG */
  int32_t l;              /* pipeline length, 1..8 (ignored for CG) */
  double lambda_min;      /* Chebyshev interval of Eq. (chebyshev), Sec. 2.2 */
  double lambda_max;
  const double *shifts;   /* host array of l shifts, or NULL for Chebyshev shifts */
  int32_t check_every;    /* iterations per host status check; <= 0: default 64 */
  int32_t max_restarts;   /* restarts after square-root breakdown; < 0: default 100 */
  int32_t history_cap;    /* keep gamma_t, delta_t, eta_t, zeta_t for t < cap (0: off) */
  int32_t precision;      /* PLCG_PREC_*; FP32_REFINED needs method PLCG */
  double inner_tol;       /* FP32_REFINED: relative tolerance of each inner solve, in (0, 1);
                             <= 0: default 1e-3 */
  int32_t launch_mode;    /* PLCG_LAUNCH_* (0 = AUTO) */
  int32_t x_update;       /* PLCG_X_* (0 = AUTO) */
} plcg_config;

typedef struct {
  int32_t iters;          /* x updates (t of Alg. 1, summed over restarts) */
  int32_t spmvs;          /* operator applications, including residuals */
  int32_t restarts;       /* explicit restarts after breakdown (Sec. 2.2) */
  int32_t reason;         /* PLCG_REASON_* */
  double rnorm0;          /* ||b - A x0|| of the caller's x0 */
  double rec_relres;      /* |zeta_t| / rnorm0 (CG: recursive ||r|| / rnorm0) */
  double true_relres;     /* ||b - A x|| / rnorm0, recomputed in FP64 at the end */
  double seconds;         /* host wall time of the call */
  double sweep_ms;        /* with timing enabled: duration of the iteration kernels that did
                             work, see plcg_set_timing (launches enqueued after the stop
                             return at once and are left out) */
  int64_t sweeps;         /* with timing enabled: number of launches in sweep_ms */
  int32_t outer;          /* FP32_REFINED: refinement steps (0 otherwise) */
  int32_t host_waits;     /* plcg_solve: times the host blocked on the device (stream and
                             event synchronisations): about (iterations + l) / check_every
                             plus a few per restart or refinement step (STREAMING), a few
                             per restart (RESIDENT); 0 from batches */
  int32_t launch_mode;    /* PLCG_LAUNCH_STREAMING or PLCG_LAUNCH_RESIDENT: how the
                             iterations of this solve ran (0 from batches) */
  int32_t x_update_every; /* 2: the streaming sweeps of this solve wrote x on every
                             second iteration (PLCG_X_PAIRED), 1: on every iteration
                             (also resident launches); 0 from batches */
} plcg_result;

/* Create a solver for one operator and one configuration.
 * Validates the descriptor (extents >= 1, n = nx*ny*nz <= 2^31 - 2^23; the
 * diagonal or CSR arrays as described at plcg_operator_desc) and the config
 * (l in 1..8, lambda_min < lambda_max unless explicit shifts are given),
 * computes the shifts (Eq. chebyshev, i = 0..l-1, so sigma_0 is the largest)
 * and allocates all device workspace on the current HIP device.
 * Returns PLCG_E_INVALID / PLCG_E_NOMEM / PLCG_E_HIP on failure (*out = NULL). */
plcg_status plcg_create(const plcg_operator_desc *op, const plcg_config *cfg,
                        plcg_handle **out);

/* Solve A x = b.  d_b: n doubles (read only).  d_x: n doubles, holds x0 on entry
 * and the final iterate on return.  Stops when the recursive residual norm
 * |zeta_t| (Alg. 1; CG: its recursive ||r_k||) falls below tol * ||b - A x0||
 * (Jacobi-scaled CSR: both norms of the scaled system), after maxit x-updates, or
 * after max_restarts explicit restarts (restart = Alg. 1 from the latest
 * iterate).  In FP32_REFINED mode the test is on the FP64 residual recomputed
 * at every refinement step, and maxit bounds the inner x-updates.  Blocks the
 * host until the result is known.  Iteration counts, residuals and the stop
 * reason are written to *out (may be NULL). */
plcg_status plcg_solve(plcg_handle *h, const double *d_b, double *d_x, double tol,
                       int32_t maxit, void *stream, plcg_result *out);

/* Same as plcg_solve, but returns at once: a host worker thread drives the
 * solve.  The handle accepts one solve at a time (PLCG_E_BUSY otherwise);
 * d_b and d_x must stay valid until plcg_poll returns PLCG_OK for *ticket. */
plcg_status plcg_submit(plcg_handle *h, const double *d_b, double *d_x, double tol,
                        int32_t maxit, void *stream, uint64_t *ticket);

/* PLCG_NOT_READY while the solve of `ticket` runs; PLCG_OK (result in *out)
 * or the solve's error status once it has finished; PLCG_E_INVALID for an
 * unknown ticket. */
plcg_status plcg_poll(plcg_handle *h, uint64_t ticket, plcg_result *out);

/* Release the handle and its workspace (waits for a submitted solve). */
plcg_status plcg_destroy(plcg_handle *h);

/* Message for the last non-OK status returned on the calling thread. */
const char *plcg_last_error(void);

/* y = A x with the handle's operator (d_x, d_y: n doubles, distinct). */
plcg_status plcg_apply(plcg_handle *h, const double *d_x, double *d_y, void *stream);

/* Number of unknowns n of the handle's operator. */
int64_t plcg_size(const plcg_handle *h);

/* The l shifts the handle uses (host array of >= l doubles). */
plcg_status plcg_get_shifts(const plcg_handle *h, double *out);

/* Diagnostics of the last solve's last restart segment: rows t = 0..count-1
 * of (gamma_t, delta_t, eta_t, zeta_t), 4 doubles per row, as computed on the
 * device (needs history_cap > 0 at create). */
plcg_status plcg_get_history(const plcg_handle *h, double *out, int32_t cap, int32_t *count);

/* Enable (1) or disable (0) timing of the iteration kernels with HIP events
 * around each group of check_every back-to-back launches; reported in
 * plcg_result.sweep_ms / sweeps, summed over the groups in which every launch
 * did work (over every group with work when a solve is shorter than a group).
 * A RESIDENT solve times each of its launches and counts in sweeps the
 * iteration launches it replaces (p(l)-CG: the sweeps it ran; CG: two per
 * iteration), so sweep_ms / sweeps compares with the STREAMING figure. */
plcg_status plcg_set_timing(plcg_handle *h, int32_t enable);

/* Measurement aid: dst[i] = src[i], i < n, with a plain streaming kernel
 * (calibrates hardware byte counters against a known traffic volume). */
plcg_status plcg_copy(const double *d_src, double *d_dst, int64_t n, void *stream);

/* 1 if plcg_create would accept PLCG_LAUNCH_RESIDENT for this operator kind,
 * size n, method and pipeline length l (FP64), else 0. */
int32_t plcg_resident_supported(int32_t kind, int64_t n, int32_t method, int32_t l);

/* Library version, major*10000 + minor*100 + patch. */
int32_t plcg_version(void);

/* Size of the static device workspace of plcg_solve_noalloc (64 MiB per GPU). */
#define PLCG_NOALLOC_BYTES (64LL << 20)

/* For callers that cannot allocate device or pinned host memory (code that
 * must not call hipMalloc: tight serving loops, harnesses that forbid it): the
 * solve of plcg_create + plcg_solve + plcg_destroy in one call, with every
 * workspace buffer (work vectors, partial sums, scalar state, progress record)
 * taken from a static device array of PLCG_NOALLOC_BYTES that each GPU holds
 * from the library's first use of it until the process ends.  It calls no
 * hipMalloc, hipFree or other allocating routine.
 *  - op: PLCG_OP_STENCIL2D5 or PLCG_OP_STENCIL3D7 with constant coefficients
 *    only (cx, cy, cz NULL, jacobi 0: the other operators need library copies
 *    of their data); cfg as for plcg_create, history_cap = 0.
 *    d_b, d_x, tol, maxit, stream and *out as for plcg_solve; the result and x
 *    are bit for bit those of plcg_solve with the same op and cfg.  Timing is
 *    not available (sweep_ms = 0).
 *  - Limits: the work vectors must fit the array: about (2l + max(2, l-1) + 2)
 *    n doubles for p(l)-CG (FP32_REFINED: that many floats plus n doubles), 4 n
 *    doubles for CG, plus about 0.2 MiB (e.g. p(1)-CG up to ~1.3 M unknowns);
 *    larger systems give PLCG_E_INVALID with the bytes needed in the message,
 *    before any device work.
 *  - Each call re-initialises the scalar state and clears the partial sums and
 *    the progress record in the array (the array keeps the last call's
 *    contents otherwise).  Calls on one GPU share its array: the library
 *    serialises them within the process (a second caller blocks until the
 *    first returns); they must not be captured into a graph (the call waits on
 *    the host).
 *  - The host reads the device's progress from an idle stream after every
 *    check_every launches, so the device idles while the host enqueues the
 *    next group (plcg_solve overlaps the two through pinned host memory). */
plcg_status plcg_solve_noalloc(const plcg_operator_desc *op, const plcg_config *cfg,
                               const double *d_b, double *d_x, double tol, int32_t maxit,
                               void *stream, plcg_result *out);

/* ------------------------------------------------------------------------
 * Batched and served solves.
 *
 * A batch holds up to max_slots independent systems at once, each in a slot of
 * HBM sized by its footprint.  One launch ("tick") advances every system by one
 * step: setup, one p(l)-CG iteration, or the final residual and report.  A
 * system's result does not depend on which other systems share the batch.
 * The operator of a batched system is the variable-coefficient Laplacian
 * (A u)_p = sum_q c_pq (u_p - u_q) over the grid edges incident to p (edges to
 * the Dirichlet boundary included, u = 0 outside), solved in its symmetrically
 * Jacobi-scaled form D^{-1/2} A D^{-1/2} (unit diagonal, spectrum in (0, 2)),
 * with Chebyshev shifts on [lambda_min, lambda_max] (default [0, 2]).  The
 * stopping test is on the scaled residual; the original-space residual is
 * reported beside it.
 * ------------------------------------------------------------------------ */

typedef struct plcg_batch plcg_batch;

typedef struct {
  int32_t l;              /* pipeline length, 2..5 (coefficients are used one launch late) */
  double lambda_min;      /* Chebyshev interval for the scaled operator; both 0: [0, 2] */
  double lambda_max;
  int32_t max_slots;      /* systems in flight, >= 1 */
  int64_t arena_bytes;    /* device memory reserved for the systems' data */
  int32_t chunks_per_block; /* unknowns per workgroup = 512 * this; <= 0: 4 (see
                               plcg_batch_autotune) */
  int32_t max_restarts;   /* < 0: default 100 */
  int32_t use_graph;      /* 1: replay groups of ticks from a captured hipGraph */
  int32_t precision;      /* PLCG_PREC_FP64, or PLCG_PREC_FP32_REFINED: every system runs
                             FP64 iterative refinement (x, residual, operator in FP64)
                             around an inner p(l)-CG whose vectors are stored in FP32
                             (dot products, G, T, LU in FP64), as for plcg_create */
  double inner_tol;       /* FP32_REFINED: inner stop |zeta_t| < inner_tol ||r_k||
                             (0 < inner_tol < 1; <= 0: 1e-3) */
} plcg_batch_config;

typedef struct {
  int32_t kind;           /* PLCG_OP_STENCIL2D5 or PLCG_OP_STENCIL3D7 */
  int32_t nx, ny, nz;     /* grid extents (nz = 1 in 2D) */
  const double *cx;       /* host, edge coefficients c > 0 between x-neighbours: per row (y, z)
                             nx+1 values, the first and last being the boundary edges;
                             NULL: all 1 */
  const double *cy;       /* host, per (z, x) column ny+1 values stored as [z][y][x] with y in
                             0..ny (edge between y-1 and y); NULL: all 1 */
  const double *cz;       /* host, 3D only, [z][y][x] with z in 0..nz; NULL: all 1 */
} plcg_system_desc;

/* Create an empty batch on the current HIP device. */
plcg_status plcg_batch_create(const plcg_batch_config *cfg, plcg_batch **out);

/* Device bytes a system takes in the batch arena (work vectors + scaled operator). */
int64_t plcg_batch_footprint(const plcg_batch *b, const plcg_system_desc *sys);

/* Admit one system: d_b, d_x device vectors of n doubles (x0 on entry, solution
 * once polled done), tol relative to the initial scaled residual, maxit x-updates
 * (FP32_REFINED: inner iterations over all refinement steps).
 * Copies and scales the coefficients (enqueued on `stream`).  PLCG_E_BUSY when
 * no slot or not enough arena space is free (nothing is changed then). */
plcg_status plcg_batch_add(plcg_batch *b, const plcg_system_desc *sys, const double *d_b,
                           double *d_x, double tol, int32_t maxit, void *stream,
                           uint64_t *ticket);

/* Enqueue `ticks` launches on `stream` (returns without waiting). */
plcg_status plcg_batch_step(plcg_batch *b, int32_t ticks, void *stream);

/* PLCG_NOT_READY until the system of `ticket` is done; then PLCG_OK with the
 * result (iters, restarts, reason, outer = refinement steps for FP32_REFINED;
 * rnorm0 = original-space ||b - A x0||, rec_relres = scaled residual (FP32_REFINED:
 * recomputed in FP64 after the last correction), true_relres = original-space
 * residual) and the slot is freed.  PLCG_E_INVALID for an unknown ticket. */
plcg_status plcg_batch_poll(plcg_batch *b, uint64_t ticket, plcg_result *out);

/* Systems admitted and not yet polled done. */
int32_t plcg_batch_active(const plcg_batch *b);

/* Workgroups per launch in the current schedule (0 when nothing is admitted). */
int32_t plcg_batch_grid(const plcg_batch *b);

/* Chunks (512 unknowns) per workgroup in use for the largest systems (more than
 * 64 chunks); after autotuning, the choice made. */
int32_t plcg_batch_chunks_per_block(const plcg_batch *b);

/* The block-to-system schedule in use: chunks (512 unknowns) per streaming
 * workgroup for systems of at most 8 chunks (cpb[0]), at most 64 chunks (cpb[1])
 * and more (cpb[2]); each system also has one owner workgroup. */
plcg_status plcg_batch_get_schedule(const plcg_batch *b, int32_t *cpb);

/* Set that schedule (each value in 1..1024) for the systems admitted from now
 * on, e.g. one plcg_batch_autotune chose on an earlier batch of similar systems. */
plcg_status plcg_batch_set_schedule(plcg_batch *b, const int32_t *cpb);

/* Autotuner of the block-to-system schedule: times `ticks` launches of the
 * systems currently admitted (the launches advance the solves) for each
 * candidate (1, 2, 4, 8, 16 chunks per workgroup), first one size for every
 * size class, then each class in turn from the largest, and keeps the fastest
 * per active unknown.  Applies to systems admitted later too.  Blocks the host. */
plcg_status plcg_batch_autotune(plcg_batch *b, int32_t ticks, void *stream);

plcg_status plcg_batch_destroy(plcg_batch *b);

/* Register an operator once (scaled and copied to the device, enqueued on
 * `stream`); requests that name it (plcg_batch_add_op) share it.  The operator
 * lives until the batch is destroyed. */
plcg_status plcg_batch_register(plcg_batch *b, const plcg_system_desc *sys, void *stream,
                                int32_t *op_id);

/* Arena bytes one request on a registered operator takes (internal_x: the
 * solution is kept in the slot instead of a caller buffer). */
int64_t plcg_batch_request_footprint(const plcg_batch *b, int32_t op_id, int32_t internal_x);

/* Admit one request on a registered operator; d_x may be NULL (the solution is
 * then kept inside the slot, x0 = 0, and released with it).  PLCG_E_BUSY when no
 * slot or arena space is free. */
plcg_status plcg_batch_add_op(plcg_batch *b, int32_t op_id, const double *d_b, double *d_x,
                              double tol, int32_t maxit, void *stream, uint64_t *ticket);

typedef struct {
  double arrival_s;       /* seconds after the start of plcg_serve; sorted */
  int32_t system;         /* index into the op_ids / d_b arrays */
  int32_t maxit;
  double tol;
  double *x;              /* device, n doubles of the request's system (16-byte aligned), or
                             NULL: receives the solution.  Set to 0 (x0) when the request is
                             admitted, written by the solve, and final when out[k].finish_s
                             is set; the caller keeps ownership.  Requests in flight at the
                             same time need distinct buffers.  NULL: the solution stays
                             inside the batch and is released with the slot. */
} plcg_request;

typedef struct {
  double admit_s;         /* admitted into the batch (-1: never) */
  double finish_s;        /* result available (-1: not finished within the time limit) */
  plcg_result result;
} plcg_request_outcome;

/* Continuous-batching serving loop on an (empty) batch: admits arrived requests
 * in FIFO order while a slot and arena space are free (admission by HBM
 * footprint), enqueues ticks_per_round launches, retires finished solves, and
 * repeats until every request is done or time_limit_s has passed.  Request k
 * solves with operator op_ids[system] and right-hand side d_b[system] (device,
 * shared, read only), x0 = 0; its solution goes to reqs[k].x (or stays inside
 * the batch when that is NULL, which also takes n more doubles of arena per
 * request).  Timings and results go to out[k].  Solves still running when the
 * time limit passes keep their slots (and keep writing reqs[k].x) until the
 * batch is destroyed.  PLCG_E_INVALID for unsorted arrivals, an unknown system,
 * a misaligned x or a request that does not fit an empty batch. */
plcg_status plcg_serve(plcg_batch *b, const int32_t *op_ids, const double *const *d_b,
                       int32_t nops, const plcg_request *reqs, int32_t nreq,
                       int32_t ticks_per_round, double time_limit_s, void *stream,
                       plcg_request_outcome *out);

#ifdef __cplusplus
}
#endif

#endif /* PLCG_H */
