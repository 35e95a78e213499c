// Internal layout shared by the HIP kernels and the host engine of libplcg.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/plcg.h"

namespace plcg {

constexpr int kLMax = 8;              // largest pipeline length
constexpr int kBand = 2 * kLMax + 1;  // stored rows per column of G (rows c-2l .. c)
constexpr int kGRing = 16;            // columns of G kept (>= l+1 are read)
constexpr int kTRing = 16;            // entries of gamma/delta/eta/zeta kept (>= l+1 are read)
// x update of a sweep with t >= 1 (Eq. x_a2): every sweep adds zeta_{t-1} p_{t-1};
// or, with two p buffers, odd sweeps skip it and even sweeps add zeta_{t-2}
// p_{t-2} and zeta_{t-1} p_{t-1} (the same two roundings, half the x traffic).
constexpr int kXEvery = 0, kXSkip = 1, kXPair = 2;
constexpr int kThreads = 256;         // threads per block of every streaming kernel
constexpr int kVec = 2;               // consecutive unknowns per thread and chunk
constexpr int kChunk = kThreads * kVec;
constexpr int kXcds = 8;              // MI355X: workgroups are dealt round-robin to 8 XCDs
constexpr int kMaxStream = 1024;      // streaming blocks per launch (multiple of kXcds)
// The p(l)-CG sweeps of a working set beyond the memory-side cache (those with
// cache hints) stream with as many workgroups as a CU keeps resident, up to six
// per CU: more waves keep more loads in flight, which is what an HBM-bound
// stream needs (256^3: p(1) 240 -> 213 us per sweep with six per CU instead of
// four; seven or eight per CU were slower than four).  Their partials are laid
// out for up to kSweepStream workgroups.
constexpr int kSweepPerCu = 6;
constexpr int kSweepStream = 1536;    // = kSweepPerCu * 256 CUs (multiple of kXcds and kThreads)
// Largest number of unknowns: indices are int32, and a loop that has reached
// the last unknown may still add one launch's stride (< 2^22) before its test.
constexpr long long kMaxUnknowns = (1LL << 31) - (1LL << 23);

enum Status : int32_t { kRunning = 0, kConverged = 1, kBroken = 2, kNonFinite = 3, kCgBreak = 4 };

// Operator data beyond the grid extents (device pointers; all NULL for the
// constant-coefficient stencils).
struct OpData {
  const double *dg;    // diagonal operator: d (n)
  const int64_t *rp;   // CSR: row offsets (n+1)
  const int32_t *ci;   // CSR: column indices (nnz), or the ELL copy below
  const double *va;    // CSR: values (nnz), or the ELL copy below
  int32_t ell_k;       // > 0: ci / va hold a padded column-major ELLPACK copy: entry j of
                       // row p at j * ell_ld + p (CSR order within the row; padding is
                       // column p with value 0), j < ell_k
  int32_t ell_ld;      // ELL leading dimension: n rounded up to a multiple of 4
  // Variable-coefficient stencil (sx != NULL): edge weights of the grid
  // operator as VarOp reads them, and its diagonal vd (NULL: the unit diagonal
  // of the Jacobi-scaled form).
  const double *sx, *sy, *sz;
  const double *vd;
};

// Host-visible progress record, written by the block that owns the scalar
// state into pinned host memory (mapped), or into device memory when the
// library cannot allocate (the host then copies it from an idle stream).
struct HostStatus {
  int32_t status;     // Status
  int32_t last_t;     // last index t whose x_t is (or will be) formed; -1: none
  int32_t cols;       // columns of G finalised (p(l)) or CG iterations completed
  int32_t seq;        // launch index of the kernel that wrote this record
  double zeta;        // |zeta_t| of the last finalised t (CG: ||r_k||)
  double beta;        // ||r_0|| of the current segment
  double rref;        // reference norm of the stopping test (caller's ||b - A x0||)
  double sumsq;       // result of the last plain reduction (residual norms)
};

// Scalar state of one solve segment.  Two copies alternate between launches:
// launch s reads copy (s-1)&1 and its owning block writes copy s&1, so no
// block ever reads a copy that is being written.
struct DevState {
  double g[kGRing][kBand];   // column c of G at g[c % kGRing][r - c + 2*kLMax], r in [c-2l, c]
  double gam[kTRing], dlt[kTRing], eta[kTRing], zeta[kTRing];
  double sigma[kLMax];
  double beta;               // ||r_0|| of this segment (Alg. 1: sqrt((u_0, r_0)))
  double rref;               // reference norm for the stopping test
  double abs_tol;            // tol * rref
  double cg_rho, cg_alpha, cg_beta;
  double cg_alpha_prev;      // alpha_{k-1} (CG sweep B with paired x updates)
  double sumsq;
  int32_t l;
  int32_t status;
  int32_t last_t;
  int32_t cols;
  int32_t hist_cap;
  int32_t pad[3];
};

// Streaming cache hints of a sweep (bits): kHintLoads - the vectors a thread
// reads only at its own unknowns are loaded non-temporally (never the operator's
// input vector, whose rows and planes other workgroups read again through L2);
// kHintStores - every vector is stored non-temporally.  The host picks none,
// kHintLoads, or both, by working-set size: they pay where the vectors cannot
// stay in the memory-side cache anyway.
constexpr int kHintLoads = 1;
constexpr int kHintStores = 2;

// Arguments of one p(l)-CG sweep (iteration i of Alg. 1).  S is the storage
// type of the vectors (double; float for the FP32-stored inner solver of the
// mixed-precision mode).  Partial sums and the scalar state are always FP64.
template <typename S>
struct SweepArgsT {
  const S *zl[kLMax];        // z^{(l)}_{i-h} for h = 0..R-1 (R ring slots; zl[0] = z^{(l)}_i)
  S *zl_out;                 // slot receiving z^{(l)}_{i+1} (the slot of z^{(l)}_{i+1-R})
  S *zk_cur[kLMax];          // basis k < l: z^{(k)}_{t+k}
  S *zk_prev[kLMax];         // basis k < l: z^{(k)}_{t+k-1}; overwritten with z^{(k)}_{t+k+1}
  S *copy_dst;               // i < l-1: basis i+1 slot receiving z^{(l)}_{i+1}; else NULL
  const S *v0;               // i == l-1: z^{(0)}_0 for the product (u_l, v_0)
  S *p;                      // p_{t-1}
  S *p_out;                  // receives p_t: p itself, or the second p buffer (holding p_{t-2})
  S *x;
  OpData od;                 // diagonal or CSR operator data; all NULL for the stencils
  const double *part_in;     // partials of sweep i-1, [l+1][pstride]
  double *part_out;          // partials of sweep i
  const DevState *st_in;     // state after column i-1
  DevState *st_out;          // state after column i (written by the owning block)
  HostStatus *hs;            // progress record (mapped pinned host memory or device memory)
  double *hist;              // [hist_cap][4] or NULL
  int32_t i, l, n, nx, ny, nz, d3;
  int32_t nchunks;           // ceil(n / (kThreads * 16 / sizeof(S))): chunks of one 16-byte access per thread
  int32_t nstream;           // streaming blocks (multiple of kXcds)
  int32_t nparts_in;         // partials per product in part_in
  int32_t pstride;
  int32_t work;              // 0: only carry the scalar state forward
  int32_t hint;              // streaming cache hints (kHint* bits)
  int32_t xmode;             // kXEvery, kXSkip or kXPair
  int32_t pad;
};
using SweepArgs = SweepArgsT<double>;

struct CgArgs {
  const double *b;
  double *x, *r, *p_old, *p_new, *q;
  OpData od;                 // diagonal or CSR operator data; all NULL for the stencils
  const double *part_in;
  double *part_out;
  const DevState *st_in;
  DevState *st_out;
  HostStatus *hs;
  int32_t k, n, nx, ny, nz, d3, nchunks, nstream, nparts_in, pstride, work;
  int32_t zseg;              // > 0: 3D sweep A marches tiles through zseg planes
  int32_t hint;              // streaming cache hints (kHint* bits)
  int32_t xmode;             // sweep B: kXEvery, kXSkip or kXPair
};

// Resident solves (plcg_resident.hip): one workgroup of kResThreads runs a whole
// segment of Alg. 1, or all of classic CG, for n <= kResMax unknowns held in
// registers, V per thread: p(l)-CG over the 960 threads of waves 1..15 with
// V <= res_vmax(l, kind) (the widths that fit in 128 VGPRs without spilling),
// CG over all 1024 threads.  kind: 0 2D stencil, 1 3D stencil, 2 diagonal, 3 CSR.
constexpr int kResThreads = 1024;
constexpr int kResMax = 5 * (kResThreads - 64);
constexpr int res_vmax(int l, int kind) {
  return kind == 3   ? (l == 1 ? 4 : l == 2 ? 3 : l <= 4 ? 2 : 1)
         : l <= 2    ? (l == 2 && kind == 2 ? 4 : 5)
         : l == 3    ? 3
         : l == 4    ? 2
                     : 1;
}
struct ResArgs {
  const double *z0;          // p(l)-CG: z_0 = u_0 / ||u_0||; CG: r_0
  double *x;                 // x at the segment start; the segment's last iterate at the end
  OpData od;
  const DevState *st_in;     // state after the segment start
  DevState *st_out;          // state at the end
  HostStatus *hs;
  double *hist;              // [hist_cap][4] or NULL
  int32_t n, nx, ny, nz;
  int32_t imax;              // p(l)-CG: last sweep index m + l; CG: maxit
  int32_t pad;
};
// Unknowns per thread of a resident solve of n unknowns (0: not supported).
int resident_width(int method_plcg, int l, int kind, int n);
hipError_t launch_plcg_resident(const ResArgs &a, int l, int kind, hipStream_t s);
hipError_t launch_cg_resident(const ResArgs &a, int kind, hipStream_t s);

// Launchers (plcg_kernels.hip).
hipError_t launch_plcg_sweep(const SweepArgsT<double> &a, hipStream_t s);
hipError_t launch_plcg_sweep(const SweepArgsT<float> &a, hipStream_t s);
// Workgroups per CU that the kernel launch_plcg_sweep would run for `a` keeps
// resident (hipOccupancyMaxActiveBlocksPerMultiprocessor); nothing is launched.
hipError_t plcg_sweep_occupancy(const SweepArgsT<double> &a, int *per_cu);
hipError_t plcg_sweep_occupancy(const SweepArgsT<float> &a, int *per_cu);
hipError_t launch_cg_sweep_a(const CgArgs &a, hipStream_t s);
hipError_t launch_cg_sweep_b(const CgArgs &a, hipStream_t s);
// r = b - A x (r may be NULL); per-block partial sums of r.r into part_out, or
// of (r / wdiv)^2 when wdiv is not NULL.  A is the stencil of (nx, ny, nz, d3),
// or the diagonal / CSR matrix of od.
hipError_t launch_residual(const double *b, const double *x, double *r, double *part_out,
                           int n, int nx, int ny, int nz, bool d3, const OpData &od,
                           const double *wdiv, int nchunks, int nstream, hipStream_t s);
// bs = dis * b, x = x / dis (into a Jacobi-scaled solve); x = x * dis (out of it).
hipError_t launch_jacobi_in(const double *b, const double *dis, double *bs, double *x, int n,
                            hipStream_t s);
hipError_t launch_jacobi_out(double *x, const double *dis, int n, hipStream_t s);
// One block: sum the residual partials and start a segment in *st:
// mode 0 = p(l)-CG (G, beta, status), 1 = CG (rho), 2 = only report the sum.
// The stopping threshold is max(tol * rref, abs_floor).
hipError_t launch_start(const double *part_in, int nparts, DevState *st, HostStatus *hs,
                        int mode, double tol, double rref_in, double abs_floor, hipStream_t s);
// z = r / beta written to up to three destinations (beta from st); no-op unless running.
hipError_t launch_scale(const double *r, double *d0, double *d1, double *d2, const DevState *st,
                        int n, hipStream_t s);
hipError_t launch_scale(const double *r, float *d0, float *d1, float *d2, const DevState *st, int n,
                        hipStream_t s);
// x += d (FP64 += FP32).
hipError_t launch_add_correction(double *x, const float *d, int n, hipStream_t s);
// x += zeta p in the storage type S (double or float), one rounding.
template <typename S>
hipError_t launch_x_step(S *x, const S *p, double zeta, int n, hipStream_t s);
hipError_t launch_apply(const double *x, double *y, int n, int nx, int ny, int nz, bool d3,
                        const OpData &od, hipStream_t s);
hipError_t launch_copy(const double *src, double *dst, int64_t n, hipStream_t s);
// The same for the variable-coefficient stencil (od.sx != NULL; plcg_var_kernels.hip);
// the launchers above hand such operators over to these.
// With occ not NULL the var launcher reports the kernel's occupancy instead of launching.
hipError_t launch_var_sweep(const SweepArgsT<double> &a, hipStream_t s, int *occ = nullptr);
hipError_t launch_var_sweep(const SweepArgsT<float> &a, hipStream_t s, int *occ = nullptr);
hipError_t launch_var_cg_sweep_a(const CgArgs &a, hipStream_t s);
hipError_t launch_var_residual(const double *b, const double *x, double *r, double *part_out,
                               int n, int nx, int ny, int nz, bool d3, const OpData &od,
                               const double *wdiv, int nchunks, int nstream, hipStream_t s);
hipError_t launch_var_apply(const double *x, double *y, int n, int nx, int ny, int nz, bool d3,
                            const OpData &od, hipStream_t s);

}  // namespace plcg

namespace plcg {

// ---------------------------------------------------------------------------
// Batched solves: many independent systems, each in a slot with its own
// vectors, scalar state and phase; one launch (a "tick") advances every slot
// by one step.
// ---------------------------------------------------------------------------

enum Phase : int32_t {
  kEmpty = 0,    // no system
  kInit = 1,     // y = D^{1/2} x0 (the solver works on the Jacobi-scaled system)
  kResid = 2,    // r = D^{-1/2} b - A~ y into ring slot 0, partial sums of r.r and r.r/dis^2
  kStart = 3,    // owner: ||r||, start of Alg. 1 (G, status); or stop
  kScale = 4,    // z_0 = r / ||r|| into ring slot 0 and basis 0 (FP32: r recomputed; c = 0)
  kSweep = 5,    // iteration i of Alg. 1
  kFinal = 6,    // true residual partial sums
  kFinal2 = 7,   // owner: residual norms; others: x = D^{-1/2} y
  kReport = 8,   // owner: result to the host (x is final: written by the previous launch)
  kDone = 9,
  kCorrect = 10  // FP32-refined: y += c (the inner solve's FP32 correction), then kResid
};

// Per slot; two copies alternate by tick parity (tick s reads copy (s-1)&1).
struct BatchState {
  DevState d;
  int32_t phase;
  int32_t i;          // sweep index within the current segment
  int32_t m;          // x-updates allowed in the current segment
  int32_t restarts;
  int32_t total;      // x-updates over all segments
  int32_t reason;     // PLCG_REASON_* once done
  int32_t first;      // 1 until the first segment has started
  int32_t nparts;     // streaming blocks of the previous tick (partials written)
  int32_t outer;      // FP32-refined: refinement steps (corrections added)
  int32_t pad2;
  double rref_orig;   // ||b - A x0|| in the original (unscaled) norm
  double res_scaled;  // final ||r~|| / ||r~_0||
  double res_orig;    // final ||b - A x|| / ||b - A x0||
};

// Per slot, written by the host at admission.
struct SlotDesc {
  double *vec;                          // bases 2l, ring R, p (FP32-refined: then the correction
                                        // c), consecutive, vstride elements of the storage type apart
  const double *sx, *sy, *sz, *dis;     // scaled edge weights, D^{-1/2}
  const double *b;                      // caller's right-hand side
  double *x;                            // caller's x0 on entry, solution at the end
  int64_t vstride;
  int32_t nx, ny, nz, d3, n, nchunks, nblocks, maxit;
  int32_t max_restarts, mixed;         // mixed: FP32-refined
  double tol;
  double inner_tol;                     // FP32-refined inner stop, relative to ||r_k||
};

// Per slot, in mapped pinned host memory: the result once phase == kDone.
struct SlotReport {
  int32_t phase, reason, iters, restarts;
  double res_scaled, res_orig, rnorm0;
  uint64_t ticket;
  int32_t outer, pad;
};

struct BatchArgs {
  const SlotDesc *slots;
  BatchState *state;       // [slots][2]
  double *part;            // [slots][2][l+1][kMaxStream]
  const int2 *sched;       // per block: (slot, streaming block index or -1 for the owner)
  SlotReport *reports;     // mapped host memory
  const uint64_t *tickets; // per slot
  int32_t tick, l;
  int32_t mixed;           // FP32-refined batch: vectors stored in FP32
  int32_t hint;            // streaming cache hints of the sweep phase (kHint* bits)
};

hipError_t launch_batch_tick(const BatchArgs &a, int blocks, hipStream_t s);

// Records msg as the calling thread's last error (plcg_last_error) and returns code.
int32_t set_last_error(int32_t code, const char *msg);

// Unknowns of registered operator op_id of a batch (-1: no such operator).
int64_t batch_op_unknowns(const plcg_batch *b, int32_t op_id);

// Host: edge weights and diagonal of the variable-coefficient grid operator
// (VarOp) from host coefficient arrays (NULL: all 1), Jacobi-scaled or not;
// PLCG_E_INVALID unless every coefficient is finite and > 0 (plcg_batch.cpp).
int32_t edge_weights(int nx, int ny, int nz, bool d3, const double *cx, const double *cy,
                     const double *cz, bool jacobi, double *wx, double *wy, double *wz,
                     double *dd);

// A whole solve (as plcg_create + plcg_solve) in ws_bytes of device memory at
// ws, with no device or pinned host allocation; 2D and 3D stencil operators.
// check_workspace_solve makes the same argument checks without any HIP call.
int32_t check_workspace_solve(const plcg_operator_desc *op, const plcg_config *cfg,
                              size_t ws_bytes);
int32_t solve_in_workspace(const plcg_operator_desc *op, const plcg_config *cfg, void *ws,
                           size_t ws_bytes, const double *d_b, double *d_x, double tol,
                           int32_t maxit, void *stream, plcg_result *out);

}  // namespace plcg
