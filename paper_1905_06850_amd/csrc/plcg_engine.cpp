// Host engine and C ABI of libplcg.
//
// The engine enqueues one fused sweep kernel per p(l)-CG iteration (two per CG
// iteration) on the caller's stream, with the buffer roles of the ring of
// basis vectors decided here on the host.  The device writes its progress
// (status, last usable t, residual norms) into mapped pinned host memory; the
// host looks at it after each group of `check_every` iterations, keeping at
// most two groups in flight, and stops enqueueing once the device reports
// convergence or breakdown.  Sweeps enqueued past the stop see the status and
// return at once.  A breakdown (Sec. 2.2, "Square root breakdowns") restarts
// Alg. 1 from the most recent iterate with a recomputed residual, keeping the
// original reference norm of the stopping test.
#include "plcg_internal.h"

#include "../../include/plcg.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

using namespace plcg;

namespace {

thread_local std::string g_last_error;

plcg_status fail(plcg_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define PLCG_HIP(call)                                                                    \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(PLCG_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_));         \
  } while (0)

constexpr int kDefaultCheck = 64;
constexpr long long kCacheBytes = 256LL << 20;   // MI355X memory-side (Infinity) cache
constexpr long long kLargeVector = 96LL << 20;   // vectors worth storing non-temporally
// Iterations one resident launch may run (about a second for the largest
// resident systems); longer runs use the streaming kernels.
constexpr int kResIterCap = 1 << 20;
constexpr int kDefaultRestarts = 100;

// Streaming cache hints for the sweeps of a solver whose vectors are `word`
// bytes per unknown (measured on 2048^2 and 256^3 Poisson, the 2048^2 CSR
// matrix and diagonal toy): non-temporal loads pay once the vectors and
// operator data a solver streams outgrow the 256 MiB memory-side cache (up to
// 12 % per iteration), and cost up to 16 % while they fit, because the
// alternating sweep order then finds them there; non-temporal stores pay
// only when each vector alone is large (3D 256^3 FP64: another 3-5 %) and cost
// up to 9 % at 2048^2, whose freshly written vectors the next sweep re-reads
// from that cache.  The footprint counts one p buffer (the second one is used
// only where it does not cross the cache size, see pair_x_updates).  The store
// rule counts the system's size in 8-byte words whatever the storage: the
// FP32-stored 256^3 sweeps (67 MB vectors) with non-temporal stores, p(3)
// 173.7 -> 169.9 us per iteration, p(1) unchanged.
int pick_hint(long long n, int method, int l, int R, int word, long long op_bytes) {
  const long long vecs = method == PLCG_METHOD_CG ? 5 : 2LL * l + R + 2;
  const long long bytes = vecs * n * word + op_bytes;
  if (bytes <= kCacheBytes) return 0;
  return n * 8 > kLargeVector ? (kHintLoads | kHintStores) : kHintLoads;
}

// PLCG_X_AUTO: whether the streaming p(l)-CG sweeps keep p in two buffers and
// update x on even t only (half a vector pass less per iteration: 2048^2 p(1)
// and p(3) 2-3 % faster).  Not for vectors under 16 MiB, whose sweeps are bound
// by launch and reduction latency (64^2 to 1024^2: from 2 % faster to 3 % slower
// paired), and not where the extra buffer pushes a working set that fits the
// memory-side cache out of it (2048^2 p(2)-CG, 8 vectors of exactly 256 MiB:
// 16 % slower paired).
constexpr long long kPairMinVector = 16LL << 20;
bool pair_x_updates(long long n, int l, int R, int word, long long op_bytes) {
  if (n * word < kPairMinVector) return false;
  const long long one = (2LL * l + R + 2) * n * word + op_bytes;
  return !(one <= kCacheBytes && one + n * word > kCacheBytes);
}

// Operator kind numbering of the kernels: 0 2D stencil, 1 3D stencil, 2 diagonal, 3 CSR.
int op_kind_index(int kind) {
  return kind == PLCG_OP_STENCIL3D7 ? 1 : kind == PLCG_OP_DIAG ? 2 : kind == PLCG_OP_CSR ? 3 : 0;
}

// Streaming workgroups of a launch: one per chunk up to kMaxStream, a multiple of 8.
int grid_blocks(int nchunks) {
  int b = ((nchunks + kXcds - 1) / kXcds) * kXcds;
  if (b > kMaxStream) b = kMaxStream;
  if (b < kXcds) b = kXcds;
  return b;
}

// Streaming workgroups of a p(l)-CG sweep.  Without cache hints (the working
// set fits the memory-side cache) grid_blocks.  With them, as many as a CU
// keeps resident of the sweep's kernel, at most kSweepPerCu per CU, when that
// is more than four; grid_blocks where the occupancy cannot be read.  A
// multiple of kXcds, at most one per chunk rounded up to kXcds.  Measured per
// sweep against grid_blocks: 256^3 p(1) 240.8 -> 215.0 us, its FP32-stored form
// 122.8 -> 109.2, p(3) -4.7 %; 2048^2 p(4), p(5) -2.9 %, the variable stencil
// -2 to -3 %, CSR -1 %; the diagonal operator 2 % slower, so not for it.
template <typename S>
int sweep_blocks(const SweepArgsT<S> &a, int device, int nchunks) {
  const int base = grid_blocks(nchunks);
  if (a.hint == 0 || a.od.dg != nullptr) return base;
  int per_cu = 0, cus = 0;
  if (plcg_sweep_occupancy(a, &per_cu) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
    return base;
  if (per_cu > kSweepPerCu) per_cu = kSweepPerCu;
  if (per_cu <= 4) return base;
  int b = (per_cu * cus / kXcds) * kXcds;
  if (b > kSweepStream) b = kSweepStream;
  const int cap = ((nchunks + kXcds - 1) / kXcds) * kXcds;
  if (b > cap) b = cap;
  return b > base ? b : base;
}

}  // namespace

int32_t plcg::set_last_error(int32_t code, const char *msg) {
  g_last_error = msg;
  return code;
}

struct plcg_handle {
  plcg_operator_desc op{};
  int method = PLCG_METHOD_PLCG;
  int l = 1;
  int R = 2;                      // ring slots of the basis Z^{(l)}
  double sigma[kLMax] = {0};
  int check_every = kDefaultCheck;
  int max_restarts = kDefaultRestarts;
  int hist_cap = 0;
  int n = 0, nchunks = 0, blocks = 0;
  bool d3 = false;
  int res_kind = -1;              // operator kind of the resident kernels; -1: streaming
  int hint64 = 0, hint32 = 0;     // streaming cache hints of the FP64 / FP32-stored sweeps
  int sweep_nb[2] = {0, 0};       // streaming workgroups of the FP32 / FP64-stored sweeps (0: not chosen yet)
  bool pair64 = false, pair32 = false;   // the same sweeps update x on even t only
  bool ran_resident = false;      // the current solve ran resident launches
  OpData od{nullptr, nullptr, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, nullptr};   // library copies of the operator data
  bool var = false;               // variable-coefficient stencil (edge weights in od.sx/sy/sz)
  bool jacobi = false;            // CSR / variable stencil solved in Jacobi-scaled form D^{-1/2} A D^{-1/2}
  double *dis = nullptr;          // D^{-1/2} (jacobi)
  double *bs = nullptr;           // D^{-1/2} b of the current solve (jacobi)
  int device = 0;
  // device buffers
  std::vector<void *> allocs;
  double *basis[kLMax][2] = {};   // basis k < l, slots by index parity
  double *ring[kLMax] = {};       // basis l, slot of z^{(l)}_j is j % R
  double *p[2] = {nullptr, nullptr};   // p_t in p[t & 1]
  double *cg_r = nullptr, *cg_p[2] = {nullptr, nullptr}, *cg_q = nullptr;
  // FP32_REFINED: FP32 storage of the inner solver and the FP64 outer residual
  int precision = PLCG_PREC_FP64;
  double inner_tol = 1e-3;
  float *basis32[kLMax][2] = {};
  float *ring32[kLMax] = {};
  float *p32[2] = {nullptr, nullptr}, *d32 = nullptr;
  double *r64 = nullptr;
  double *part[2] = {nullptr, nullptr};   // partials of launches with even / odd index
  DevState *st[2] = {nullptr, nullptr};   // scalar state read by odd / even launches
  double *hist = nullptr;
  HostStatus *hs_host = nullptr;  // pinned, mapped (NULL: the record is in device memory)
  HostStatus *hs_dev = nullptr;
  HostStatus hs_copy{};           // host copy of a device-memory record (see wait_stream)
  // timing
  bool timing = false;
  std::vector<hipEvent_t> tev;
  hipEvent_t chunk_ev[2] = {nullptr, nullptr};
  // asynchronous solves
  std::mutex mu;
  std::thread worker;
  std::atomic<bool> busy{false};
  uint64_t next_ticket = 1, cur_ticket = 0;
  plcg_status async_status = PLCG_OK;
  std::string async_error;
  plcg_result async_result{};
  int last_hist_count = 0;
  int host_waits = 0;             // host blocking waits of the current call
};

namespace {

plcg_status dev_alloc(plcg_handle *h, void **ptr, size_t bytes) {
  hipError_t e = hipMalloc(ptr, bytes);
  if (e != hipSuccess) {
    *ptr = nullptr;
    return fail(PLCG_E_NOMEM, std::string("hipMalloc(") + std::to_string(bytes) +
                                  " bytes): " + hipGetErrorString(e));
  }
  h->allocs.push_back(*ptr);
  return PLCG_OK;
}

void release(plcg_handle *h) {
  for (void *p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
  if (h->hs_host) (void)hipHostFree(h->hs_host);
  h->hs_host = nullptr;
  for (hipEvent_t e : h->tev) (void)hipEventDestroy(e);
  h->tev.clear();
  for (auto &e : h->chunk_ev)
    if (e) (void)hipEventDestroy(e);
}

// The device's progress record: mapped pinned host memory written by the
// device (handles from plcg_create), or the host copy that wait_stream takes of
// a record kept in device memory (workspace without host allocations).
volatile HostStatus *hstat(plcg_handle *h) { return h->hs_host ? h->hs_host : &h->hs_copy; }

// Every place where the host blocks on the device goes through here or
// throttle(), so that plcg_result.host_waits counts them.
hipError_t wait_stream(plcg_handle *h, hipStream_t s) {
  ++h->host_waits;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess && h->hs_host == nullptr)
    e = hipMemcpy(&h->hs_copy, h->hs_dev, sizeof(HostStatus), hipMemcpyDeviceToHost);
  return e;
}

// Keep at most two groups of iterations in flight; returns the device status.
// With the record in device memory the host can only read it from an idle
// stream: it waits for every group before enqueueing the next.
plcg_status throttle(plcg_handle *h, hipStream_t s, int group, int *status) {
  if (h->hs_host == nullptr) {
    PLCG_HIP(wait_stream(h, s));
    *status = hstat(h)->status;
    return PLCG_OK;
  }
  PLCG_HIP(hipEventRecord(h->chunk_ev[group & 1], s));
  if (group >= 1) {
    ++h->host_waits;
    PLCG_HIP(hipEventSynchronize(h->chunk_ev[(group - 1) & 1]));
  }
  *status = hstat(h)->status;
  return PLCG_OK;
}

// Timing mode: HIP events around each group of back-to-back iteration
// launches (an event pair around every single launch would add its own gap to
// each).  A group counts only if every launch in it streamed; launches
// enqueued after the stop return at once and would bias the average down.
struct TimedLaunch {
  plcg_handle *h;
  hipStream_t s;
  struct Group {
    size_t ev;      // events ev (start) and ev + 1 (end)
    size_t first;   // index of the group's first launch
    size_t count;   // launches in the group
  };
  std::vector<Group> groups;
  std::vector<uint32_t> counted;  // per launch: iteration launches it stands for (0: no work)
  plcg_status begin_group() {
    if (!h->timing) return PLCG_OK;
    const size_t ev = 2 * groups.size();
    while (h->tev.size() < ev + 2) {
      hipEvent_t e;
      PLCG_HIP(hipEventCreate(&e));
      h->tev.push_back(e);
    }
    PLCG_HIP(hipEventRecord(h->tev[ev], s));
    groups.push_back(Group{ev, counted.size(), 0});
    return PLCG_OK;
  }
  void launched() {
    if (!h->timing) return;
    counted.push_back(1);
    ++groups.back().count;
  }
  // A resident launch stands for `units` iteration launches.
  void set_units(size_t launch, uint32_t units) {
    if (h->timing && launch < counted.size()) counted[launch] = units;
  }
  plcg_status end_group() {
    if (!h->timing) return PLCG_OK;
    PLCG_HIP(hipEventRecord(h->tev[groups.back().ev + 1], s));
    return PLCG_OK;
  }
  size_t launches() const { return counted.size(); }
  // Launches [first + working, launches()) were enqueued after the stop and
  // returned without streaming.
  void keep(size_t first, size_t working) {
    for (size_t k = first + working; k < counted.size(); ++k) counted[k] = 0;
  }
  // Summed duration and launch count of the groups in which every launch
  // streamed; if there is none (a solve shorter than one group), of every
  // group that holds a streaming launch.
  plcg_status total(double *ms, int64_t *count) {
    for (int pass = 0; pass < 2; ++pass) {
      *ms = 0.0;
      *count = 0;
      for (const Group &g : groups) {
        size_t work = 0, streamed = 0;
        for (size_t k = g.first; k < g.first + g.count; ++k) {
          work += counted[k];
          streamed += counted[k] != 0;
        }
        if (work == 0 || (pass == 0 && streamed != g.count)) continue;
        float e = 0.f;
        PLCG_HIP(hipEventElapsedTime(&e, h->tev[g.ev], h->tev[g.ev + 1]));
        *ms += e;
        *count += (int64_t)work;
      }
      if (*count > 0) break;
    }
    return PLCG_OK;
  }
};

// Pointers of iteration i: ring roles, basis roles, start-up copies, and the
// alternating partials / state copies (launch i reads copy (i-1)&1, writes i&1).
template <typename S>
void fill_sweep_args(plcg_handle *h, int i, S *const (*basis)[2], S *const *ring, S *const *p,
                     S *x, SweepArgsT<S> &a) {
  std::memset(&a, 0, sizeof(a));
  const int l = h->l, R = h->R;
  const int t = i - l;
  for (int k = 0; k < R; ++k) {
    const int j = i - k;
    a.zl[k] = j >= 0 ? ring[j % R] : nullptr;
  }
  a.zl_out = ring[(i + 1) % R];
  if (t >= 0) {
    for (int k = 0; k < l; ++k) {
      a.zk_cur[k] = basis[k][(t + k) & 1];
      a.zk_prev[k] = basis[k][(t + k + 1) & 1];
    }
  }
  a.copy_dst = (i < l - 1) ? basis[i + 1][(i + 1) & 1] : nullptr;
  a.v0 = (i == l - 1) ? basis[0][0] : nullptr;
  if (sizeof(S) == 8 ? h->pair64 : h->pair32) {
    // p_t goes to p[t & 1] over p_{t-2}; x is updated on even t only, by both
    // steps since the last even t (an odd last step is made by x_step at the end)
    a.p = p[(t + 1) & 1];
    a.p_out = p[t & 1];
    a.xmode = (t & 1) ? kXSkip : kXPair;
  } else {
    a.p = a.p_out = p[0];
    a.xmode = kXEvery;
  }
  a.x = x;
  a.od = h->od;
  a.part_in = h->part[(i + 1) & 1];
  a.part_out = h->part[i & 1];
  a.st_in = h->st[(i + 1) & 1];
  a.st_out = h->st[i & 1];
  a.hs = h->hs_dev;
  a.hist = h->hist;
  a.i = i;
  a.l = l;
  a.n = h->n;
  a.nx = h->op.nx;
  a.ny = h->op.ny;
  a.nz = h->op.nz;
  a.d3 = h->d3 ? 1 : 0;
  // chunks of kThreads * (16 / sizeof(S)) unknowns: 512 doubles or 1024 floats
  const int chunk = kThreads * (16 / (int)sizeof(S));
  a.nchunks = (h->n + chunk - 1) / chunk;
  a.hint = sizeof(S) == 8 ? h->hint64 : h->hint32;
  // chosen at the first sweep of the handle (the kernel is then known), kept
  // for every later one: a sweep sums the partials of the one before it
  int &nb = h->sweep_nb[sizeof(S) == 8 ? 1 : 0];
  if (nb == 0) nb = sweep_blocks(a, h->device, a.nchunks);
  a.nstream = nb;
  a.nparts_in = i >= 1 ? nb : 0;
  a.pstride = kSweepStream;
  a.work = 1;
}

// r = b - A x (r may be NULL) and ||r||^2 into state copy `slot`; mode as in
// launch_start.
plcg_status residual(plcg_handle *h, const double *b, const double *x, double *r, int slot,
                     int mode, double tol, double rref_in, hipStream_t s,
                     const double *wdiv = nullptr, double abs_floor = 0.0) {
  PLCG_HIP(launch_residual(b, x, r, h->part[0], h->n, h->op.nx, h->op.ny, h->op.nz, h->d3,
                           h->od, wdiv, h->nchunks, h->blocks, s));
  PLCG_HIP(launch_start(h->part[0], h->blocks, h->st[slot], h->hs_dev, mode, tol, rref_in,
                        abs_floor, s));
  return PLCG_OK;
}

struct Segment {
  int status, last_t, t_done, sweeps_run, final_slot;
  double rec;
};

// Sweeps i = 0 .. m + l of one run of Alg. 1 (setup already done; sweep 0 reads
// state copy 1), with lagged status checks; stops early once the device reports
// a stop.  t_done = x-updates made; rec = |zeta_{t_done}|.  p: the two p buffers.
template <typename S>
plcg_status run_segment(plcg_handle *h, S *const (*basis)[2], S *const *ring, S *const *p, S *x,
                        int m, hipStream_t s, TimedLaunch &tl, Segment *out) {
  const int l = h->l;
  const int imax = m + l;               // Alg. 1 loop: i = 0 .. imax
  int status = kRunning;
  int group = 0;
  int last_i = -1;
  const size_t first_launch = tl.launches();
  plcg_status e;
  const bool resident = h->res_kind >= 0 && std::is_same<S, double>::value && m <= kResIterCap;
  if constexpr (std::is_same<S, double>::value) {
    if (resident) {
      // the whole segment in one resident launch: state copy 1 in, copy 0 out
      ResArgs ra;
      std::memset(&ra, 0, sizeof(ra));
      ra.z0 = ring[0];
      ra.x = x;
      ra.od = h->od;
      ra.st_in = h->st[1];
      ra.st_out = h->st[0];
      ra.hs = h->hs_dev;
      ra.hist = h->hist;
      ra.n = h->n;
      ra.nx = h->op.nx;
      ra.ny = h->op.ny;
      ra.nz = h->op.nz;
      ra.imax = imax;
      if ((e = tl.begin_group()) != PLCG_OK) return e;
      PLCG_HIP(launch_plcg_resident(ra, l, h->res_kind, s));
      h->ran_resident = true;
      tl.launched();
      if ((e = tl.end_group()) != PLCG_OK) return e;
      last_i = 0;   // final state in copy 0
    }
  }
  for (int i0 = 0; !resident && i0 <= imax; i0 += h->check_every, ++group) {
    const int i1 = std::min(imax + 1, i0 + h->check_every);
    if ((e = tl.begin_group()) != PLCG_OK) return e;
    for (int i = i0; i < i1; ++i) {
      SweepArgsT<S> a;
      fill_sweep_args<S>(h, i, basis, ring, p, x, a);
      PLCG_HIP(launch_plcg_sweep(a, s));
      tl.launched();
      last_i = i;
    }
    if ((e = tl.end_group()) != PLCG_OK) return e;
    if ((e = throttle(h, s, group, &status)) != PLCG_OK) return e;
    if (status != kRunning) break;
  }
  PLCG_HIP(wait_stream(h, s));
  out->final_slot = last_i & 1;
  DevState ds;
  PLCG_HIP(hipMemcpy(&ds, h->st[out->final_slot], sizeof(ds), hipMemcpyDeviceToHost));
  // The stop can come from a launch near the end of the last group (the owner
  // publishes it at the start of its launch), while x_{last_t} is complete only
  // after sweep last_t + l: enqueue the sweeps up to there that were not
  // enqueued yet.  They run as ordinary sweeps (t <= last_t) and carry the
  // state forward.
  if (!resident && ds.status != kRunning) {
    const int need = std::min(imax, std::max(ds.last_t, -1) + l);
    if (need > last_i) {
      if ((e = tl.begin_group()) != PLCG_OK) return e;
      for (int i = last_i + 1; i <= need; ++i) {
        SweepArgsT<S> a;
        fill_sweep_args<S>(h, i, basis, ring, p, x, a);
        PLCG_HIP(launch_plcg_sweep(a, s));
        tl.launched();
        last_i = i;
      }
      if ((e = tl.end_group()) != PLCG_OK) return e;
      PLCG_HIP(wait_stream(h, s));
      out->final_slot = last_i & 1;
      PLCG_HIP(hipMemcpy(&ds, h->st[out->final_slot], sizeof(ds), hipMemcpyDeviceToHost));
    }
  }
  out->status = ds.status;
  out->last_t = ds.last_t;
  // Iterations that ran: every sweep up to last_t + l (or the whole loop).
  out->t_done = ds.status == kRunning ? m : std::min(std::max(ds.last_t, 0), m);
  out->sweeps_run = std::min(imax, (ds.status == kRunning ? imax : ds.last_t + l)) + 1;
  if (resident)
    tl.set_units(first_launch, (uint32_t)out->sweeps_run);
  else
    tl.keep(first_launch, (size_t)out->sweeps_run);
  out->rec = out->t_done == 0 ? ds.beta : std::fabs(ds.zeta[out->t_done % kTRing]);
  // The streaming sweeps left x at x_{t_done-1} if t_done is odd: add the last
  // step zeta_{t_done-1} p_{t_done-1} (p_{t_done-1} is intact in its buffer).
  if (!resident && (sizeof(S) == 8 ? h->pair64 : h->pair32) && (out->t_done & 1)) {
    const int tl1 = out->t_done - 1;
    PLCG_HIP(launch_x_step<S>(x, p[tl1 & 1], ds.zeta[tl1 % kTRing], h->n, s));
  }
  // t = 0 .. cols-1 were recorded unless the last column broke down.
  h->last_hist_count =
      std::min(h->hist_cap, std::max(ds.cols - (ds.status == kBroken ? 1 : 0), 0));
  return PLCG_OK;
}

// FP32_REFINED: FP64 iterative refinement around an FP32-stored p(l)-CG.
plcg_status solve_mixed(plcg_handle *h, const double *b, double *x, double tol, int maxit,
                        hipStream_t s, plcg_result *res, TimedLaunch &tl, int *final_slot) {
  int total = 0, outer = 0, restarts = 0;
  int64_t spmvs = 0;
  double rref = -1.0, rn = 0.0;
  int reason = PLCG_REASON_MAXIT;
  const int max_outer = 1000;
  plcg_status e;
  *final_slot = 1;
  while (true) {
    // r = b - A x in FP64; the inner solve starts from z_0 = r / ||r|| (FP32) and
    // stops at max(inner_tol ||r||, tol ||r_0|| / 2): the last correction need
    // not be more accurate than the outer goal.
    const double floor_abs = rref > 0 ? 0.5 * tol * rref : 0.0;
    if ((e = residual(h, b, x, h->r64, 1, 0, h->inner_tol, -1.0, s, nullptr, floor_abs)) !=
        PLCG_OK)
      return e;
    PLCG_HIP(launch_scale(h->r64, h->ring32[0], h->basis32[0][0], (float *)nullptr, h->st[1], h->n,
                          s));
    PLCG_HIP(hipMemsetAsync(h->d32, 0, sizeof(float) * (size_t)h->n, s));
    PLCG_HIP(wait_stream(h, s));
    spmvs += 1;
    *final_slot = 1;
    rn = std::sqrt(hstat(h)->sumsq);
    if (rref < 0) {
      rref = rn;
      res->rnorm0 = rref;
    }
    if (!std::isfinite(rn)) {
      res->reason = PLCG_REASON_NONFINITE;
      return fail(PLCG_E_NONFINITE, "residual is not finite");
    }
    if (rn == 0.0 || rn < tol * rref) {
      reason = PLCG_REASON_CONVERGED;
      break;
    }
    if (total >= maxit || outer >= max_outer) break;
    Segment sg;
    if ((e = run_segment<float>(h, h->basis32, h->ring32, h->p32, h->d32, maxit - total, s, tl,
                                &sg)) != PLCG_OK)
      return e;
    *final_slot = sg.final_slot;
    spmvs += sg.sweeps_run;
    total += sg.t_done;
    if (sg.status == kBroken) ++restarts;
    PLCG_HIP(launch_add_correction(x, h->d32, h->n, s));
    ++outer;
    if (sg.status == kBroken && restarts > h->max_restarts) {
      reason = PLCG_REASON_BREAKDOWN_LIMIT;
      break;
    }
  }
  res->iters = total;
  res->outer = outer;
  res->restarts = restarts;
  res->reason = reason;
  res->spmvs = (int32_t)spmvs;
  res->rec_relres = rref > 0 ? rn / rref : 0.0;
  return PLCG_OK;
}

plcg_status solve_plcg(plcg_handle *h, const double *b, double *x, double tol, int maxit,
                       hipStream_t s, plcg_result *res, TimedLaunch &tl, int *final_slot) {
  int total = 0, restarts = 0;
  int64_t spmvs = 0;
  double rref = -1.0;
  int reason = PLCG_REASON_NONE;
  double rec = 0.0;
  h->last_hist_count = 0;
  *final_slot = 1;
  while (true) {
    // Alg. 1, first line: u_0 = b - A x_0; z^{(k)}_0 = u_0 / ||u_0||; g_00 = 1.
    // Sweep 0 reads state copy 1.
    plcg_status e = residual(h, b, x, h->ring[0], 1, 0, tol, rref, s);
    if (e != PLCG_OK) return e;
    PLCG_HIP(launch_scale(h->ring[0], h->ring[0], h->basis[0][0], nullptr, h->st[1], h->n, s));
    PLCG_HIP(wait_stream(h, s));
    spmvs += 1;
    *final_slot = 1;
    const int st0 = hstat(h)->status;
    if (rref < 0) {
      rref = hstat(h)->rref;
      res->rnorm0 = rref;
    }
    if (st0 == kNonFinite) {
      res->reason = PLCG_REASON_NONFINITE;
      return fail(PLCG_E_NONFINITE, "initial residual is not finite");
    }
    if (st0 == kConverged) {
      reason = PLCG_REASON_CONVERGED;
      rec = hstat(h)->beta;
      break;
    }
    const int m = maxit - total;          // x-updates allowed in this segment
    Segment sg;
    if ((e = run_segment<double>(h, h->basis, h->ring, h->p, x, m, s, tl, &sg)) != PLCG_OK)
      return e;
    *final_slot = sg.final_slot;
    const int status = sg.status;
    const int last_t = sg.last_t;
    const int t_done = sg.t_done;
    spmvs += sg.sweeps_run;
    total += t_done;
    rec = sg.rec;
    if (status == kConverged && last_t <= m) {
      reason = PLCG_REASON_CONVERGED;
      break;
    }
    if (status == kBroken && last_t < m) {
      ++restarts;
      if (restarts > h->max_restarts) {
        reason = PLCG_REASON_BREAKDOWN_LIMIT;
        break;
      }
      if (total >= maxit) {
        reason = PLCG_REASON_MAXIT;
        break;
      }
      continue;
    }
    reason = PLCG_REASON_MAXIT;
    break;
  }
  res->iters = total;
  res->restarts = restarts;
  res->reason = reason;
  res->spmvs = (int32_t)spmvs;
  res->rec_relres = rref > 0 ? rec / rref : 0.0;
  return PLCG_OK;
}

plcg_status solve_cg(plcg_handle *h, const double *b, double *x, double tol, int maxit,
                     hipStream_t s, plcg_result *res, TimedLaunch &tl, int *final_slot) {
  // Sweep A reads state copy 1 and partials 1, writes copy 0 and partials 0;
  // sweep B the other way round.  The segment start writes copy 1.
  plcg_status e = residual(h, b, x, h->cg_r, 1, 1, tol, -1.0, s);
  if (e != PLCG_OK) return e;
  PLCG_HIP(wait_stream(h, s));
  *final_slot = 1;
  const double rref = hstat(h)->rref;
  res->rnorm0 = rref;
  int status = hstat(h)->status;
  if (status == kNonFinite) {
    res->reason = PLCG_REASON_NONFINITE;
    return fail(PLCG_E_NONFINITE, "initial residual is not finite");
  }
  if (status == kConverged) {
    res->iters = 0;
    res->reason = PLCG_REASON_CONVERGED;
    res->rec_relres = rref > 0 ? hstat(h)->beta / rref : 0.0;
    res->spmvs = 1;
    return PLCG_OK;
  }
  CgArgs a;
  std::memset(&a, 0, sizeof(a));
  a.b = b;
  a.x = x;
  a.r = h->cg_r;
  a.q = h->cg_q;
  a.od = h->od;
  a.hs = h->hs_dev;
  a.n = h->n;
  a.nx = h->op.nx;
  a.ny = h->op.ny;
  a.nz = h->op.nz;
  a.d3 = h->d3 ? 1 : 0;
  a.nchunks = h->nchunks;
  a.nstream = h->blocks;
  a.nparts_in = h->blocks;
  a.pstride = kMaxStream;
  a.hint = h->hint64;
  // 3D grids whose planes are whole chunks (and even nx): sweep A marches each
  // chunk-sized tile through zseg planes, about one tile-segment per workgroup.
  a.zseg = 0;
  if (h->op.kind == PLCG_OP_STENCIL3D7 && h->op.nz >= 2 && (h->op.nx & 1) == 0 &&
      ((long long)h->op.nx * h->op.ny) % kChunk == 0) {
    const long long tiles = (long long)h->op.nx * h->op.ny / kChunk;
    a.zseg = (int)std::max(1LL, tiles * h->op.nz / h->blocks);
  }
  auto set_a = [&](int k, int work) {
    a.k = k;
    a.work = work;
    a.p_new = h->cg_p[k & 1];
    a.p_old = h->cg_p[(k + 1) & 1];
    a.part_in = h->part[1];
    a.part_out = h->part[0];
    a.st_in = h->st[1];
    a.st_out = h->st[0];
  };
  // Paired x updates: sweep B of odd k writes x_{k+1} from x_{k-1}, even k none.
  auto set_b = [&](int k) {
    a.k = k;
    a.work = 1;
    a.xmode = !h->pair64 ? kXEvery : (k & 1) ? kXPair : kXSkip;
    a.p_new = h->cg_p[k & 1];
    a.p_old = h->cg_p[(k + 1) & 1];
    a.part_in = h->part[0];
    a.part_out = h->part[1];
    a.st_in = h->st[0];
    a.st_out = h->st[1];
  };
  int group = 0;
  bool stopped = false;
  const size_t first_launch = tl.launches();
  const bool resident = h->res_kind >= 0 && maxit <= kResIterCap;
  if (resident) {
    // all iterations in one resident launch: state copy 1 in, copy 0 out
    ResArgs ra;
    std::memset(&ra, 0, sizeof(ra));
    ra.z0 = h->cg_r;
    ra.x = x;
    ra.od = h->od;
    ra.st_in = h->st[1];
    ra.st_out = h->st[0];
    ra.hs = h->hs_dev;
    ra.n = h->n;
    ra.nx = h->op.nx;
    ra.ny = h->op.ny;
    ra.nz = h->op.nz;
    ra.imax = maxit;
    if ((e = tl.begin_group()) != PLCG_OK) return e;
    PLCG_HIP(launch_cg_resident(ra, h->res_kind, s));
    h->ran_resident = true;
    tl.launched();
    if ((e = tl.end_group()) != PLCG_OK) return e;
  }
  for (int k0 = 0; !resident && k0 < maxit; k0 += h->check_every, ++group) {
    const int k1 = std::min(maxit, k0 + h->check_every);
    if ((e = tl.begin_group()) != PLCG_OK) return e;
    for (int k = k0; k < k1; ++k) {
      set_a(k, 1);
      PLCG_HIP(launch_cg_sweep_a(a, s));
      tl.launched();
      set_b(k);
      PLCG_HIP(launch_cg_sweep_b(a, s));
      tl.launched();
    }
    if ((e = tl.end_group()) != PLCG_OK) return e;
    if ((e = throttle(h, s, group, &status)) != PLCG_OK) return e;
    if (status != kRunning) {
      stopped = true;
      break;
    }
  }
  if (resident) {
    *final_slot = 0;
  } else if (!stopped) {
    // Form rho_maxit and the stopping test of the last iterate (no streaming).
    set_a(maxit, 0);
    PLCG_HIP(launch_cg_sweep_a(a, s));
    *final_slot = 0;
  }
  PLCG_HIP(wait_stream(h, s));
  if (stopped) *final_slot = 1;
  DevState ds;
  PLCG_HIP(hipMemcpy(&ds, h->st[*final_slot], sizeof(ds), hipMemcpyDeviceToHost));
  status = ds.status;
  const int iters = status == kRunning ? maxit : ds.last_t;
  // Paired updates left x at x_{iters-1} if iters is odd: add alpha_{iters-1}
  // p_{iters-1} (p_{iters-1} is intact in its buffer, alpha_{iters-1} the last
  // alpha formed).
  if (!resident && h->pair64 && (iters & 1))
    PLCG_HIP(launch_x_step<double>(x, h->cg_p[(iters - 1) & 1], ds.cg_alpha, h->n, s));
  if (resident)
    tl.set_units(first_launch, (uint32_t)(2 * iters));   // stands for sweeps A and B
  else
    tl.keep(first_launch, 2 * (size_t)iters);   // sweeps A and B of iterations 0 .. iters-1
  res->iters = iters;
  res->spmvs = (int32_t)(1 + iters);
  res->rec_relres = rref > 0 ? std::sqrt(ds.cg_rho) / rref : 0.0;
  res->reason = status == kConverged  ? PLCG_REASON_CONVERGED
                : status == kCgBreak ? PLCG_REASON_BREAKDOWN
                                     : PLCG_REASON_MAXIT;
  return PLCG_OK;
}

plcg_status check_vectors(const plcg_handle *h, const double *b, const double *x) {
  if (b == nullptr || x == nullptr) return fail(PLCG_E_INVALID, "NULL vector");
  if ((reinterpret_cast<uintptr_t>(b) & 15) || (reinterpret_cast<uintptr_t>(x) & 15))
    return fail(PLCG_E_INVALID, "vectors must be 16-byte aligned");
  if (b == x) return fail(PLCG_E_INVALID, "b and x must be distinct buffers");
  (void)h;
  return PLCG_OK;
}

plcg_status do_solve(plcg_handle *h, const double *b, double *x, double tol, int32_t maxit,
                     void *stream, plcg_result *out) {
  const auto t0 = std::chrono::steady_clock::now();
  plcg_result res{};
  plcg_status e = check_vectors(h, b, x);
  if (e != PLCG_OK) return e;
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(PLCG_E_INVALID, "tol must be > 0");
  if (maxit < 0) return fail(PLCG_E_INVALID, "maxit must be >= 0");
  PLCG_HIP(hipSetDevice(h->device));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  h->host_waits = 0;
  h->ran_resident = false;
  TimedLaunch tl{h, s};
  int final_slot = 1;
  // Jacobi-scaled CSR: solve D^{-1/2} A D^{-1/2} y = D^{-1/2} b for y = D^{1/2} x
  // (x transformed in place, and back at the end); the original-space residual
  // norm ||b - A x|| = ||(D^{-1/2} b - A~ y) / D^{-1/2}|| is reported beside it.
  const double *bb = b;
  double rnorm0_orig = 0.0;
  if (h->jacobi) {
    PLCG_HIP(launch_jacobi_in(b, h->dis, h->bs, x, h->n, s));
    bb = h->bs;
    if ((e = residual(h, bb, x, nullptr, 1, 2, tol, -1.0, s, h->dis)) != PLCG_OK) return e;
    PLCG_HIP(wait_stream(h, s));
    rnorm0_orig = std::sqrt(hstat(h)->sumsq);
  }
  if (h->method == PLCG_METHOD_CG)
    e = solve_cg(h, bb, x, tol, maxit, s, &res, tl, &final_slot);
  else if (h->precision == PLCG_PREC_FP32_REFINED)
    e = solve_mixed(h, bb, x, tol, maxit, s, &res, tl, &final_slot);
  else
    e = solve_plcg(h, bb, x, tol, maxit, s, &res, tl, &final_slot);
  if (e != PLCG_OK) {
    if (h->jacobi) (void)launch_jacobi_out(x, h->dis, h->n, s);
    if (out) *out = res;
    return e;
  }
  // True residual ||b - A x|| in FP64 (one more operator application).
  if ((e = residual(h, bb, x, nullptr, final_slot, 2, tol, -1.0, s,
                    h->jacobi ? h->dis : nullptr)) != PLCG_OK)
    return e;
  if (h->jacobi) PLCG_HIP(launch_jacobi_out(x, h->dis, h->n, s));
  PLCG_HIP(wait_stream(h, s));
  res.spmvs += h->jacobi ? 2 : 1;
  if (h->jacobi) res.rnorm0 = rnorm0_orig;
  res.true_relres = res.rnorm0 > 0 ? std::sqrt(hstat(h)->sumsq) / res.rnorm0 : 0.0;
  if (h->timing) {
    double ms = 0;
    int64_t count = 0;
    if ((e = tl.total(&ms, &count)) != PLCG_OK) return e;
    res.sweep_ms = ms;
    res.sweeps = count;
  }
  res.host_waits = h->host_waits;
  res.launch_mode = h->ran_resident ? PLCG_LAUNCH_RESIDENT : PLCG_LAUNCH_STREAMING;
  res.x_update_every =
      h->ran_resident || (h->precision == PLCG_PREC_FP32_REFINED ? !h->pair32 : !h->pair64) ? 1 : 2;
  res.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (out) *out = res;
  return PLCG_OK;
}

// Library copy of a CSR operator, checked once on the host: rowptr[0] = 0,
// nondecreasing, rowptr[n] = nnz, every column index in [0, n), every value
// finite.  (Symmetry and definiteness are the caller's promise.)
plcg_status copy_csr(plcg_handle *h, const plcg_operator_desc *op) {
  const size_t n = (size_t)h->n, nnz = (size_t)op->nnz;
  if (nnz >= (size_t)1 << 40) return fail(PLCG_E_INVALID, "nnz too large");
  std::vector<int64_t> rp(n + 1);
  std::vector<int32_t> ci(nnz);
  std::vector<double> va(nnz);
  hipError_t he;
  if ((he = hipMemcpy(rp.data(), op->rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost)) !=
          hipSuccess ||
      (nnz > 0 && (he = hipMemcpy(ci.data(), op->colind, sizeof(int32_t) * nnz,
                                  hipMemcpyDeviceToHost)) != hipSuccess) ||
      (nnz > 0 && (he = hipMemcpy(va.data(), op->vals, sizeof(double) * nnz,
                                  hipMemcpyDeviceToHost)) != hipSuccess))
    return fail(PLCG_E_HIP, std::string("hipMemcpy(CSR): ") + hipGetErrorString(he));
  if (rp[0] != 0 || rp[n] != (int64_t)nnz)
    return fail(PLCG_E_INVALID, "CSR rowptr must start at 0 and end at nnz");
  for (size_t p = 0; p < n; ++p)
    if (rp[p + 1] < rp[p]) return fail(PLCG_E_INVALID, "CSR rowptr must be nondecreasing");
  for (size_t j = 0; j < nnz; ++j) {
    if (ci[j] < 0 || (size_t)ci[j] >= n)
      return fail(PLCG_E_INVALID, "CSR column index out of range");
    if (!std::isfinite(va[j])) return fail(PLCG_E_INVALID, "CSR values must be finite");
  }
  if (h->jacobi) {
    // d_p = a_pp (sum of the stored diagonal entries of row p), which must be
    // positive; a_pq <- a_pq d_p^{-1/2} d_q^{-1/2}.
    std::vector<double> dis(n, 0.0);
    for (size_t p = 0; p < n; ++p)
      for (int64_t j = rp[p]; j < rp[p + 1]; ++j)
        if ((size_t)ci[j] == p) dis[p] += va[j];
    for (size_t p = 0; p < n; ++p) {
      if (!(dis[p] > 0.0) || !std::isfinite(dis[p]))
        return fail(PLCG_E_INVALID, "Jacobi scaling needs a positive diagonal");
      dis[p] = 1.0 / std::sqrt(dis[p]);
    }
    for (size_t p = 0; p < n; ++p)
      for (int64_t j = rp[p]; j < rp[p + 1]; ++j) va[j] *= dis[p] * dis[ci[j]];
    double *ddis = nullptr, *dbs = nullptr;
    plcg_status e = dev_alloc(h, reinterpret_cast<void **>(&ddis), sizeof(double) * n);
    if (e == PLCG_OK) e = dev_alloc(h, reinterpret_cast<void **>(&dbs), sizeof(double) * n);
    if (e != PLCG_OK) return e;
    if ((he = hipMemcpy(ddis, dis.data(), sizeof(double) * n, hipMemcpyHostToDevice)) != hipSuccess)
      return fail(PLCG_E_HIP, std::string("hipMemcpy(D^-1/2): ") + hipGetErrorString(he));
    h->dis = ddis;
    h->bs = dbs;
  }
  // Rows of nearly equal length (stencil-like matrices): keep a padded
  // column-major ELLPACK copy instead, so that consecutive lanes read
  // consecutive rows' j-th entries.  Entry order within a row is the CSR order;
  // padding is the row's own column with value 0.
  int64_t kmax = 0;
  for (size_t p = 0; p < n; ++p) kmax = std::max<int64_t>(kmax, rp[p + 1] - rp[p]);
  const size_t ld = (n + 3) / 4 * 4;
  const bool ell = n > 0 && kmax > 0 && kmax <= 64 && (size_t)kmax * ld <= 2 * nnz + 4 * n;
  if (ell) {
    std::vector<int32_t> eci((size_t)kmax * ld);
    std::vector<double> eva((size_t)kmax * ld, 0.0);
    for (size_t p = 0; p < ld; ++p) {
      const int64_t b0 = p < n ? rp[p] : 0, len = p < n ? rp[p + 1] - rp[p] : 0;
      for (int64_t j = 0; j < kmax; ++j) {
        const size_t e = (size_t)j * ld + p;
        eci[e] = j < len ? ci[b0 + j] : (int32_t)(p < n ? p : 0);
        if (j < len) eva[e] = va[b0 + j];
      }
    }
    ci.swap(eci);
    va.swap(eva);
  }
  const size_t stored = ell ? (size_t)kmax * ld : nnz;
  int64_t *drp = nullptr;
  int32_t *dci = nullptr;
  double *dva = nullptr;
  plcg_status e = dev_alloc(h, reinterpret_cast<void **>(&drp), sizeof(int64_t) * (n + 1));
  if (e == PLCG_OK)
    e = dev_alloc(h, reinterpret_cast<void **>(&dci), sizeof(int32_t) * (stored + 1));
  if (e == PLCG_OK) e = dev_alloc(h, reinterpret_cast<void **>(&dva), sizeof(double) * (stored + 1));
  if (e != PLCG_OK) return e;
  if ((he = hipMemcpy(drp, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (stored > 0 && (he = hipMemcpy(dci, ci.data(), sizeof(int32_t) * stored,
                                     hipMemcpyHostToDevice)) != hipSuccess) ||
      (stored > 0 && (he = hipMemcpy(dva, va.data(), sizeof(double) * stored,
                                     hipMemcpyHostToDevice)) != hipSuccess))
    return fail(PLCG_E_HIP, std::string("hipMemcpy(CSR): ") + hipGetErrorString(he));
  h->od.rp = drp;
  h->od.ci = dci;
  h->od.va = dva;
  h->od.ell_k = ell ? (int32_t)kmax : 0;
  h->od.ell_ld = ell ? (int32_t)ld : 0;
  return PLCG_OK;
}

// Checks the descriptor and the configuration and sets every parameter of a
// solver that needs no device memory (makes no HIP call).  *res_ok: the
// resident kernels could take this system.
plcg_status setup_handle(const plcg_operator_desc *op, const plcg_config *cfg, plcg_handle *h,
                         bool *res_ok) {
  if (op == nullptr || cfg == nullptr) return fail(PLCG_E_INVALID, "NULL descriptor or config");
  if (op->kind != PLCG_OP_STENCIL2D5 && op->kind != PLCG_OP_STENCIL3D7 &&
      op->kind != PLCG_OP_DIAG && op->kind != PLCG_OP_CSR)
    return fail(PLCG_E_INVALID, "unknown operator kind");
  if (op->kind == PLCG_OP_DIAG && op->diag == nullptr)
    return fail(PLCG_E_INVALID, "diagonal operator needs diag");
  if (op->kind == PLCG_OP_CSR &&
      (op->rowptr == nullptr || op->colind == nullptr || op->vals == nullptr || op->nnz < 0))
    return fail(PLCG_E_INVALID, "CSR operator needs rowptr, colind, vals and nnz >= 0");
  const bool stencil = op->kind == PLCG_OP_STENCIL2D5 || op->kind == PLCG_OP_STENCIL3D7;
  const bool var = stencil && op->cx != nullptr;
  if (!stencil && (op->cx != nullptr || op->cy != nullptr || op->cz != nullptr))
    return fail(PLCG_E_INVALID, "edge coefficients are for the stencil operator kinds");
  if (stencil && op->cx == nullptr && (op->cy != nullptr || op->cz != nullptr))
    return fail(PLCG_E_INVALID, "edge coefficients need cx");
  if (var && (op->cy == nullptr || (op->kind == PLCG_OP_STENCIL3D7 && op->cz == nullptr)))
    return fail(PLCG_E_INVALID, "a variable-coefficient stencil needs cx, cy (and cz in 3D)");
  if (op->jacobi != 0 && op->kind != PLCG_OP_CSR && !var)
    return fail(PLCG_E_INVALID,
                "Jacobi scaling is offered for CSR operators and variable-coefficient stencils");
  const int nz = op->kind == PLCG_OP_STENCIL2D5 ? 1 : op->nz;
  if (op->nx < 1 || op->ny < 1 || nz < 1) return fail(PLCG_E_INVALID, "grid extents must be >= 1");
  if (op->kind == PLCG_OP_STENCIL2D5 && op->nz > 1)
    return fail(PLCG_E_INVALID, "2D operator needs nz = 1");
  const long long n = (long long)op->nx * op->ny * nz;
  if (n > kMaxUnknowns) return fail(PLCG_E_INVALID, "too many unknowns (n > 2^31 - 2^23)");
  if (cfg->method != PLCG_METHOD_CG && cfg->method != PLCG_METHOD_PLCG)
    return fail(PLCG_E_INVALID, "unknown method");
  const bool pl = cfg->method == PLCG_METHOD_PLCG;
  if (pl && (cfg->l < 1 || cfg->l > kLMax)) return fail(PLCG_E_INVALID, "l must be in 1..8");
  if (pl && cfg->shifts == nullptr &&
      !(cfg->lambda_max > cfg->lambda_min && std::isfinite(cfg->lambda_min) &&
        std::isfinite(cfg->lambda_max)))
    return fail(PLCG_E_INVALID, "need lambda_min < lambda_max (or explicit shifts)");
  if (cfg->history_cap < 0) return fail(PLCG_E_INVALID, "history_cap must be >= 0");
  if (cfg->precision != PLCG_PREC_FP64 && cfg->precision != PLCG_PREC_FP32_REFINED)
    return fail(PLCG_E_INVALID, "unknown precision");
  if (cfg->precision == PLCG_PREC_FP32_REFINED && !pl)
    return fail(PLCG_E_INVALID, "FP32_REFINED needs method PLCG");
  if (cfg->precision == PLCG_PREC_FP32_REFINED && !(cfg->inner_tol < 1.0))
    return fail(PLCG_E_INVALID, "inner_tol must be < 1");
  if (cfg->launch_mode < PLCG_LAUNCH_AUTO || cfg->launch_mode > PLCG_LAUNCH_RESIDENT)
    return fail(PLCG_E_INVALID, "unknown launch_mode");
  if (cfg->x_update < PLCG_X_AUTO || cfg->x_update > PLCG_X_PAIRED)
    return fail(PLCG_E_INVALID, "unknown x_update");
  *res_ok = cfg->precision == PLCG_PREC_FP64 && !var &&
            plcg_resident_supported(op->kind, n, cfg->method, cfg->l) == 1;
  if (cfg->launch_mode == PLCG_LAUNCH_RESIDENT && !*res_ok)
    return fail(PLCG_E_INVALID,
                "PLCG_LAUNCH_RESIDENT needs FP64, a constant-coefficient operator, "
                "n <= PLCG_RESIDENT_MAX and a supported l");

  h->op = *op;
  h->op.nz = nz;
  h->var = var;
  h->jacobi = (op->kind == PLCG_OP_CSR || var) && op->jacobi != 0;
  h->d3 = op->kind == PLCG_OP_STENCIL3D7;
  h->method = cfg->method;
  h->l = pl ? cfg->l : 1;
  h->R = h->l - 1 > 2 ? h->l - 1 : 2;
  h->check_every = cfg->check_every > 0 ? cfg->check_every : kDefaultCheck;
  h->max_restarts = cfg->max_restarts >= 0 ? cfg->max_restarts : kDefaultRestarts;
  h->hist_cap = cfg->history_cap;
  h->precision = cfg->precision;
  h->inner_tol = cfg->inner_tol > 0.0 ? cfg->inner_tol : 1e-3;
  h->n = (int)n;
  h->nchunks = (int)((n + kChunk - 1) / kChunk);
  h->blocks = grid_blocks(h->nchunks);
  if (pl) {
    // Eq. (chebyshev): sigma_i = (lmax + lmin)/2 + (lmax - lmin)/2 cos((2i+1) pi / (2l)).
    for (int i = 0; i < h->l; ++i) {
      if (cfg->shifts) {
        h->sigma[i] = cfg->shifts[i];
      } else {
        const double mid = 0.5 * (cfg->lambda_max + cfg->lambda_min);
        const double half = 0.5 * (cfg->lambda_max - cfg->lambda_min);
        h->sigma[i] = mid + half * std::cos((2 * i + 1) * M_PI / (2 * h->l));
      }
      if (!std::isfinite(h->sigma[i])) return fail(PLCG_E_INVALID, "shifts must be finite");
    }
  }
  return PLCG_OK;
}

// A solver's workspace is one block of device memory: the work vectors, the
// two sets of partial sums, the two copies of the scalar state, the history
// and, where the library cannot allocate pinned host memory, the progress
// record.  Consecutive vectors are spaced by their size rounded up to 64 KiB
// plus a stagger, so that the many streams of a sweep do not start on the same
// HBM channel when n*8 is a power of two.
struct Workspace {
  size_t vstride, vstride32;      // bytes between FP64 / FP32 vectors
  int nvec, nvec32;
  size_t vec32_at, part_at, st_at, hist_at, hs_at, total;   // offsets (bytes) and size
};
constexpr size_t kPartBytes = sizeof(double) * (kLMax + 1) * kSweepStream;

Workspace workspace_layout(const plcg_handle *h, bool status_record) {
  auto up = [](size_t v, size_t a) { return (v + a - 1) / a * a; };
  Workspace w;
  const size_t stagger = 4096 + 256;
  w.vstride = up((size_t)h->n * sizeof(double), 65536) + stagger;
  w.vstride32 = up((size_t)h->n * sizeof(float), 65536) + stagger;
  const bool pl = h->method == PLCG_METHOD_PLCG;
  const bool mixed = h->precision == PLCG_PREC_FP32_REFINED;
  // FP64 vectors: bases + ring + 2 p (p(l)-CG), r (mixed), r, p, p, q (CG);
  // FP32 (mixed): bases + ring + 2 p + the correction.
  w.nvec = mixed ? 1 : (pl ? 2 * h->l + h->R + 2 : 4);
  w.nvec32 = mixed ? 2 * h->l + h->R + 3 : 0;
  w.vec32_at = w.vstride * w.nvec;
  w.part_at = up(w.vec32_at + w.vstride32 * w.nvec32, 4096);
  w.st_at = w.part_at + 2 * kPartBytes;
  w.hist_at = up(w.st_at + 2 * sizeof(DevState), 256);
  w.hs_at = up(w.hist_at + sizeof(double) * 4 * (size_t)h->hist_cap, 256);
  w.total = w.hs_at + (status_record ? up(sizeof(HostStatus), 256) : 0);
  return w;
}

void carve_workspace(plcg_handle *h, const Workspace &w, char *base, bool status_record) {
  int used = 0, used32 = 0;
  auto vec = [&](double **dst) { *dst = reinterpret_cast<double *>(base + w.vstride * used++); };
  auto vec32 = [&](float **dst) {
    *dst = reinterpret_cast<float *>(base + w.vec32_at + w.vstride32 * used32++);
  };
  if (h->precision == PLCG_PREC_FP32_REFINED) {
    vec(&h->r64);
    for (int k = 0; k < h->l; ++k) {
      vec32(&h->basis32[k][0]);
      vec32(&h->basis32[k][1]);
    }
    for (int k = 0; k < h->R; ++k) vec32(&h->ring32[k]);
    vec32(&h->p32[0]);
    vec32(&h->p32[1]);
    vec32(&h->d32);
  } else if (h->method == PLCG_METHOD_PLCG) {
    for (int k = 0; k < h->l; ++k) {
      vec(&h->basis[k][0]);
      vec(&h->basis[k][1]);
    }
    for (int k = 0; k < h->R; ++k) vec(&h->ring[k]);
    vec(&h->p[0]);
    vec(&h->p[1]);
  } else {
    vec(&h->cg_r);
    vec(&h->cg_p[0]);
    vec(&h->cg_p[1]);
    vec(&h->cg_q);
  }
  for (int k = 0; k < 2; ++k) {
    h->part[k] = reinterpret_cast<double *>(base + w.part_at + k * kPartBytes);
    h->st[k] = reinterpret_cast<DevState *>(base + w.st_at + k * sizeof(DevState));
  }
  h->hist = h->hist_cap > 0 ? reinterpret_cast<double *>(base + w.hist_at) : nullptr;
  if (status_record) h->hs_dev = reinterpret_cast<HostStatus *>(base + w.hs_at);
}

// Bytes of operator data a variable-coefficient SpMV reads: the edge weights
// of every direction, and the diagonal of the unscaled form.
long long var_op_bytes(const plcg_handle *h) {
  const long long nx = h->op.nx, ny = h->op.ny, nz = h->op.nz;
  long long e = (nx + 1) * ny * nz + nx * (ny + 1) * nz + (h->d3 ? nx * ny * (nz + 1) : 0);
  return 8 * (e + (h->jacobi ? 0 : (long long)h->n));
}

// Library copy of a variable-coefficient stencil: the caller's edge coefficients
// (device arrays) checked on the host, turned into the edge weights the kernels
// read (scaled by D^{-1/2} on both sides for a Jacobi solve) and uploaded with
// D^{-1/2} (jacobi) or the diagonal d.
plcg_status copy_var(plcg_handle *h, const plcg_operator_desc *op) {
  const int nx = h->op.nx, ny = h->op.ny, nz = h->op.nz;
  const bool d3 = h->d3;
  const size_t n = (size_t)h->n;
  const size_t nsx = (size_t)(nx + 1) * ny * nz, nsy = (size_t)nx * (ny + 1) * nz;
  const size_t nsz = d3 ? (size_t)nx * ny * (nz + 1) : 0;
  std::vector<double> cx(nsx), cy(nsy), cz(nsz);
  hipError_t he;
  if ((he = hipMemcpy(cx.data(), op->cx, 8 * nsx, hipMemcpyDeviceToHost)) != hipSuccess ||
      (he = hipMemcpy(cy.data(), op->cy, 8 * nsy, hipMemcpyDeviceToHost)) != hipSuccess ||
      (d3 && (he = hipMemcpy(cz.data(), op->cz, 8 * nsz, hipMemcpyDeviceToHost)) != hipSuccess))
    return fail(PLCG_E_HIP, std::string("hipMemcpy(edge coefficients): ") + hipGetErrorString(he));
  std::vector<double> wx(nsx), wy(nsy), wz(nsz), dd(n);
  plcg_status e = edge_weights(nx, ny, nz, d3, cx.data(), cy.data(), d3 ? cz.data() : nullptr,
                               h->jacobi, wx.data(), wy.data(), wz.data(), dd.data());
  if (e != PLCG_OK) return e;
  double *dsx = nullptr, *dsy = nullptr, *dsz = nullptr, *ddd = nullptr;
  e = dev_alloc(h, reinterpret_cast<void **>(&dsx), 8 * nsx);
  if (e == PLCG_OK) e = dev_alloc(h, reinterpret_cast<void **>(&dsy), 8 * nsy);
  if (e == PLCG_OK && d3) e = dev_alloc(h, reinterpret_cast<void **>(&dsz), 8 * nsz);
  if (e == PLCG_OK) e = dev_alloc(h, reinterpret_cast<void **>(&ddd), 8 * n);
  if (e == PLCG_OK && h->jacobi) e = dev_alloc(h, reinterpret_cast<void **>(&h->bs), 8 * n);
  if (e != PLCG_OK) return e;
  if ((he = hipMemcpy(dsx, wx.data(), 8 * nsx, hipMemcpyHostToDevice)) != hipSuccess ||
      (he = hipMemcpy(dsy, wy.data(), 8 * nsy, hipMemcpyHostToDevice)) != hipSuccess ||
      (d3 && (he = hipMemcpy(dsz, wz.data(), 8 * nsz, hipMemcpyHostToDevice)) != hipSuccess) ||
      (he = hipMemcpy(ddd, dd.data(), 8 * n, hipMemcpyHostToDevice)) != hipSuccess)
    return fail(PLCG_E_HIP, std::string("hipMemcpy(edge weights): ") + hipGetErrorString(he));
  h->od.sx = dsx;
  h->od.sy = dsy;
  h->od.sz = dsz;
  if (h->jacobi)
    h->dis = ddd;
  else
    h->od.vd = ddd;
  return PLCG_OK;
}

// Streaming cache hints, x-update cadence and launch mode, once the operator
// data is in place.
plcg_status finish_setup(plcg_handle *h, const plcg_operator_desc *op, const plcg_config *cfg,
                         bool res_ok) {
  const long long n = h->n;
  const bool pl = h->method == PLCG_METHOD_PLCG;
  const long long op_bytes = op->kind == PLCG_OP_CSR  ? 12LL * op->nnz
                             : op->kind == PLCG_OP_DIAG ? 8LL * n
                             : h->var                   ? var_op_bytes(h)
                                                        : 0;
  h->hint64 = pick_hint(n, h->method, h->l, h->R, 8, op_bytes);
  h->hint32 = pick_hint(n, h->method, h->l, h->R, 4, op_bytes);
  const int xu = cfg->x_update;
  // CG pairs with the two p buffers it has anyway, at any size (streaming CG,
  // paired against every iteration: 256^2 even, 1024^2 9 %, 2048^2 8.5 % and
  // 256^3 11 % faster)
  h->pair64 = xu == PLCG_X_PAIRED ||
              (xu == PLCG_X_AUTO && (!pl || pair_x_updates(n, h->l, h->R, 8, op_bytes)));
  h->pair32 = pl && (xu == PLCG_X_PAIRED ||
                     (xu == PLCG_X_AUTO && pair_x_updates(n, h->l, h->R, 4, op_bytes)));
  // The resident kernels index the matrix with 32-bit offsets.
  const long long stored =
      h->od.ell_k > 0 ? (long long)h->od.ell_k * h->od.ell_ld : (long long)op->nnz;
  if (res_ok && cfg->launch_mode != PLCG_LAUNCH_STREAMING) {
    if (op->kind != PLCG_OP_CSR || stored < (1LL << 30))
      h->res_kind = op_kind_index(op->kind);
    else if (cfg->launch_mode == PLCG_LAUNCH_RESIDENT)
      return fail(PLCG_E_INVALID, "PLCG_LAUNCH_RESIDENT: too many stored entries");
  }
  return PLCG_OK;
}

// Both copies of the scalar state start from this (shifts, l, history size).
DevState initial_state(const plcg_handle *h) {
  DevState init;
  std::memset(&init, 0, sizeof(init));
  init.l = h->l;
  init.hist_cap = h->hist_cap;
  for (int k = 0; k < kLMax; ++k) init.sigma[k] = h->sigma[k];
  return init;
}

}  // namespace

extern "C" {

const char *plcg_last_error(void) { return g_last_error.c_str(); }

int32_t plcg_version(void) { return 100; }

int32_t plcg_resident_supported(int32_t kind, int64_t n, int32_t method, int32_t l) {
  if (kind != PLCG_OP_STENCIL2D5 && kind != PLCG_OP_STENCIL3D7 && kind != PLCG_OP_CSR &&
      kind != PLCG_OP_DIAG)
    return 0;
  if (n < 1 || n > PLCG_RESIDENT_MAX) return 0;
  if (method != PLCG_METHOD_CG && method != PLCG_METHOD_PLCG) return 0;
  return resident_width(method == PLCG_METHOD_PLCG ? 1 : 0, l, op_kind_index(kind), (int)n) > 0
             ? 1
             : 0;
}

plcg_status plcg_create(const plcg_operator_desc *op, const plcg_config *cfg, plcg_handle **out) {
  if (out == nullptr) return fail(PLCG_E_INVALID, "out is NULL");
  *out = nullptr;
  plcg_handle *h = new plcg_handle();
  bool res_ok = false;
  plcg_status e = setup_handle(op, cfg, h, &res_ok);
  if (e != PLCG_OK) {
    delete h;
    return e;
  }
  hipError_t he;
  if ((he = hipGetDevice(&h->device)) != hipSuccess) {
    delete h;
    return fail(PLCG_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
  }
  const long long n = h->n;
  const Workspace w = workspace_layout(h, false);
  char *arena = nullptr;
  e = dev_alloc(h, reinterpret_cast<void **>(&arena), w.total);
  if (e == PLCG_OK) carve_workspace(h, w, arena, false);
  if (e == PLCG_OK && op->kind == PLCG_OP_DIAG) {
    // The library keeps its own copy of d; every entry must be finite and > 0
    // (an SPD diagonal), checked once here on the host.
    std::vector<double> d((size_t)n);
    if ((he = hipMemcpy(d.data(), op->diag, sizeof(double) * (size_t)n,
                        hipMemcpyDeviceToHost)) != hipSuccess) {
      e = fail(PLCG_E_HIP, std::string("hipMemcpy(diag): ") + hipGetErrorString(he));
    } else {
      for (double v : d)
        if (!(std::isfinite(v) && v > 0.0)) {
          e = fail(PLCG_E_INVALID, "diagonal entries must be finite and > 0");
          break;
        }
    }
    double *dg = nullptr;
    if (e == PLCG_OK) e = dev_alloc(h, reinterpret_cast<void **>(&dg), sizeof(double) * (size_t)n);
    if (e == PLCG_OK &&
        (he = hipMemcpy(dg, d.data(), sizeof(double) * (size_t)n, hipMemcpyHostToDevice)) !=
            hipSuccess)
      e = fail(PLCG_E_HIP, std::string("hipMemcpy(diag): ") + hipGetErrorString(he));
    h->od.dg = dg;
  }
  if (e == PLCG_OK && op->kind == PLCG_OP_CSR) e = copy_csr(h, op);
  if (e == PLCG_OK && h->var) e = copy_var(h, op);
  if (e == PLCG_OK) e = finish_setup(h, op, cfg, res_ok);
  if (e != PLCG_OK) {
    release(h);
    delete h;
    return e;
  }
  if ((he = hipHostMalloc(reinterpret_cast<void **>(&h->hs_host), sizeof(HostStatus),
                          hipHostMallocMapped | hipHostMallocCoherent)) != hipSuccess) {
    release(h);
    delete h;
    return fail(PLCG_E_NOMEM, std::string("hipHostMalloc: ") + hipGetErrorString(he));
  }
  std::memset(h->hs_host, 0, sizeof(HostStatus));
  void *dptr = nullptr;
  if ((he = hipHostGetDevicePointer(&dptr, h->hs_host, 0)) != hipSuccess) {
    release(h);
    delete h;
    return fail(PLCG_E_HIP, std::string("hipHostGetDevicePointer: ") + hipGetErrorString(he));
  }
  h->hs_dev = reinterpret_cast<HostStatus *>(dptr);
  const DevState init = initial_state(h);
  bool ok = hipMemcpy(h->st[0], &init, sizeof(init), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemcpy(h->st[1], &init, sizeof(init), hipMemcpyHostToDevice) == hipSuccess &&
            hipMemset(h->part[0], 0, 2 * kPartBytes) == hipSuccess &&
            hipEventCreateWithFlags(&h->chunk_ev[0], hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&h->chunk_ev[1], hipEventDisableTiming) == hipSuccess &&
            hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    release(h);
    delete h;
    return fail(PLCG_E_HIP, "initialising device state failed");
  }
  *out = h;
  return PLCG_OK;
}

plcg_status plcg_solve(plcg_handle *h, const double *d_b, double *d_x, double tol, int32_t maxit,
                       void *stream, plcg_result *out) {
  if (h == nullptr) return fail(PLCG_E_INVALID, "NULL handle");
  bool expected = false;
  if (!h->busy.compare_exchange_strong(expected, true))
    return fail(PLCG_E_BUSY, "a solve is already in flight on this handle");
  plcg_status e = do_solve(h, d_b, d_x, tol, maxit, stream, out);
  h->busy = false;
  return e;
}

plcg_status plcg_submit(plcg_handle *h, const double *d_b, double *d_x, double tol,
                        int32_t maxit, void *stream, uint64_t *ticket) {
  if (h == nullptr || ticket == nullptr) return fail(PLCG_E_INVALID, "NULL handle or ticket");
  bool expected = false;
  if (!h->busy.compare_exchange_strong(expected, true))
    return fail(PLCG_E_BUSY, "a solve is already in flight on this handle");
  plcg_status e = check_vectors(h, d_b, d_x);
  if (e != PLCG_OK) {
    h->busy = false;
    return e;
  }
  std::lock_guard<std::mutex> lk(h->mu);
  if (h->worker.joinable()) h->worker.join();
  h->cur_ticket = h->next_ticket++;
  *ticket = h->cur_ticket;
  h->worker = std::thread([h, d_b, d_x, tol, maxit, stream]() {
    plcg_result r{};
    plcg_status st = do_solve(h, d_b, d_x, tol, maxit, stream, &r);
    h->async_result = r;
    h->async_status = st;
    // the worker's error message, handed to the thread that polls
    h->async_error = st != PLCG_OK ? g_last_error : std::string();
    h->busy = false;
  });
  return PLCG_OK;
}

plcg_status plcg_poll(plcg_handle *h, uint64_t ticket, plcg_result *out) {
  if (h == nullptr) return fail(PLCG_E_INVALID, "NULL handle");
  std::lock_guard<std::mutex> lk(h->mu);
  if (ticket == 0 || ticket != h->cur_ticket) return fail(PLCG_E_INVALID, "unknown ticket");
  if (h->busy) return PLCG_NOT_READY;
  if (h->worker.joinable()) h->worker.join();
  if (out) *out = h->async_result;
  if (h->async_status != PLCG_OK)
    return fail(h->async_status, "submitted solve failed: " + h->async_error);
  return PLCG_OK;
}

plcg_status plcg_destroy(plcg_handle *h) {
  if (h == nullptr) return PLCG_OK;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    if (h->worker.joinable()) h->worker.join();
  }
  (void)hipSetDevice(h->device);
  (void)hipDeviceSynchronize();
  release(h);
  delete h;
  return PLCG_OK;
}

plcg_status plcg_apply(plcg_handle *h, const double *d_x, double *d_y, void *stream) {
  if (h == nullptr || d_x == nullptr || d_y == nullptr)
    return fail(PLCG_E_INVALID, "NULL argument");
  if (d_x == d_y) return fail(PLCG_E_INVALID, "x and y must be distinct");
  PLCG_HIP(launch_apply(d_x, d_y, h->n, h->op.nx, h->op.ny, h->op.nz, h->d3, h->od,
                        reinterpret_cast<hipStream_t>(stream)));
  return PLCG_OK;
}

int64_t plcg_size(const plcg_handle *h) { return h ? (int64_t)h->n : -1; }

plcg_status plcg_get_shifts(const plcg_handle *h, double *out) {
  if (h == nullptr || out == nullptr) return fail(PLCG_E_INVALID, "NULL argument");
  for (int k = 0; k < h->l; ++k) out[k] = h->sigma[k];
  return PLCG_OK;
}

plcg_status plcg_get_history(const plcg_handle *h, double *out, int32_t cap, int32_t *count) {
  if (h == nullptr || out == nullptr || count == nullptr)
    return fail(PLCG_E_INVALID, "NULL argument");
  if (h->hist == nullptr) return fail(PLCG_E_INVALID, "history not enabled (history_cap = 0)");
  const int c = std::min(cap, h->last_hist_count);
  if (c > 0) PLCG_HIP(hipMemcpy(out, h->hist, sizeof(double) * 4 * c, hipMemcpyDeviceToHost));
  *count = c;
  return PLCG_OK;
}

plcg_status plcg_set_timing(plcg_handle *h, int32_t enable) {
  if (h == nullptr) return fail(PLCG_E_INVALID, "NULL handle");
  h->timing = enable != 0;
  return PLCG_OK;
}

plcg_status plcg_copy(const double *d_src, double *d_dst, int64_t n, void *stream) {
  if (d_src == nullptr || d_dst == nullptr || n < 0) return fail(PLCG_E_INVALID, "bad argument");
  if ((reinterpret_cast<uintptr_t>(d_src) & 15) || (reinterpret_cast<uintptr_t>(d_dst) & 15))
    return fail(PLCG_E_INVALID, "buffers must be 16-byte aligned");
  if (n == 0) return PLCG_OK;
  PLCG_HIP(launch_copy(d_src, d_dst, n, reinterpret_cast<hipStream_t>(stream)));
  return PLCG_OK;
}

}  // extern "C"

// A whole solve in a workspace the caller provides (device memory of ws_bytes
// at ws): no device or pinned host memory is allocated.  The progress record
// lives in the workspace, so the host reads it from an idle stream after each
// group of launches; no history, no timing.  Constant-coefficient stencils
// only: the other operators keep library copies of their data.
namespace {

// Arguments of a workspace solve: the checks of plcg_create plus its own limits
// (no HIP call).  On success the handle holds every parameter and *w its layout.
plcg_status check_workspace_solve(const plcg_operator_desc *op, const plcg_config *cfg,
                                  size_t ws_bytes, plcg_handle *h, bool *res_ok, Workspace *w) {
  if (op == nullptr || cfg == nullptr) return fail(PLCG_E_INVALID, "NULL descriptor or config");
  if ((op->kind != PLCG_OP_STENCIL2D5 && op->kind != PLCG_OP_STENCIL3D7) || op->cx != nullptr ||
      op->cy != nullptr || op->cz != nullptr || op->jacobi != 0)
    return fail(PLCG_E_INVALID,
                "the allocation-free solve takes the constant-coefficient 2D and 3D stencils "
                "only");
  if (cfg->history_cap != 0)
    return fail(PLCG_E_INVALID, "the allocation-free solve keeps no history (history_cap = 0)");
  plcg_status e = setup_handle(op, cfg, h, res_ok);
  if (e != PLCG_OK) return e;
  *w = workspace_layout(h, true);
  if (w->total > ws_bytes)
    return fail(PLCG_E_INVALID, "the allocation-free solve needs " + std::to_string(w->total) +
                                    " bytes of workspace for this system and configuration; "
                                    "its static workspace holds " +
                                    std::to_string(ws_bytes) +
                                    " (use plcg_create / plcg_solve for larger systems)");
  return PLCG_OK;
}

}  // namespace

plcg_status plcg::check_workspace_solve(const plcg_operator_desc *op, const plcg_config *cfg,
                                        size_t ws_bytes) {
  plcg_handle h;
  bool res_ok = false;
  Workspace w;
  return ::check_workspace_solve(op, cfg, ws_bytes, &h, &res_ok, &w);
}

plcg_status plcg::solve_in_workspace(const plcg_operator_desc *op, const plcg_config *cfg,
                                     void *ws, size_t ws_bytes, const double *d_b, double *d_x,
                                     double tol, int32_t maxit, void *stream, plcg_result *out) {
  plcg_handle h;
  bool res_ok = false;
  Workspace w;
  plcg_status e = ::check_workspace_solve(op, cfg, ws_bytes, &h, &res_ok, &w);
  if (e != PLCG_OK) return e;
  if (ws == nullptr) return fail(PLCG_E_INVALID, "NULL workspace");
  PLCG_HIP(hipGetDevice(&h.device));
  carve_workspace(&h, w, static_cast<char *>(ws), true);
  if ((e = finish_setup(&h, op, cfg, res_ok)) != PLCG_OK) return e;
  // The workspace holds whatever the previous call left: start both state
  // copies afresh and clear the partial sums and the progress record.
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const DevState init = initial_state(&h);
  PLCG_HIP(hipMemcpyAsync(h.st[0], &init, sizeof(init), hipMemcpyHostToDevice, s));
  PLCG_HIP(hipMemcpyAsync(h.st[1], &init, sizeof(init), hipMemcpyHostToDevice, s));
  PLCG_HIP(hipMemsetAsync(h.part[0], 0, 2 * kPartBytes, s));
  PLCG_HIP(hipMemsetAsync(h.hs_dev, 0, sizeof(HostStatus), s));
  PLCG_HIP(hipStreamSynchronize(s));
  return do_solve(&h, d_b, d_x, tol, maxit, stream, out);
}
